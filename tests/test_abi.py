"""The C-ABI library loads on the CPU and exports every symbol the headers
declare (no compute calls: those need a GPU)."""
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


def declared_symbols():
    names = set()
    for h in (ROOT / "include").glob("*.h"):
        text = h.read_text()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(bmc_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("bmc_price", "bmc_estimate_continuation", "bmc_fit_rule", "bmc_iz_search",
                 "bmc_final_price", "bmc_sample_points"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_0805_1827_amd import bmc
    if not bmc.LIB_PATH.exists():
        pytest.fail("libbmc.so is not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", str(bmc.LIB_PATH)], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_symbols() if n not in exported]
    assert not missing, missing
    assert sorted(bmc.SYMBOLS) == declared_symbols()


def test_library_loads_without_gpu():
    from paper_0805_1827_amd import bmc
    L = bmc.load()
    assert L.bmc_version() == 10000
    assert L.bmc_last_error() == b""


def test_binding_fails_loudly_when_library_missing(tmp_path, monkeypatch):
    from paper_0805_1827_amd import bmc
    monkeypatch.setattr(bmc, "LIB_PATH", tmp_path / "libbmc.so")
    monkeypatch.setattr(bmc, "_lib", None)
    with pytest.raises(ImportError):
        bmc.load()
