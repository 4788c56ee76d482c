"""The serving loop's host-side policy on the CPU (no device): the first-fit
arena against a brute-force unit model, and the admission pass with fake
requests -- first come first served, the in-flight and device-slot limits,
waiting on memory without overtaking, one learner per rule table, cache hits,
least-recently-used eviction that spares tables in use -- plus the
submission-time refusal (BMC_ENOMEM) of footprints above the arena.  The
policy is the header the server compiles (csrc/admission.hpp); the driver is
tests/admission_policy.cpp, built here with the host compiler."""
import shutil
import subprocess
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent
CSRC = HERE.parent / "paper_0805_1827_amd" / "csrc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("admission") / "admission_policy"
    subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I" + str(CSRC),
                    str(HERE / "admission_policy.cpp"), "-o", str(exe)], check=True)
    return exe


def test_admission_policy(driver):
    out = subprocess.run([str(driver)], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.splitlines()
    for what in ("arena: first fit", "first come, first served", "in-flight limit", "free device slot",
                 "waiting on memory", "one learner per rule table", "cache hits share", "eviction spares",
                 "larger than the arena"):
        assert any(what in line and line.startswith("ok ") for line in lines), what
    assert lines[-1].startswith("all ") and lines[-1].endswith("checks passed")
