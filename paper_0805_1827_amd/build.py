"""Builds libbmc.so (HIP, gfx950) in-tree.

Every translation unit under csrc/ is compiled separately (in parallel) and
linked into one shared library next to this file.  Usage:
    python -m paper_0805_1827_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OBJ = PKG / "_build"
LIB = PKG / "libbmc.so"
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 ops: ordinary float code is compiled to scalar VALU ops
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core accumulators in ordinary VGPRs (no AGPR copies around
         # the correlation MFMAs of the continuation kernel)
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I" + str(ROOT / "include"), "-I" + str(CSRC)]


def sources() -> list[Path]:
    return sorted(CSRC.glob("*.hip"))


def _headers_mtime() -> float:
    hdrs = list(CSRC.glob("*.hpp")) + list((ROOT / "include").glob("*.h"))
    return max(h.stat().st_mtime for h in hdrs)


def _compile(src: Path, incremental: bool = False) -> Path:
    obj = OBJ / (src.stem + ".o")
    if incremental and obj.exists() and obj.stat().st_mtime > max(src.stat().st_mtime, _headers_mtime()):
        return obj
    cmd = [HIPCC, *FLAGS, "-c", str(src), "-o", str(obj)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {src.name}\n{res.stdout}\n{res.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> Path:
    OBJ.mkdir(exist_ok=True)
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), len(os.sched_getaffinity(0)), 16))
    # largest instantiations first so that they overlap the rest
    order = sorted(srcs, key=lambda p: (0 if p.stem.startswith("cont_d") and int(p.stem[6:]) > 8 else 1,
                                        -(int(p.stem[6:]) if p.stem.startswith("cont_d") else 0)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), order))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", file=sys.stderr)
    return LIB


def build_calib() -> list[Path]:
    """Builds the VALU-rate and copy probes (roofline calibration) into calib/bin/."""
    out = PKG / "calib" / "bin"
    out.mkdir(parents=True, exist_ok=True)
    exes = []
    for src in sorted((PKG / "calib").glob("*.hip")):
        exe = out / src.stem
        subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", "-I" + str(CSRC), str(src), "-o", str(exe)], check=True,
                       capture_output=True)
        exes.append(exe)
    return exes


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--calib", action="store_true", help="also build the calibration probes")
    ap.add_argument("--incremental", action="store_true",
                    help="skip objects newer than their source and every header")
    args = ap.parse_args()
    build(args.jobs, verbose=True, incremental=args.incremental)
    if args.calib:
        build_calib()
