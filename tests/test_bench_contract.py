"""Host-side pieces of bench.py: the one-GPU refusal and the algorithmic
issue-slot model behind the roofline fraction (no GPU needed)."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402
from paper_0805_1827_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""


def test_slot_model_of_the_headline_step():
    # d = 5 geometric put under a CMC rule: the 5 random words of a path-step
    # are 5/4 Philox blocks (10 rounds of two 32x32->64 multiplies and two
    # three-input xors) and 5/2 Box-Muller pairs; 2d + d(d+1)/2 step FMAs, one
    # exp and d + 3 payoff ops, 3d + 4 rule ops
    c = bench.COST
    philox = 10 * (2 * c["mul64"] + 2 * c["xor3"])
    bm = 4 + 1 + 2 + 4 * c["trans"]
    step = 5 + 15 + 5
    pay = c["trans"] + 8
    rule = 19
    assert bench.slots_per_step_fp32(5, inputs.PUT_GEO, 0) == pytest.approx(1.25 * philox + 2.5 * bm + step + pay + rule)
    assert bench.slots_per_step_fp32(5, inputs.PUT_GEO, 0) == pytest.approx(135.15)
    # as the kernel draws them: whole blocks (2) and pairs (3) per step
    assert bench.slots_per_step_fp32(5, inputs.PUT_GEO, 0, layout=True) == pytest.approx(
        2 * philox + 3 * bm + step + pay + rule)
    # the two counts agree where d fills whole blocks
    for d in (4, 8):
        assert bench.slots_per_step_fp32(d, inputs.PUT_GEO, 0) == pytest.approx(
            bench.slots_per_step_fp32(d, inputs.PUT_GEO, 0, layout=True))


def test_fp64_slot_model_counts_library_calls():
    # FP64 form: same operation list with the FP64 library calls; every class
    # has a positive cost and the count grows with d
    c = bench.COST64
    assert all(v > 0 for v in c.values())
    s5 = bench.slots_per_step_fp64(5, inputs.PUT_GEO, 0)
    assert s5 > bench.slots_per_step_fp32(5, inputs.PUT_GEO, 0) * 0.5
    assert bench.slots_per_step_fp64(6, inputs.PUT_GEO, 0) > s5


def test_slot_model_leaves_matrix_core_correlation_out():
    # from d = 25 the correlation runs on the matrix cores: the VALU count drops
    # by d(d+1)/2 and the flops are reported separately
    v24 = bench.slots_per_step_fp32(24, inputs.PUT_GEO, 0)
    v25 = bench.slots_per_step_fp32(25, inputs.PUT_GEO, 0)
    assert not bench.uses_mfma(24) and bench.uses_mfma(25)
    assert v25 < v24 - 200
    assert bench.mfma_flops_per_step(25) == 650.0
    for d in range(1, 65):
        for pay in (inputs.PUT_BASKET, inputs.PUT_GEO, inputs.CALL_MAX, inputs.CALL_MIN):
            assert bench.slots_per_step_fp32(d, pay, 0) > 0


def test_traffic_record_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """The committed HBM traffic is reported only while the kernel sources hash
    to the profiled version."""
    rec = (ROOT / "profiles" / "k_cont_geo5_fp32_traffic.json").read_text()
    fake = tmp_path / "traffic.json"
    fake.write_text(rec.replace('"src_sha256": "', '"src_sha256": "0'))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", fake)
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", tmp_path / "missing.json")
    assert bench.measured_traffic() is None
