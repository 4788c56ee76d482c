"""The no-allocation continuation entry point (bmc_estimate_continuation_noalloc)
against bmc_estimate_continuation on the same context: identical outputs on
two calls in a row (the second with fewer points, at another date), in FP64
and FP32, and a clear error beyond the scratch array's size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch


@pytest.fixture(scope="module")
def bmc(torch_mod):
    from paper_0805_1827_amd import bmc as m
    return m


def _rules_with_exercise(bmc, ctx, spec, N, seed):
    """Rules learned by a small FP64 CMC pricing (so that inner paths stop early)."""
    _, rules = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, N=N, n=256, n_final=1024, seed=seed, want_rules=True)
    return rules


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_noalloc_matches_estimate_continuation(torch_mod, bmc, inputs, prec):
    torch = torch_mod
    precision = getattr(bmc, prec)
    spec = inputs.geometric_put5(n_dates=6)
    ctx = bmc.Context(0)
    try:
        rules = _rules_with_exercise(bmc, ctx, spec, 512, 11)
        for date, N, n in ((2, 700, 3000), (4, 133, 1500)):   # second call: fewer points
            print(f"noalloc {prec} date {date} N {N} n {n}", flush=True)
            x = bmc.bmc_sample_points(ctx, spec, bmc.CMC, date, N, 5)
            c_ref, se_ref, st_ref = bmc.bmc_estimate_continuation(ctx, spec, rules, date, x, n, 5, precision)
            c = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
            se = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
            st = torch.full((N,), -1, dtype=torch.int64, device="cuda")
            bmc.bmc_estimate_continuation_noalloc(ctx, spec, rules, date, x, c, se, st, n, 5, precision)
            torch.cuda.synchronize()
            assert np.array_equal(c.cpu().numpy(), c_ref.cpu().numpy())
            assert np.array_equal(se.cpu().numpy(), se_ref.cpu().numpy())
            assert np.array_equal(st.cpu().numpy(), st_ref.cpu().numpy())
            assert (st.cpu().numpy() > 0).all()
        rules.close()
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_the_scratch(torch_mod, bmc, inputs):
    torch = torch_mod
    spec = inputs.one_asset_put(n_dates=4)
    ctx = bmc.Context(0)
    try:
        rules = bmc.bmc_rules_create(ctx, spec, bmc.CMC)
        N = 1 << 20   # 2^20 points x >= 1 chunk x 24 bytes > 16 MiB
        x = torch.full((1, N), 100.0, dtype=torch.float64, device="cuda")
        c = torch.zeros(N, dtype=torch.float64, device="cuda")
        se = torch.zeros(N, dtype=torch.float64, device="cuda")
        with pytest.raises(bmc.BmcError) as ei:
            bmc.bmc_estimate_continuation_noalloc(ctx, spec, rules, 1, x, c, se, None, 4096, 1, bmc.FP64)
        assert ei.value.status == bmc.ENOMEM
        assert "no-allocation" in str(ei.value)
        assert float(c.abs().sum()) == 0.0   # nothing written
        rules.close()
    finally:
        ctx.close()
