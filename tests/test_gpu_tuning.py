"""Launch shapes and the autotuner (bmc_tuning_*, bmc_autotune).

Bars: every shape gives prices within the parity tolerance of the oracle;
a tuned table is used by standalone and batched calls alike, so a price is
bit-identical alone and in a batch under it.
"""
import numpy as np
import pytest

from conftest import cpu_threads

pytestmark = pytest.mark.gpu
NT_CPU = cpu_threads()


@pytest.fixture(scope="module")
def bmc():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_0805_1827_amd import bmc as m
    return m


def test_every_shape_within_parity(bmc, orc, inputs):
    spec = inputs.one_asset_put()
    ref = orc.price(spec, orc.CMC, 500, 500, 50000, 1, nthreads=NT_CPU)
    ctx = bmc.Context(0)
    try:
        prices = []
        for ppt in (1, 2, 4, 16):
            bmc.bmc_tuning_set(ctx, 0, -1, 0, ppt)
            assert bmc.bmc_tuning_get(ctx, 1, bmc.FP64, 500, 500) == ppt
            r = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, N=500, n=500, n_final=50000, seed=1)
            assert abs(r["price"] - ref["price"]) <= 1e-10 * abs(ref["price"]) + 1e-12 * spec.K, ppt
            assert r["inner_path_steps"] == ref["inner_path_steps"]
            prices.append(r["price"])
        bmc.bmc_tuning_set(ctx, 0, -1, 0, 0)    # back to the heuristic
        with pytest.raises(bmc.BmcError):
            bmc.bmc_tuning_set(ctx, 0, -1, 0, 65)
    finally:
        ctx.close()


def test_autotuned_table_shared_by_standalone_and_batch(bmc, inputs):
    ctx = bmc.Context(0)
    try:
        specs = [inputs.random_option(900 + k, d_range=(d, d), dates_range=(6, 6), n_choices=(4096,))
                 for k, d in enumerate((5, 5, 12))]
        tuned = {}
        for s in specs:
            tuned[s.d] = bmc.bmc_autotune(ctx, s, bmc.FP32, 256, 4096)
            assert tuned[s.d] in (1, 2, 4, 8, 16)
            assert bmc.bmc_tuning_get(ctx, s.d, bmc.FP32, 256, 4096) == tuned[s.d]
        opts = [dict(method=bmc.CMC, precision=bmc.FP32, N=256, n=4096, n_final=20000, seed=9 + k)
                for k in range(len(specs))]
        batch = bmc.bmc_price_batch(ctx, specs, opts)
        for s, o, b in zip(specs, opts, batch):
            alone = bmc.bmc_price(ctx, s, **o)
            assert alone["price"] == b["price"] and alone["inner_path_steps"] == b["inner_path_steps"]
    finally:
        ctx.close()
