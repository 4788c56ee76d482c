"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on identical seeded inputs.

Bars: integer outputs (Philox words, executed path-steps, I&Z iteration
counts) bit-exact; FP64 values |a - b| <= 1e-10 max(|a|, |b|) + 1e-12 K;
FP32 mode within 0.1 of the Monte Carlo standard error of the FP64 oracle.
"""
import numpy as np
import pytest

from conftest import cpu_threads

pytestmark = pytest.mark.gpu
NT_CPU = cpu_threads()
REL = 1e-10


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


@pytest.fixture(scope="module")
def ctx(bmc):
    c = bmc.Context(0)
    yield c
    c.close()


def dev(torch_mod, a, dtype=None):
    dtype = dtype or torch_mod.float64
    return torch_mod.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def assert_close(a, b, K, rel=REL, what=""):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    tol = rel * np.maximum(np.abs(a), np.abs(b)) + 1e-12 * K
    bad = np.abs(a - b) > tol
    assert not bad.any(), f"{what}: {bad.sum()} mismatches, worst {np.max(np.abs(a - b) / (tol + 1e-300)):.3g}x tol; " \
                          f"first idx {np.argmax(bad)} gpu {a.flat[np.argmax(bad)]!r} oracle {b.flat[np.argmax(bad)]!r}"


# FP32 continuation estimates against the FP64 oracle.  They differ by
# rounding and by the inner paths whose exercise test flips at a near tie
# (one path moves an estimate by its payoff difference / n); over every point
# and date of the 256-option uneven workload the largest distance measured is
# 0.61 standard errors (99th percentile 0.26).  Each point is held to one
# standard error and the points to a tenth of it on average; the whole FP32
# prices, whose labels the FP64 refinement of near ties keeps equal to the
# FP64 ones, are held to a tenth of their standard error.
FP32_POINT_SE = 1.0
FP32_MEAN_SE = 0.1


def assert_fp32_cont(c, ref_cont, ref_se, K, what=""):
    c, ref_cont, ref_se = (np.asarray(v, dtype=float) for v in (c, ref_cont, ref_se))
    dist = np.abs(c - ref_cont)
    assert np.all(dist <= FP32_POINT_SE * ref_se + 1e-9 * K), (what, float(np.max(dist / (ref_se + 1e-300))))
    ok = ref_se > 0
    if ok.any():
        assert float(np.mean(dist[ok] / ref_se[ok])) <= FP32_MEAN_SE, (what, float(np.mean(dist[ok] / ref_se[ok])))


def cmc_scores(spec, table_rows, x):
    """F = w . [1, u, u^2, g, g^2] of each rule row at the points x (columns)."""
    u = np.log(x) - np.log(spec.K)
    if spec.payoff == 1:
        pay = np.maximum(x.max(axis=0) - spec.K, 0.0)
    elif spec.payoff == 2:
        pay = np.maximum(spec.K - np.exp(np.log(x).mean(axis=0)), 0.0)
    else:
        pay = np.maximum(spec.K - x.mean(axis=0), 0.0)
    g = pay / spec.K
    phi = np.column_stack([np.ones(x.shape[1]), u.T, (u ** 2).T, g, g * g])
    return np.atleast_2d(table_rows) @ phi.T


def assert_same_rule(spec, w_gpu, w_ref, x, what=""):
    """The learned exercise rules agree where they are used: the classifier
    values at the points agree (individual weights of nearly collinear
    features are not determined to full precision)."""
    Fg, Fr = cmc_scores(spec, w_gpu, x), cmc_scores(spec, w_ref, x)
    assert np.all(np.abs(Fg - Fr) <= 1e-6 * (1.0 + np.abs(Fr))), f"{what}: max |dF| {np.max(np.abs(Fg - Fr)):.3g}"


def assert_same_labels(orc, spec, x, c_gpu, c_ref, what=""):
    """CMC exercise labels (Phi > 0 and Phi - C > 0) from the GPU and the
    oracle continuation values agree, except where |Phi - C| < 1e-9."""
    phi = np.array([orc.payoff(spec, np.log(x[:, j])) for j in range(x.shape[1])])
    y_gpu, y_ref = phi - c_gpu, phi - c_ref
    lab_gpu, lab_ref = (phi > 0) & (y_gpu > 0), (phi > 0) & (y_ref > 0)
    far = np.abs(y_ref) >= 1e-9
    assert np.array_equal(lab_gpu[far], lab_ref[far]), f"{what}: {np.sum(lab_gpu[far] != lab_ref[far])} labels differ"


def gpu_rules(bmc, ctx, spec, method, table):
    r = bmc.bmc_rules_create(ctx, spec, method)
    bmc.set_rules_table(r, table)
    return r


def cont_parity(bmc, ctx, orc, torch_mod, spec, method, table, m, x, n, seed, ids=None, prec=None):
    rules = gpu_rules(bmc, ctx, spec, method, table)
    c, se, st = bmc.bmc_estimate_continuation(ctx, spec, rules, m, dev(torch_mod, x), n, seed,
                                              bmc.FP64 if prec is None else prec)
    torch_mod.cuda.synchronize()
    ref = orc.continuation(spec, method, table, m, x, n, seed, nthreads=NT_CPU, ids=ids)
    return host(c), host(se), host(st), ref


# --- random numbers -------------------------------------------------------

def test_philox_bit_exact(bmc, ctx, orc, torch_mod):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
               [0xFFFFFFFF] * 4, [9, 499, 123, 0], [3, 7, 11, 13]]
    for k0, k1 in ((1, (2 << 16) | 9), (0xDEADBEEF, 0x12345678)):
        out = host(bmc.bmc_philox(ctx, k0, k1, dev(torch_mod, ctr.view(np.int32), torch_mod.int32)))
        ref = np.stack([orc.philox(k0, k1, c) for c in ctr])
        assert np.array_equal(out.view(np.uint32), ref)


def test_normals_fp64_and_fp32(bmc, ctx, orc, torch_mod):
    rng = np.random.default_rng(6)
    ctr = rng.integers(0, 2 ** 32, size=(8192, 4), dtype=np.uint64).astype(np.uint32)
    dctr = dev(torch_mod, ctr.view(np.int32), torch_mod.int32)
    ref = np.stack([orc.normal_block(77, 99, c) for c in ctr])
    z64 = host(bmc.bmc_normals(ctx, 77, 99, dctr, bmc.FP64))
    assert np.max(np.abs(z64 - ref)) < 1e-13
    z32 = host(bmc.bmc_normals(ctx, 77, 99, dctr, bmc.FP32))
    err = np.abs(z32 - ref)
    assert err.max() < 5e-4 and err.mean() < 2e-6


# --- sample points ----------------------------------------------------------

def test_cmc_points_parity(bmc, ctx, orc, torch_mod, inputs):
    for spec, N in ((inputs.geometric_put5(), 1000), (inputs.one_asset_put(), 333),
                    (inputs.max_call(3, 90.0), 517)):
        for m in sorted({1, spec.n_dates // 2, spec.n_dates - 1, spec.n_dates}):
            x = host(bmc.bmc_sample_points(ctx, spec, bmc.CMC, m, N, 7))
            assert_close(x, orc.points_cmc(spec, m, N, 7), spec.K, rel=1e-12, what=f"points m={m}")


def asym_max_call2(inputs):
    return inputs.basket(2, [100.0, 90.0], 100.0, 0.05, 0.1, [0.2, 0.3], 0.0, 3.0, 9, inputs.CALL_MAX)


def asym_min_call2(inputs):
    return inputs.min_call(2, [100.0, 110.0], sigma=[0.2, 0.3])


def test_iz_lattice_parity(bmc, ctx, orc, torch_mod, inputs):
    for spec, J in ((inputs.geometric_put5(), 256), (inputs.one_asset_put(), 8),
                    (inputs.basket(3, 100.0, 100.0, 0.05, 0.0, 0.25, 0.2, 1.0, 6, inputs.PUT_BASKET), 97),
                    (inputs.basket(3, [90.0, 100.0, 115.0], 100.0, 0.05, 0.1, [0.2, 0.25, 0.3], 0.3, 3.0, 9,
                                   inputs.CALL_MAX), 61),
                    (asym_max_call2(inputs), 20), (asym_min_call2(inputs), 33),
                    (inputs.min_call(3, [95.0, 100.0, 108.0], sigma=[0.2, 0.3, 0.25]), 40)):
        assert bmc.bmc_iz_regions(spec) == orc.iz_regions(spec)
        for region in range(bmc.bmc_iz_regions(spec)):
            for m in (1, spec.n_dates - 1):
                x = host(bmc.bmc_sample_points(ctx, spec, bmc.IZ, m, J, 1, region=region))
                assert_close(x, orc.points_iz(spec, m, J, region=region), spec.K, rel=1e-12,
                             what=f"lattice m={m} region={region}")
    # the context keeps the last (J, q) generator: back to earlier shapes,
    # twice in a row
    for spec, J in ((inputs.geometric_put5(), 256), (inputs.geometric_put5(), 256),
                    (inputs.min_call(3, [95.0, 100.0, 108.0], sigma=[0.2, 0.3, 0.25]), 97)):
        x = host(bmc.bmc_sample_points(ctx, spec, bmc.IZ, 2, J, 1))
        assert_close(x, orc.points_iz(spec, 2, J), spec.K, rel=1e-12, what=f"lattice again J={J}")


# --- continuation estimates -------------------------------------------------

@pytest.fixture(scope="module")
def c1_rules(orc, inputs):
    spec = inputs.one_asset_put()
    return spec, orc.price(spec, orc.CMC, 500, 500, 1000, 1, nthreads=NT_CPU)["rules"]


def test_continuation_c1_every_date(bmc, ctx, orc, torch_mod, c1_rules):
    """1-asset put, N = n = 500 (ragged chunks), every date, oracle's rules."""
    spec, table = c1_rules
    for m in range(1, spec.n_dates):
        x = orc.points_cmc(spec, m, 500, 1)
        c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, m, x, 500, 1)
        assert_close(c, ref["cont"], spec.K, what=f"cont m={m}")
        assert_close(se, ref["se"], spec.K, rel=1e-8, what=f"se m={m}")
        assert np.array_equal(st, ref["steps"]), m
        assert_same_labels(orc, spec, x, c, ref["cont"], what=f"labels m={m}")


def _small_rules(orc, spec, method=0, N=128, n=128):
    return orc.price(spec, method, N, n, 256, 11, nthreads=NT_CPU)["rules"]


@pytest.mark.parametrize("case", ["geo5", "maxcall3", "basket4", "mincall3"])
def test_continuation_multi_asset(bmc, ctx, orc, torch_mod, inputs, case):
    spec = {"geo5": inputs.geometric_put5(), "maxcall3": inputs.max_call(3, 100.0),
            "basket4": inputs.basket(4, [95, 100, 105, 110], 100.0, 0.05, [0.0, 0.01, 0.02, 0.0],
                                     [0.2, 0.25, 0.3, 0.15], 0.4, 1.0, 8, inputs.PUT_BASKET),
            "mincall3": inputs.min_call(3, [100.0, 110.0, 120.0], sigma=[0.2, 0.3, 0.25])}[case]
    table = _small_rules(orc, spec)
    for m, n in ((1, 1000), (spec.n_dates // 2, 4096), (spec.n_dates - 1, 777)):
        x = orc.points_cmc(spec, m, 48, 3)
        c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, m, x, n, 5)
        assert_close(c, ref["cont"], spec.K, what=f"{case} m={m}")
        assert np.array_equal(st, ref["steps"])
        assert_same_labels(orc, spec, x, c, ref["cont"], what=f"{case} labels m={m}")


@pytest.mark.parametrize("d,payoff", [(12, 0), (20, 1), (40, 2), (34, 3), (13, 3)])
def test_continuation_large_d(bmc, ctx, orc, torch_mod, inputs, d, payoff):
    """Dimension buckets (runtime d below the compiled bound, so padded assets
    carry the payoff's neutral log-price), Wishart correlation."""
    rng = np.random.default_rng(d)
    sigma = rng.uniform(0.1, 0.4, size=d)
    rho = inputs.wishart_corr(d, rng)
    T, delta = (3.0, 0.1) if payoff in (1, 3) else (1.0, 0.0)
    S0 = 130.0 if payoff == 3 else 100.0          # the min of 34 assets: start in the money
    spec = inputs.basket(d, S0, 100.0, 0.05, delta, sigma, rho, T, 6, payoff)
    table = _small_rules(orc, spec, N=96, n=64)
    for m in (1, 5):
        x = orc.points_cmc(spec, m, 24, 2)
        c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, m, x, 600, 9)
        assert_close(c, ref["cont"], spec.K, what=f"d={d} m={m}")
        assert np.array_equal(st, ref["steps"])


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_maximum_dimension_and_dates(bmc, ctx, orc, torch_mod, inputs, prec):
    """d = 64 (the largest bound, every asset live) and N_T = 512 exercise
    dates (the largest table): continuation estimates against the oracle;
    FP32 within a tenth of the standard error."""
    rng = np.random.default_rng(64)
    wide = inputs.basket(64, 100.0, 100.0, 0.05, 0.0, rng.uniform(0.1, 0.3, 64), inputs.wishart_corr(64, rng),
                         1.0, 5, inputs.PUT_GEO)
    long = inputs.one_asset_put(n_dates=512)
    p = getattr(bmc, prec)
    for spec, ms, npts, n in ((wide, (1, 3), 20, 500), (long, (1, 256, 511), 16, 300)):
        table = _small_rules(orc, spec, N=64, n=32)
        for m in ms:
            x = orc.points_cmc(spec, m, npts, 4)
            c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, m, x, n, 6, prec=p)
            if p == bmc.FP64:
                assert_close(c, ref["cont"], spec.K, what=f"d={spec.d} dates={spec.n_dates} m={m}")
                assert np.array_equal(st, ref["steps"])
            else:
                assert_fp32_cont(c, ref["cont"], ref["se"], spec.K, what=(spec.d, m))


def test_oversized_rule_table_is_refused(bmc, ctx, torch_mod, inputs):
    """An FP64 I&Z min-call on 16 assets with 100 dates has rule rows of
    16 x 136 coefficients: more than a workgroup's LDS holds."""
    spec = inputs.min_call(16, 100.0, n_dates=100)
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, spec, bmc.IZ, bmc.FP64, N=8, n=8, n_final=8)
    assert e.value.status == bmc.EUNSUPPORTED
    assert "LDS" in bmc.load().bmc_last_error().decode()
    rules = bmc.bmc_rules_create(ctx, inputs.one_asset_put(), bmc.CMC)
    with pytest.raises(bmc.BmcError) as e:        # an empty point set
        bmc.bmc_estimate_continuation(ctx, inputs.one_asset_put(), rules, 3, dev(torch_mod, np.zeros((1, 0))), 8, 1)
    assert e.value.status == bmc.EINVAL


def test_continuation_under_iz_rules(bmc, ctx, orc, torch_mod, inputs):
    spec = inputs.geometric_put5()
    table = orc.price(spec, orc.IZ, 32, 400, 256, 4, nthreads=NT_CPU)["rules"]
    for m in (1, 4, 8):
        x = orc.points_cmc(spec, m, 40, 3)
        c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.IZ, table, m, x, 2000, 6)
        assert_close(c, ref["cont"], spec.K, what=f"iz rules m={m}")
        assert np.array_equal(st, ref["steps"])


def test_continuation_single_point_two_paths(bmc, ctx, orc, torch_mod, c1_rules):
    spec, table = c1_rules
    x = np.array([[97.5]])
    c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, 3, x, 2, 1)
    assert_close(c, ref["cont"], spec.K)
    assert np.array_equal(st, ref["steps"])


def test_continuation_deep_out_of_the_money_is_zero(bmc, ctx, orc, torch_mod, c1_rules):
    spec, table = c1_rules
    x = np.array([[400.0, 1000.0]])
    c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, 8, x, 300, 1)
    assert np.all(c == 0.0) and np.all(ref["cont"] == 0.0)


# --- rule fits -----------------------------------------------------------------

def test_cmc_fit_parity(bmc, ctx, orc, torch_mod, inputs, c1_rules):
    cases = [(c1_rules[0], c1_rules[1], 5, 500), (inputs.geometric_put5(), None, 6, 700),
             (inputs.max_call(3, 110.0), None, 4, 900)]
    for spec, table, m, N in cases:
        if table is None:
            table = _small_rules(orc, spec)
        x = orc.points_cmc(spec, m, N, 1)
        cont = orc.continuation(spec, orc.CMC, table, m, x, 300, 1, nthreads=NT_CPU)["cont"]
        w_ref = orc.fit_cmc(spec, x, cont, rounds=8)
        rules = bmc.bmc_rules_create(ctx, spec, bmc.CMC)
        bmc.bmc_fit_rule(ctx, spec, rules, m, dev(torch_mod, x), dev(torch_mod, cont), rounds=8)
        w = bmc.bmc_rules_get(rules, m)
        assert_same_rule(spec, w, w_ref, x, what=f"fit d={spec.d}")
        assert_same_rule(spec, w, w_ref, orc.points_cmc(spec, m, 2000, 99), what=f"fit d={spec.d} fresh")


@pytest.mark.parametrize("d,N", [(8, 300), (10, 300), (30, 200), (50, 100)])
def test_cmc_fit_parity_wide(bmc, ctx, orc, torch_mod, inputs, d, N):
    """Wide rules: matrix-core normal equations in 16x16 blocks (p = 19..63,
    ragged tiles of 128 and 64 points) and the scalar path (p = 103)."""
    rng = np.random.default_rng(100 + d)
    spec = inputs.basket(d, 100.0, 100.0, 0.05, 0.0, rng.uniform(0.1, 0.4, d), inputs.wishart_corr(d, rng), 1.0,
                         6, inputs.PUT_BASKET)
    m = 3
    x = orc.points_cmc(spec, m, N, 2)
    cont = orc.continuation(spec, orc.CMC, orc.empty_rules(spec, orc.CMC), m, x, 100, 2, nthreads=NT_CPU)["cont"]
    w_ref = orc.fit_cmc(spec, x, cont, rounds=8)
    rules = bmc.bmc_rules_create(ctx, spec, bmc.CMC)
    bmc.bmc_fit_rule(ctx, spec, rules, m, dev(torch_mod, x), dev(torch_mod, cont), rounds=8)
    w = bmc.bmc_rules_get(rules, m)
    assert_same_rule(spec, w, w_ref, x, what=f"fit d={d}")


def test_iz_fit_parity(bmc, ctx, orc, torch_mod, inputs):
    spec = inputs.geometric_put5()
    m = 7
    x = orc.points_iz(spec, m, 200)
    rng = np.random.default_rng(1)
    sstar = 90.0 * np.exp(rng.normal(0, 0.05, 200))
    sstar[::17] = -1.0                     # dropped points
    b_ref = orc.fit_iz(spec, x, sstar)
    xs = x.copy()
    xs[0] = sstar
    rules = bmc.bmc_rules_create(ctx, spec, bmc.IZ)
    bmc.bmc_fit_rule(ctx, spec, rules, m, dev(torch_mod, xs))
    assert np.allclose(bmc.bmc_rules_get(rules, m), b_ref, rtol=1e-9, atol=1e-11)


def test_iz_fit_parity_max_call_regions(bmc, ctx, orc, torch_mod, inputs):
    """Each region's block is fitted from its own row of s* and its own
    features, and lands at its offset in the row; other blocks untouched."""
    spec = inputs.basket(3, [90.0, 100.0, 115.0], 100.0, 0.05, 0.1, [0.2, 0.25, 0.3], 0.3, 3.0, 9,
                         inputs.CALL_MAX)
    m, J = 6, 150
    rules = bmc.bmc_rules_create(ctx, spec, bmc.IZ)
    W = orc.rule_width(orc.IZ, 3)
    assert bmc.bmc_rules_width(rules) == orc.row_width(spec, orc.IZ) == 3 * W
    want = bmc.bmc_rules_get(rules, m)
    rng = np.random.default_rng(4)
    for region in (2, 0, 1):
        x = orc.points_iz(spec, m, J, region=region)
        sstar = (130.0 + 10 * region) * np.exp(rng.normal(0, 0.05, J))
        sstar[region::13] = -1.0
        b_ref = orc.fit_iz(spec, x, sstar, region=region)
        xs = x.copy()
        xs[region] = sstar
        bmc.bmc_fit_rule(ctx, spec, rules, m, dev(torch_mod, xs), region=region)
        want[region * W:(region + 1) * W] = b_ref
        assert np.allclose(bmc.bmc_rules_get(rules, m), want, rtol=1e-9, atol=1e-11), region


def test_iz_fit_without_points_never_exercises(bmc, ctx, orc, torch_mod, inputs):
    spec = inputs.geometric_put5()
    x = orc.points_iz(spec, 3, 16)
    sstar = -np.ones(16)
    xs = x.copy()
    xs[0] = sstar
    rules = bmc.bmc_rules_create(ctx, spec, bmc.IZ)
    bmc.bmc_fit_rule(ctx, spec, rules, 3, dev(torch_mod, xs))
    assert np.array_equal(bmc.bmc_rules_get(rules, 3), orc.fit_iz(spec, x, sstar))


# --- I&Z search -------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["plain", "secant"])
@pytest.mark.parametrize("case", ["put1", "geo5", "maxcall3", "maxcall2", "mincall2"])
def test_iz_search_parity(bmc, ctx, orc, torch_mod, inputs, case, mode):
    """Per region: the searched asset, the region's counter word, the rules
    of later dates (every region's block exercised on the inner paths) and
    the drop of fixed points outside the region; plain and secant steps."""
    spec = {"put1": inputs.one_asset_put(), "geo5": inputs.geometric_put5(),
            "maxcall3": inputs.max_call(3, 100.0), "maxcall2": asym_max_call2(inputs),
            "mincall2": asym_min_call2(inputs)}[case]
    J, n = {"put1": (8, 3000), "geo5": (40, 1500), "maxcall3": (24, 800), "maxcall2": (40, 1000),
            "mincall2": (40, 1000)}[case]
    md = bmc.SEARCH_SECANT if mode == "secant" else bmc.SEARCH_PLAIN
    assert md == (orc.SEARCH_SECANT if mode == "secant" else orc.SEARCH_PLAIN)
    table = orc.empty_rules(spec, orc.IZ)
    if case != "put1":
        table = orc.price(spec, orc.IZ, 16, 300, 256, 2, nthreads=NT_CPU)["rules"]
    dropped = 0
    for m in (spec.n_dates - 1, 3):
        for region in range(orc.iz_regions(spec)):
            x = orc.points_iz(spec, m, J, region=region)
            rules = gpu_rules(bmc, ctx, spec, bmc.IZ, table)
            s, it, steps = bmc.bmc_iz_search(ctx, spec, rules, m, dev(torch_mod, x), n, 2, region=region, mode=md)
            ref = orc.iz_search(spec, table, m, x, n, 2, nthreads=NT_CPU, region=region, mode=md)
            assert np.array_equal(host(it), ref["iters"]), (m, region)
            assert_close(host(s), ref["s"], spec.K, what=f"s* m={m} region={region}")
            assert steps == ref["steps"]
            dropped += int(np.sum(ref["s"] <= 0))
    assert case not in ("maxcall2", "mincall2") or dropped < 2 * 2 * J


@pytest.mark.parametrize("max_iter,eps", [(1, 0.01), (2, 0.01), (3, 0.01), (4, 0.01), (5, 0.01), (8, 1e-4),
                                          (9, 1e-4), (100, 1e-5)])
def test_iz_search_iteration_limits(bmc, ctx, orc, torch_mod, inputs, max_iter, eps):
    """Searches cut off by the iteration limit (points left without a boundary
    point) and long searches with a tight tolerance: identical iteration
    counts, boundary points and step totals, whatever the number of
    iterations enqueued before the host learns that every point has stopped;
    the same context searches again right after."""
    spec = inputs.max_call(3, 100.0)
    table = orc.price(spec, orc.IZ, 16, 300, 256, 2, nthreads=NT_CPU)["rules"]
    rules = gpu_rules(bmc, ctx, spec, bmc.IZ, table)
    for m, region in ((spec.n_dates - 1, 0), (4, 2)):
        x = orc.points_iz(spec, m, 33, region=region)
        s, it, steps = bmc.bmc_iz_search(ctx, spec, rules, m, dev(torch_mod, x), 700, 5, eps=eps,
                                         max_iter=max_iter, region=region)
        ref = orc.iz_search(spec, table, m, x, 700, 5, eps=eps, max_iter=max_iter, nthreads=NT_CPU, region=region)
        assert np.array_equal(host(it), ref["iters"]), (m, region)
        assert_close(host(s), ref["s"], spec.K, what=f"s* m={m} max_iter={max_iter}")
        assert steps == ref["steps"]
        assert int(host(it).max()) <= max_iter


# --- final pricing and the whole pricer ----------------------------------------------

def test_final_price_parity(bmc, ctx, orc, torch_mod, c1_rules):
    spec, table = c1_rules
    rules = gpu_rules(bmc, ctx, spec, bmc.CMC, table)
    r = bmc.bmc_final_price(ctx, spec, rules, 100000, 1)
    ref = orc.final_price(spec, orc.CMC, table, 100000, 1, nthreads=NT_CPU)
    assert_close(r["price"], ref["price"], spec.K)
    assert_close(r["std_err"], ref["std_err"], spec.K, rel=1e-8)
    assert r["final_path_steps"] == ref["final_steps"]


@pytest.mark.parametrize("case", ["c1_cmc", "c1_iz", "geo5_cmc", "geo5_iz", "maxcall3_cmc", "maxcall3_iz",
                                  "maxcall2_iz", "mincall2_cmc", "mincall2_iz", "c1_izsec", "maxcall3_izsec",
                                  "mincall2_izsec"])
def test_price_end_to_end_fp64(bmc, ctx, orc, torch_mod, inputs, case):
    spec = {"c1": inputs.one_asset_put(), "geo5": inputs.geometric_put5(),
            "maxcall3": inputs.max_call(3, 100.0), "maxcall2": asym_max_call2(inputs),
            "mincall2": asym_min_call2(inputs)}[case.split("_")[0]]
    method = bmc.CMC if case.endswith("cmc") else bmc.IZ
    search = bmc.SEARCH_SECANT if case.endswith("izsec") else bmc.SEARCH_PLAIN
    N, n, nf = {"c1_cmc": (500, 500, 100000), "c1_iz": (16, 500, 100000), "geo5_cmc": (512, 512, 100000),
                "geo5_iz": (48, 400, 50000), "maxcall3_cmc": (400, 300, 50000), "maxcall3_iz": (32, 300, 50000),
                "maxcall2_iz": (48, 400, 50000), "mincall2_cmc": (400, 300, 50000),
                "mincall2_iz": (48, 400, 50000), "c1_izsec": (16, 500, 100000),
                "maxcall3_izsec": (32, 300, 50000), "mincall2_izsec": (48, 400, 50000)}[case]
    res, rules = bmc.bmc_price(ctx, spec, method, bmc.FP64, N=N, n=n, n_final=nf, seed=1, want_rules=True,
                               iz_search=search)
    ref = orc.price(spec, method, N, n, nf, 1, nthreads=NT_CPU, search_mode=search)
    assert_close(res["price"], ref["price"], spec.K, what="price")
    table = bmc.rules_table(rules)
    for m in range(1, spec.n_dates):
        if method == bmc.CMC:
            assert_same_rule(spec, table[m], ref["rules"][m], orc.points_cmc(spec, m, 1000, 5), what=f"m={m}")
        else:
            assert np.allclose(table[m], ref["rules"][m], rtol=1e-8, atol=1e-10)
    assert res["inner_path_steps"] == ref["inner_path_steps"]
    assert res["final_path_steps"] == ref["final_path_steps"]
    if method == bmc.IZ:
        assert res["iz_iterations"] == ref["iz_iterations"]
        assert res["iz_unconverged"] == ref["iz_unconverged"]


@pytest.mark.parametrize("prec", ["FP32", "FP32_KAHAN"])
@pytest.mark.parametrize("case", ["c1_cmc", "geo5_cmc", "geo5_iz", "maxcall3_iz"])
def test_price_fp32_within_tenth_of_std_err(bmc, ctx, orc, torch_mod, inputs, case, prec):
    spec = {"c1": inputs.one_asset_put(), "geo5": inputs.geometric_put5(),
            "maxcall3": inputs.max_call(3, 100.0)}[case.split("_")[0]]
    method = bmc.CMC if case.endswith("cmc") else bmc.IZ
    N, n = (500, 500) if method == bmc.CMC else (256, 1000)
    res = bmc.bmc_price(ctx, spec, method, getattr(bmc, prec), N=N, n=n, n_final=200000, seed=1)
    ref = orc.price(spec, method, N, n, 200000, 1, nthreads=NT_CPU)
    assert abs(res["price"] - ref["price"]) <= 0.1 * ref["std_err"], (res["price"], ref["price"], ref["std_err"])


def test_fp32_continuation_near_fp64(bmc, ctx, orc, torch_mod, c1_rules):
    spec, table = c1_rules
    x = orc.points_cmc(spec, 4, 500, 1)
    for prec in (bmc.FP32, bmc.FP32_KAHAN):
        c, se, st, ref = cont_parity(bmc, ctx, orc, torch_mod, spec, bmc.CMC, table, 4, x, 500, 1, prec=prec)
        assert_fp32_cont(c, ref["cont"], ref["se"], spec.K)


# --- full-size workload, sampled ----------------------------------------------------

def test_full_size_geometric_put_sampled(bmc, ctx, orc, torch_mod, inputs):
    """5-asset geometric put at N = n = 4096 (the benchmark's shape): every point
    on the GPU, a sample of points re-evaluated by the oracle."""
    spec = inputs.geometric_put5()
    table = _small_rules(orc, spec, N=256, n=256)
    m = 5
    N, n = 4096, 4096
    x = orc.points_cmc(spec, m, N, 1)
    rules = gpu_rules(bmc, ctx, spec, bmc.CMC, table)
    for prec in (bmc.FP64, bmc.FP32):
        c, se, st = bmc.bmc_estimate_continuation(ctx, spec, rules, m, dev(torch_mod, x), n, 1, prec)
        c, se, st = host(c), host(se), host(st)
        ids = np.array([0, 1, 2, 1023, 2047, 2048, 3000, 4094, 4095])
        ref = orc.continuation(spec, orc.CMC, table, m, x[:, ids], n, 1, nthreads=NT_CPU, ids=ids)
        if prec == bmc.FP64:
            assert_close(c[ids], ref["cont"], spec.K, what="full-size cont")
            assert np.array_equal(st[ids], ref["steps"])
            assert_same_labels(orc, spec, x[:, ids], c[ids], ref["cont"], what="full-size labels")
        else:
            assert_fp32_cont(c[ids], ref["cont"], ref["se"], spec.K)
        assert np.all(c >= 0) and np.all(np.isfinite(se))


def test_full_size_geometric_put_whole_price_fp64(bmc, ctx, orc, inputs):
    """The benchmark's workload priced whole in FP64: 5-asset geometric put,
    CMC with N = n = 4096 at every date and 1e6 final paths, seed 1: price to
    1e-10 with identical inner and final step counts, and every learned rule
    row equal to the oracle's at the fit tolerance."""
    spec = inputs.geometric_put5()
    print("geometric put N = n = 4096, 1e6 final paths: GPU", flush=True)
    res, rules = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, N=4096, n=4096, n_final=1_000_000, seed=1,
                               want_rules=True)
    print("geometric put N = n = 4096, 1e6 final paths: oracle", flush=True)
    ref = orc.price(spec, orc.CMC, 4096, 4096, 1_000_000, 1, nthreads=NT_CPU)
    assert_close(res["price"], ref["price"], spec.K, what="whole FP64 price at N = n = 4096")
    assert res["inner_path_steps"] == ref["inner_path_steps"]
    assert res["final_path_steps"] == ref["final_path_steps"]
    table = bmc.rules_table(rules)
    rng = np.random.default_rng(9)
    xs = 100.0 * np.exp(rng.normal(-0.05, 0.15, size=(spec.d, 500)))
    for m in range(1, spec.n_dates):
        fg, fo = cmc_scores(spec, table[m], xs), cmc_scores(spec, ref["rules"][m], xs)
        assert np.all(np.abs(fg - fo) <= 1e-6 * (1.0 + np.abs(fo))), m
    rules.close()


@pytest.mark.parametrize("N", [65536, 70000])
def test_whole_price_bucket_and_point_order(bmc, ctx, orc, inputs, N):
    """The pricer's date launches start their jobs bucket by bucket (by the
    points' intrinsic values) up to 65536 points and in point order above;
    either way the FP64 price equals the oracle's with identical step counts.
    N = 70000 also runs the one-launch fit with more tiles than blocks."""
    spec = inputs.basket(2, 100.0, 100.0, 0.05, 0.0, 0.2, 0.3, 1.0, 4, inputs.PUT_BASKET)
    print(f"two-asset basket put, N = {N}, n = 64: GPU", flush=True)
    res = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, N=N, n=64, n_final=20000, seed=5)
    print(f"two-asset basket put, N = {N}, n = 64: oracle", flush=True)
    ref = orc.price(spec, orc.CMC, N, 64, 20000, 5, nthreads=NT_CPU)
    assert_close(res["price"], ref["price"], spec.K, what=f"whole FP64 price at N = {N}")
    assert res["inner_path_steps"] == ref["inner_path_steps"]
    assert res["final_path_steps"] == ref["final_path_steps"]


def test_full_size_final_pricing(bmc, ctx, orc, torch_mod, inputs):
    spec = inputs.geometric_put5()
    table = _small_rules(orc, spec, N=256, n=256)
    rules = gpu_rules(bmc, ctx, spec, bmc.CMC, table)
    r = bmc.bmc_final_price(ctx, spec, rules, 1000000, 1)
    ref = orc.final_price(spec, orc.CMC, table, 1000000, 1, nthreads=NT_CPU)
    assert_close(r["price"], ref["price"], spec.K)
    assert r["final_path_steps"] == ref["final_steps"]


@pytest.mark.parametrize("S0", [90.0, 100.0, 110.0])
def test_full_size_max_call5_sampled(bmc, ctx, orc, torch_mod, inputs, S0):
    """Five-asset max-call at N = n = 16384 with 1e6 final paths (one run per
    S0): every point on the GPU in FP64 and in FP32 with compensated sums, a
    sample of points (across several workgroup chunks and the last point)
    re-evaluated by the oracle, then final pricing in both precisions."""
    spec = inputs.max_call(5, S0)
    table = _small_rules(orc, spec, N=256, n=256)
    m, N, n = 4, 16384, 16384
    x = orc.points_cmc(spec, m, N, 1)
    rules = gpu_rules(bmc, ctx, spec, bmc.CMC, table)
    ids = np.array([0, 1, 4095, 4096, 8191, 12000, 16383])
    ref = orc.continuation(spec, orc.CMC, table, m, x[:, ids], n, 1, nthreads=NT_CPU, ids=ids)
    for prec in (bmc.FP64, bmc.FP32_KAHAN):
        c, se, st = bmc.bmc_estimate_continuation(ctx, spec, rules, m, dev(torch_mod, x), n, 1, prec)
        c, se, st = host(c), host(se), host(st)
        if prec == bmc.FP64:
            assert_close(c[ids], ref["cont"], spec.K, what="max-call full-size cont")
            assert np.array_equal(st[ids], ref["steps"])
            assert_same_labels(orc, spec, x[:, ids], c[ids], ref["cont"], what="max-call full-size labels")
        else:
            assert_fp32_cont(c[ids], ref["cont"], ref["se"], spec.K)
        assert np.all(c >= 0) and np.all(np.isfinite(se))
    fin = orc.final_price(spec, orc.CMC, table, 1000000, 1, nthreads=NT_CPU)
    r64 = bmc.bmc_final_price(ctx, spec, rules, 1000000, 1, bmc.FP64)
    assert_close(r64["price"], fin["price"], spec.K)
    assert r64["final_path_steps"] == fin["final_steps"]
    r32 = bmc.bmc_final_price(ctx, spec, rules, 1000000, 1, bmc.FP32_KAHAN)
    assert abs(r32["price"] - fin["price"]) <= 0.1 * fin["std_err"], (r32["price"], fin["price"], fin["std_err"])


# --- determinism, errors, serialisation --------------------------------------------

def test_repeat_is_bit_identical(bmc, ctx, torch_mod, inputs):
    spec = inputs.geometric_put5()
    a = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32, N=256, n=256, n_final=20000, seed=4)
    b = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32, N=256, n=256, n_final=20000, seed=4)
    assert a["price"] == b["price"] and a["inner_path_steps"] == b["inner_path_steps"]


def test_error_statuses(bmc, ctx, torch_mod, inputs):
    spec = inputs.geometric_put5()
    odd = inputs.geometric_put5()
    odd.payoff = 4
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, odd, N=8, n=8, n_final=8)
    assert e.value.status == bmc.EINVAL
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, spec, bmc.IZ, N=8, n=8, n_final=8, iz_search=2)
    assert e.value.status == bmc.EINVAL
    bad = inputs.basket(3, 100.0, 100.0, 0.05, 0.0, 0.2, 0.0, 1.0, 4, inputs.PUT_GEO)
    bad.rho = np.array([[1.0, 0.9, 0.9], [0.9, 1.0, -0.9], [0.9, -0.9, 1.0]])
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, bad, N=8, n=8, n_final=8)
    assert e.value.status == bmc.ENOTSPD
    late = inputs.geometric_put5()
    late.dates = late.dates[::-1].copy()
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, late, N=8, n=8, n_final=8)
    assert e.value.status == bmc.EINVAL
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_price(ctx, spec, N=8, n=8, n_final=8, seed=2 ** 32)
    assert e.value.status == bmc.EINVAL
    mc3 = inputs.max_call(3, 100.0)
    mc_rules = bmc.bmc_rules_create(ctx, mc3, bmc.IZ)
    assert bmc.bmc_rules_width(mc_rules) == 3 * 6
    assert np.all(bmc.bmc_rules_get(mc_rules, 4)[::6] == 1e300)    # every region starts "never"
    x3 = bmc.bmc_sample_points(ctx, mc3, bmc.IZ, 4, 8, 1, region=2)
    for region in (-1, 3):
        with pytest.raises(bmc.BmcError) as e:
            bmc.bmc_sample_points(ctx, mc3, bmc.IZ, 4, 8, 1, region=region)
        assert e.value.status == bmc.EINVAL
        with pytest.raises(bmc.BmcError) as e:
            bmc.bmc_iz_search(ctx, mc3, mc_rules, 4, x3, 100, 1, region=region)
        assert e.value.status == bmc.EINVAL
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_sample_points(ctx, mc3, bmc.CMC, 4, 8, 1, region=1)
    assert e.value.status == bmc.EINVAL
    put3 = inputs.basket(3, 100.0, 100.0, 0.05, 0.0, 0.2, 0.0, 3.0, 9, inputs.PUT_BASKET)
    with pytest.raises(bmc.BmcError) as e:       # one region's rows for a three-region payoff
        bmc.bmc_iz_search(ctx, mc3, bmc.bmc_rules_create(ctx, put3, bmc.IZ), 4, x3, 100, 1)
    assert e.value.status == bmc.EINVAL
    other = bmc.bmc_rules_create(ctx, inputs.one_asset_put(), bmc.CMC)
    with pytest.raises(bmc.BmcError) as e:
        bmc.bmc_final_price(ctx, spec, other, 100, 1)
    assert e.value.status == bmc.EINVAL
    assert "does not match" in bmc.load().bmc_last_error().decode()


def test_rules_export_import_roundtrip(bmc, ctx, torch_mod, inputs):
    spec = inputs.geometric_put5()
    res, rules = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, N=256, n=128, n_final=10000, seed=2,
                               want_rules=True)
    blob = bmc.bmc_rules_export(rules)
    back = bmc.bmc_rules_import(ctx, blob)
    assert np.array_equal(bmc.rules_table(back), bmc.rules_table(rules))
    a = bmc.bmc_final_price(ctx, spec, rules, 10000, 2)
    b = bmc.bmc_final_price(ctx, spec, back, 10000, 2)
    assert a["price"] == b["price"] == res["price"]


def test_phase_times_are_measured(bmc, ctx, inputs):
    """Every phase of repeated prices on one context (pooled timing events)
    has a positive time and the phases fit inside the call's wall time."""
    spec = inputs.geometric_put5()
    for _ in range(4):
        r = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32, N=1024, n=1024, n_final=200000, seed=2)
        assert r["calc_seconds"] > 0 and r["fit_seconds"] > 0 and r["final_seconds"] > 0, r
        assert r["calc_seconds"] + r["fit_seconds"] + r["final_seconds"] <= r["seconds"] * 1.001


# --- randomized whole prices --------------------------------------------------------

# Seeds whose inner-path step count may differ by one: an exercise test at
# rounding level, traced on the oracle alone (its own count moves by one when
# S0 moves by a few ulps).  Every other seed's counts are exact.
TRACED_NEAR_TIES = {2000: 1}


@pytest.mark.parametrize("seed", range(2000, 2024))
def test_random_specs_fp64_price(bmc, ctx, orc, torch_mod, inputs, seed):
    """Seeded random options (d 1-12, 2-12 dates, Wishart correlation, the
    three batch payoffs; every fourth one a min-call on at most 3 assets at
    S0 = 110) priced whole in FP64 by CMC, AdaBoost stumps or I&Z (cycling
    with the seed; I&Z at d <= 6): price to 1e-10 with identical iteration and
    unconverged counts, and identical step counts except at a traced near
    tie: an inner path whose exercise test sits at rounding level (GPU and
    oracle round their log, exp, sin/cos and fused products differently) may
    stop one date apart.  Seed 2000 has one: the oracle's own count moves
    between 733861 and 733862 when S0 moves by 3e-15 relative."""
    spec = inputs.random_option(seed, d_range=(1, 12), dates_range=(2, 12), n_choices=(64, 96, 200))
    if seed % 4 == 0:
        d = min(spec.d, 3)
        spec = inputs.basket(d, 110.0, 100.0, 0.05, 0.1, spec.sigma[:d], inputs.wishart_corr(d, np.random.default_rng(seed)),
                             3.0, spec.n_dates, inputs.CALL_MIN)
    method = (bmc.CMC, bmc.CMC_ADA, bmc.IZ)[seed % 3 if spec.d <= 6 else seed % 2]
    N = 16 if method == bmc.IZ else 64
    n = spec.meta["n"] if getattr(spec, "meta", None) else 96
    res = bmc.bmc_price(ctx, spec, method, bmc.FP64, N=N, n=n, n_final=4096, seed=seed)
    ref = orc.price(spec, method, N, n, 4096, seed, nthreads=NT_CPU)
    assert_close(res["price"], ref["price"], spec.K, what=f"seed {seed} method {method} d {spec.d}")
    allowed = TRACED_NEAR_TIES.get(seed, 0)
    for key in ("inner_path_steps", "final_path_steps"):
        assert abs(res[key] - ref[key]) <= allowed, (key, res[key], ref[key])
    if method == bmc.IZ:
        assert res["iz_iterations"] == ref["iz_iterations"]
        assert res["iz_unconverged"] == ref["iz_unconverged"]
