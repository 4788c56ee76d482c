"""Whole-method pins of the oracle: special cases that reduce to closed forms,
the CRR Bermudan tree (1-asset put and the geometric reduction of the 5-asset
put), the paper's printed max-call values, the learned exercise rules against
the tree's critical prices, and the classifier against an independent
logistic-regression solver."""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import pins
from conftest import cpu_threads

GOLDEN = Path(__file__).resolve().parent / "golden"
NT = cpu_threads()


def test_single_date_is_european(orc, inputs):
    """N_T = 1: no early exercise, the price is Black-Scholes (5.57353)."""
    spec = inputs.one_asset_put(n_dates=1)
    r = orc.price(spec, orc.CMC, 50, 50, 400000, 1, nthreads=NT)
    ref = pins.bs_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0)
    assert ref == pytest.approx(5.573526, abs=1e-6)
    assert abs(r["price"] - ref) < 3 * r["std_err"]
    assert r["inner_path_steps"] == 0
    assert r["final_path_steps"] == 400000


def test_put_with_zero_rate_is_european(orc, inputs):
    """r = 0: early exercise of a put never pays, so the learned rule must not
    lose value against the European price."""
    spec = inputs.one_asset_put(r=0.0)
    r = orc.price(spec, orc.CMC, 400, 400, 200000, 2, nthreads=NT)
    ref = pins.bs_put(100.0, 100.0, 0.0, 0.0, 0.2, 1.0)
    assert abs(r["price"] - ref) < 3 * r["std_err"] + 0.005 * ref


def test_max_call_without_dividends_is_european(orc, inputs):
    spec = inputs.basket(2, 100.0, 100.0, 0.05, 0.0, 0.2, 0.0, 1.0, 5, inputs.CALL_MAX)
    r = orc.price(spec, orc.CMC, 400, 300, 200000, 3, nthreads=NT)
    ref = pins.max_call_european(spec.S0, 100.0, 0.05, 0.0, 0.2, 1.0)
    assert abs(r["price"] - ref) < 3 * r["std_err"] + 0.005 * ref


@pytest.fixture(scope="module")
def c1_tree():
    """1-asset Bermudan put, 10 dates: CRR 2000 steps."""
    berm, bnd = pins.crr_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0, 2000, n_dates=10, want_boundary=True)
    amer = pins.crr_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0, 2000, american=True)
    euro = pins.bs_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0)
    return {"berm": berm, "amer": amer, "euro": euro, "boundary": bnd}


def test_tree_values_and_ordering(c1_tree):
    assert c1_tree["berm"] == pytest.approx(6.0334, abs=2e-4)
    assert c1_tree["amer"] >= c1_tree["berm"] >= c1_tree["euro"]


@pytest.mark.parametrize("method", ["CMC", "IZ"])
def test_one_asset_put_against_tree(orc, inputs, c1_tree, method):
    spec = inputs.one_asset_put()
    meth = getattr(orc, method)
    N = 500 if method == "CMC" else 32
    r = orc.price(spec, meth, N, 500, 100000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - c1_tree["berm"]) <= 3 * se + 0.01 * c1_tree["berm"]
    assert r["price"] <= c1_tree["berm"] + 3 * se          # low-biased estimator
    assert r["price"] >= c1_tree["euro"] - 3 * se          # never worse than holding to T
    assert r["ci95"] == pytest.approx(1.96 * se)


def test_cmc_boundary_matches_tree_critical_price(orc, inputs, c1_tree):
    """The root of the learned F_m for the 1-asset put is the critical price."""
    spec = inputs.one_asset_put()
    r = orc.price(spec, orc.CMC, 2000, 1000, 1000, 5, nthreads=NT)
    w = r["rules"]
    lnK = math.log(spec.K)
    learned, tree = [], []
    for m in range(1, 10):
        xs = np.linspace(60.0, 99.99, 40000)
        u = np.log(xs) - lnK
        g = (spec.K - xs) / spec.K
        F = w[m, 0] + w[m, 1] * u + w[m, 2] * u * u + w[m, 3] * g + w[m, 4] * g * g
        ex = xs[F > 0]
        assert len(ex) > 0
        learned.append(ex.max())
        tree.append(c1_tree["boundary"][m * 200])
    learned, tree = np.array(learned), np.array(tree)
    assert np.all(np.abs(learned - tree) < 1.2)
    # the rule of date m matches the tree at date m, not at a neighbouring date
    err = np.sum((learned - tree) ** 2)
    assert err < np.sum((learned[1:] - tree[:-1]) ** 2)
    assert err < np.sum((learned[:-1] - tree[1:]) ** 2)


def test_iz_price_rules_match_tree_critical_prices(orc, inputs, c1_tree):
    spec = inputs.one_asset_put()
    r = orc.price(spec, orc.IZ, 16, 4000, 1000, 5, nthreads=NT)
    learned = np.exp(r["rules"][1:10, 0])
    tree = np.array([c1_tree["boundary"][m * 200] for m in range(1, 10)])
    assert np.all(np.abs(learned - tree) < 1.2)
    err = np.sum((learned - tree) ** 2)
    assert err < np.sum((learned[1:] - tree[:-1]) ** 2)
    assert err < np.sum((learned[:-1] - tree[1:]) ** 2)


def test_iz_boundary_is_a_fixed_point_and_matches_tree(orc, inputs, c1_tree):
    """Section 2.1 eq. (1): at the converged point, exercise value equals the
    continuation value (to the search tolerance); and it sits at the tree's
    critical price."""
    spec = inputs.one_asset_put()
    rules = orc.empty_rules(spec, orc.IZ)
    m = 9
    x = orc.points_iz(spec, m, 4)
    res = orc.iz_search(spec, rules, m, x, 20000, seed=1, nthreads=NT)
    assert np.all(res["s"] > 0)
    for j in range(4):
        xs = x.copy()
        xs[0, :] = res["s"][j]
        c = orc.continuation(spec, orc.IZ, rules, m, xs, 20000, 1, nthreads=NT)["cont"][j]
        assert spec.K - res["s"][j] == pytest.approx(c, abs=0.011)
    assert np.mean(res["s"]) == pytest.approx(c1_tree["boundary"][1800], abs=1.0)


def test_iz_geometric_put_boundary_shape(orc, inputs):
    """For the geometric put the exercise region is {prod S_i < G*^d}: the
    regressed log-boundary of asset 1 has slope -1 on each other log-price and
    no curvature, with intercept d ln G* - (d-1) ln K (G* from the tree)."""
    spec = inputs.geometric_put5()
    m = 9
    rules = orc.empty_rules(spec, orc.IZ)
    x = orc.points_iz(spec, m, 128)
    res = orc.iz_search(spec, rules, m, x, 4000, seed=1, nthreads=NT)
    b = orc.fit_iz(spec, x, res["s"])
    q = spec.d - 1
    assert np.allclose(b[1:1 + q], -1.0, atol=0.05)
    assert np.all(np.abs(b[1 + q:]) < 0.3)
    G0, sG, dG = pins.geometric_reduction(spec)
    _, bnd = pins.crr_put(G0, 100.0, 0.05, dG, sG, 1.0, 2000, n_dates=10, want_boundary=True)
    Gstar = bnd[1800]
    assert b[0] == pytest.approx(spec.d * math.log(Gstar) - q * math.log(spec.K), abs=0.02)


def test_geometric_put5_against_reduced_tree(orc, inputs):
    spec = inputs.geometric_put5()
    G0, sG, dG = pins.geometric_reduction(spec)
    assert sG ** 2 == pytest.approx(0.0176, rel=1e-12)
    assert dG == pytest.approx(0.0112, rel=1e-12)
    tree = pins.crr_put(G0, 100.0, 0.05, dG, sG, 1.0, 2000, n_dates=10)
    assert tree == pytest.approx(3.832, abs=1e-3)
    r = orc.price(spec, orc.CMC, 1000, 400, 200000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - tree) <= 3 * se + 0.01 * tree
    assert r["price"] <= tree + 3 * se
    euro = pins.bs_put(G0, 100.0, 0.05, dG, sG, 1.0)
    assert r["price"] >= euro - 3 * se


def test_max_call_d3_against_paper_table4(orc, inputs):
    """Table 4 (Section 3.4): binomial reference 18.69 at S0 = 100."""
    gold = json.loads((GOLDEN / "paper_tables.json").read_text())["table4_cmc"]["rows"]
    row = [r for r in gold if r["S0"] == 100][0]
    spec = inputs.max_call(3, 100.0)
    r = orc.price(spec, orc.CMC, 2000, 300, 200000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - row["binomial"]) <= 3 * se + 0.01 * row["binomial"]
    assert r["price"] <= row["binomial"] + 3 * se
    euro = pins.max_call_european(spec.S0, 100.0, 0.05, 0.1, 0.2, 3.0)
    assert r["price"] > euro + 10 * se          # early exercise is worth something here
    # variance of the same order as the paper's (Table 4 prints 286.679)
    assert 0.7 * row["variance"] < r["variance"] < 1.3 * row["variance"]


def test_table_ci_column_is_1_96_se():
    """Reading of the CI column: 1.96 sqrt(Var / N) with N = 1e6 reproduces
    every CMC row of Table 4."""
    gold = json.loads((GOLDEN / "paper_tables.json").read_text())["table4_cmc"]["rows"]
    for row in gold:
        assert 1.96 * math.sqrt(row["variance"] / 1e6) == pytest.approx(row["ci95"], abs=6e-4)
        assert abs(row["binomial"] - row["price"]) == pytest.approx(row["error"], abs=1e-9)


def _features(spec, x):
    u = np.log(x / spec.K)
    if spec.payoff == 1:
        pay = np.maximum(x.max(axis=0) - spec.K, 0.0)
    elif spec.payoff == 2:
        pay = np.maximum(spec.K - np.exp(np.log(x).mean(axis=0)), 0.0)
    else:
        pay = np.maximum(spec.K - x.mean(axis=0), 0.0)
    g = pay / spec.K
    return np.column_stack([np.ones(x.shape[1]), u.T, (u ** 2).T, g, g * g]), pay


def test_logitboost_is_logistic_maximum_likelihood(orc, inputs):
    """LogitBoost with a linear base learner is Newton's method for the
    logistic log-likelihood: on noisy labels (no clipping active) the folded
    weights equal the maximum-likelihood weights found by BFGS."""
    spec = inputs.geometric_put5()
    rng = np.random.default_rng(12)
    x = 100.0 * np.exp(rng.normal(-0.05, 0.1, size=(5, 3000)))
    Phi, pay = _features(spec, x)
    itm = pay > 0
    true_w = np.zeros(Phi.shape[1])
    true_w[[0, 11]] = [-0.1, 1.0]
    prob = 1.0 / (1.0 + np.exp(-2.0 * Phi @ true_w))
    lab = rng.random(x.shape[1]) < prob
    cont = np.where(lab, pay - 0.5, pay + 0.5)
    w = orc.fit_cmc(spec, x, cont, rounds=12)
    w_ref = pins.logistic_mle(Phi[itm], lab[itm].astype(float))
    F, Fr = Phi[itm] @ w, Phi[itm] @ w_ref
    pi = 1.0 / (1.0 + np.exp(-2.0 * F))
    assert np.all((pi > 0.25) & (pi < 0.75))      # |z| <= 4: clipping inactive
    assert np.max(np.abs(F - Fr)) < 1e-6
    # score equations of the likelihood vanish at the fitted weights
    Z = (Phi[itm] - Phi[itm].mean(axis=0)) / np.where(Phi[itm].std(axis=0) > 0, Phi[itm].std(axis=0), 1)
    Z[:, 0] = 1.0
    assert np.max(np.abs(Z.T @ (lab[itm] - pi))) < 1e-6 * itm.sum()


def test_fit_without_in_the_money_points_never_exercises(orc, inputs):
    spec = inputs.one_asset_put()
    x = np.full((1, 10), 150.0)
    w = orc.fit_cmc(spec, x, np.zeros(10))
    assert np.all(w == 0.0)


def test_same_seed_same_price_bitwise(orc, inputs):
    spec = inputs.geometric_put5(n_dates=4)
    a = orc.price(spec, orc.CMC, 64, 64, 4096, 9, nthreads=1)
    b = orc.price(spec, orc.CMC, 64, 64, 4096, 9, nthreads=NT)
    assert a["price"] == b["price"] and np.array_equal(a["rules"], b["rules"])
    c = orc.price(spec, orc.CMC, 64, 64, 4096, 10, nthreads=NT)
    assert c["price"] != a["price"]


# ---------------------------------------------------------------------------
# I&Z on the max-call: d exercise regions (Section 2.2, Algorithm 1).

def _asym_max_call2(inputs):
    """Two independent assets with unequal spot and volatility, delta = 0.1."""
    return inputs.basket(2, [100.0, 90.0], 100.0, 0.05, 0.1, [0.2, 0.3], 0.0, 3.0, 9, inputs.CALL_MAX)


def test_iz_max_call_fixed_points_per_region(orc, inputs):
    """At the last date before maturity the continuation is the one-period
    European max-call, so every region's boundary point solves
    s = K + C_E(s, others) with C_E by quadrature; the searched coordinate is
    the region's own asset and the fixed point lies above the other asset."""
    from scipy import optimize
    spec = _asym_max_call2(inputs)
    m, J, n = 8, 8, 20000
    tau = spec.T / spec.n_dates
    rules = orc.empty_rules(spec, orc.IZ)
    assert rules.shape[1] == 2 * orc.rule_width(orc.IZ, 2) == 2 * 3
    for a in (0, 1):
        x = orc.points_iz(spec, m, J, region=a)
        assert np.all(x[a] == spec.K)
        assert not np.allclose(x[1 - a], x[1 - a][0])
        res = orc.iz_search(spec, rules, m, x, n, seed=1, nthreads=NT, region=a, max_iter=300)
        assert np.all(res["s"] > x[1 - a])
        for j in range(J):
            xo = x[:, j].copy()

            def g(s):
                xx = xo.copy()
                xx[a] = s
                return spec.K + pins.max_call_european(xx, spec.K, spec.r, spec.delta, spec.sigma, tau) - s

            ref = optimize.brentq(g, max(spec.K, xo[1 - a]) + 1e-9, 10 * spec.K)
            assert res["s"][j] == pytest.approx(ref, rel=0.01), (a, j, xo[1 - a])


def test_iz_max_call2_against_two_asset_tree(orc, inputs):
    """Price against the product binomial tree of the two assets (15.345), and
    each region's regressed boundary against the tree's critical prices where
    the other asset is low (flat part of the boundary): the more volatile
    asset has the higher boundary, so a region mix-up shows."""
    spec = _asym_max_call2(inputs)
    tree, bnd = pins.max_call2_tree(spec.S0, spec.K, spec.r, spec.delta, spec.sigma, spec.T, 360, 9,
                                    want_boundary=True)
    assert tree == pytest.approx(15.345, abs=0.01)
    r = orc.price(spec, orc.IZ, 128, 2000, 200000, 1, nthreads=NT, max_iter=200)
    se = r["std_err"]
    assert abs(r["price"] - tree) <= 3 * se + 0.01 * tree
    euro = pins.max_call_european(spec.S0, spec.K, spec.r, spec.delta, spec.sigma, spec.T)
    assert r["price"] > euro + 10 * se
    W = orc.rule_width(orc.IZ, 2)
    for m in (8, 6, 4):
        flat = {}
        for a in (0, 1):
            others, crit = bnd[m * 40][a]
            x = orc.points_iz(spec, m, 128, region=a)
            lo, hi = np.quantile(x[1 - a], [0.05, 0.3])
            sel = (others > lo) & (others < hi)
            assert sel.sum() >= 3
            v = np.log(others[sel] / spec.K)
            c = r["rules"][m, a * W:(a + 1) * W]
            learned = np.exp(c[0] + c[1] * v + c[2] * v * v)
            assert np.all(np.abs(learned / crit[sel] - 1.0) < 0.05), (m, a)
            flat[a] = float(np.median(learned))
        assert flat[1] > flat[0] + 3.0, (m, flat)


@pytest.mark.parametrize("S0", [90, 100, 110])
def test_iz_max_call_d3_against_paper_table1(orc, inputs, S0):
    """Table 1 (Section 2.4, I&Z, J = 128): binomial references 11.29 /
    18.69 / 27.58; by the symmetry of the three assets the three regions learn
    the same boundary."""
    gold = json.loads((GOLDEN / "paper_tables.json").read_text())["table1_iz"]["rows"]
    row = [g for g in gold if g["S0"] == S0][0]
    spec = inputs.max_call(3, float(S0))
    r = orc.price(spec, orc.IZ, 128, 1500, 200000, 1, nthreads=NT, max_iter=200)
    se = r["std_err"]
    assert abs(r["price"] - row["binomial"]) <= 3 * se + 0.01 * row["binomial"]
    assert abs(r["price"] - row["price"]) <= 3 * se + 0.01 * row["price"]
    euro = pins.max_call_european(spec.S0, 100.0, 0.05, 0.1, 0.2, 3.0)
    assert r["price"] > euro + 10 * se
    W = orc.rule_width(orc.IZ, 3)
    blocks = r["rules"][1:9].reshape(8, 3, W)
    assert np.all(np.abs(blocks[:, :, 0] - blocks[:, :1, 0]) < 0.02)
    assert r["iz_unconverged"] < 0.2 * 3 * 128 * 8


# ---------------------------------------------------------------------------
# Call on the minimum (regions by the smallest asset) and the secant search.

def _asym_min_call2(inputs):
    return inputs.min_call(2, [100.0, 110.0], sigma=[0.2, 0.3])


def test_min_call_single_date_is_european(orc, inputs):
    spec = inputs.min_call(3, [100.0, 105.0, 110.0], sigma=[0.2, 0.25, 0.3], n_dates=1, T=1.0)
    ref = pins.min_call_european(spec.S0, 100.0, 0.05, 0.1, spec.sigma, 1.0)
    r = orc.price(spec, orc.CMC, 50, 50, 400000, 2, nthreads=NT)
    assert abs(r["price"] - ref) < 3 * r["std_err"]
    assert r["inner_path_steps"] == 0


def test_iz_min_call_fixed_points_per_region(orc, inputs):
    """Last date before maturity: each region's point solves
    s = K + C_E(s, other) with the one-period European min-call, and lies
    below the other asset (the region of the smallest asset)."""
    from scipy import optimize
    spec = _asym_min_call2(inputs)
    m, J, n = 8, 8, 20000
    tau = spec.T / spec.n_dates
    rules = orc.empty_rules(spec, orc.IZ)
    assert orc.iz_regions(spec) == 2
    kept = 0
    for a in (0, 1):
        x = orc.points_iz(spec, m, J, region=a)
        res = orc.iz_search(spec, rules, m, x, n, seed=1, nthreads=NT, region=a, max_iter=300)
        for j in range(J):
            xo = x[:, j].copy()

            def g(s):
                xx = xo.copy()
                xx[a] = s
                return spec.K + pins.min_call_european(xx, spec.K, spec.r, spec.delta, spec.sigma, tau) - s

            if res["s"][j] > 0:
                kept += 1
                assert res["s"][j] < xo[1 - a]
                ref = optimize.brentq(g, spec.K, xo[1 - a])
                assert res["s"][j] == pytest.approx(ref, rel=0.01), (a, j, xo[1 - a])
            else:   # dropped: no fixed point below the other asset (within the search tolerance)
                assert g(xo[1 - a] - 0.05) > -0.05 or xo[1 - a] <= spec.K
    assert kept >= 4


@pytest.mark.parametrize("method", ["CMC", "CMC_ADA", "IZ"])
def test_min_call2_against_two_asset_tree(orc, inputs, method):
    """Price of the asymmetric two-asset min-call against the product tree
    (3.770 within its discretisation wobble); for I&Z, each region's boundary
    where the other asset is high against the tree's critical prices (there
    the boundary is the one-asset call boundary of the region's asset: the
    more volatile asset's is higher)."""
    spec = _asym_min_call2(inputs)
    tree, bnd = pins.max_call2_tree(spec.S0, spec.K, spec.r, spec.delta, spec.sigma, spec.T, 720, 9,
                                    want_boundary=True, kind="min")
    assert tree == pytest.approx(3.770, abs=0.01)
    m_ = getattr(orc, method)
    N, n = (128, 2000) if m_ == orc.IZ else (1000, 500)
    r = orc.price(spec, m_, N, n, 200000, 1, nthreads=NT, max_iter=200)
    se = r["std_err"]
    assert abs(r["price"] - tree) <= 3 * se + 0.01 * tree
    euro = pins.min_call_european(spec.S0, spec.K, spec.r, spec.delta, spec.sigma, spec.T)
    assert r["price"] > euro + 10 * se
    if m_ != orc.IZ:
        return
    W = orc.rule_width(orc.IZ, 2)
    for m in (8, 6, 4):
        for a in (0, 1):
            others, crit = bnd[m * 80][a]
            x = orc.points_iz(spec, m, 128, region=a)
            lo, hi = np.quantile(x[1 - a], [0.75, 0.97])
            sel = (others > lo) & (others < hi)
            assert sel.sum() >= 3
            v = np.log(others[sel] / spec.K)

            def boundary(block):
                c = r["rules"][m, block * W:(block + 1) * W]
                return np.exp(c[0] + c[1] * v + c[2] * v * v)

            own = np.abs(boundary(a) / crit[sel] - 1.0)
            swapped = np.abs(boundary(1 - a) / crit[sel] - 1.0)
            assert np.all(own < 0.03), (m, a, own)
            assert swapped.mean() > 2 * own.mean() + 0.005, (m, a, own.mean(), swapped.mean())


@pytest.mark.parametrize("case", ["put1", "maxcall3"])
def test_secant_search_agrees_with_plain_and_saves_iterations(orc, inputs, case):
    """Both searches stop at |G(s) - s| < eps on the same common-random-number
    map, so their points agree to a few eps; the secant needs fewer map
    evaluations in total."""
    spec = inputs.one_asset_put() if case == "put1" else inputs.max_call(3, 90.0)
    m = spec.n_dates - 3
    table = orc.price(spec, orc.IZ, 16, 300, 256, 2, nthreads=NT)["rules"]
    tot_plain = tot_sec = 0
    for region in range(orc.iz_regions(spec)):
        x = orc.points_iz(spec, m, 32, region=region)
        a = orc.iz_search(spec, table, m, x, 3000, 5, nthreads=NT, region=region, max_iter=300)
        b = orc.iz_search(spec, table, m, x, 3000, 5, nthreads=NT, region=region, max_iter=300,
                          mode=orc.SEARCH_SECANT)
        both = (a["s"] > 0) & (b["s"] > 0)
        assert both.sum() >= 0.8 * max((a["s"] > 0).sum(), 1)
        assert np.all(np.abs(a["s"][both] - b["s"][both]) < 0.25), np.max(np.abs(a["s"][both] - b["s"][both]))
        tot_plain += int(a["iters"].sum())
        tot_sec += int(b["iters"].sum())
    assert tot_sec < 0.75 * tot_plain, (tot_sec, tot_plain)


def test_secant_price_matches_tree(orc, inputs, c1_tree):
    spec = inputs.one_asset_put()
    r = orc.price(spec, orc.IZ, 16, 4000, 200000, 5, nthreads=NT, search_mode=orc.SEARCH_SECANT)
    p = orc.price(spec, orc.IZ, 16, 4000, 200000, 5, nthreads=NT)
    assert abs(r["price"] - c1_tree["berm"]) <= 3 * r["std_err"] + 0.01 * c1_tree["berm"]
    assert r["iz_iterations"] < 0.6 * p["iz_iterations"]
