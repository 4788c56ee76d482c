"""Pins of the oracle's model pieces: Cholesky, payoffs, the CMC Brownian-bridge
training points, the lattice points, and the one-interval continuation value
(no exercise rule involved) against closed forms."""
import math

import numpy as np
import pytest
from scipy import stats

import pins
from conftest import cpu_threads


def test_cholesky_matches_numpy(orc, inputs):
    rng = np.random.default_rng(3)
    for d in (1, 2, 5, 13, 40):
        R = inputs.wishart_corr(d, rng)
        L = orc.cholesky(R)
        assert np.allclose(L, np.linalg.cholesky(R), rtol=0, atol=1e-13)
        assert np.allclose(L @ L.T, R, rtol=0, atol=1e-14)


def test_cholesky_rejects_non_spd(orc):
    R = np.array([[1.0, 0.9, 0.9], [0.9, 1.0, -0.9], [0.9, -0.9, 1.0]])
    with pytest.raises(ValueError):
        orc.cholesky(R)


def test_payoffs_by_hand(orc, inputs):
    S = np.array([90.0, 110.0, 100.0])
    mc = inputs.basket(3, 100.0, 100.0, 0.05, 0.1, 0.2, 0.0, 3.0, 9, inputs.CALL_MAX)
    assert orc.payoff(mc, np.log(S)) == pytest.approx(10.0, rel=1e-14)
    bp = inputs.basket(3, 100.0, 105.0, 0.05, 0.0, 0.2, 0.0, 1.0, 9, inputs.PUT_BASKET)
    assert orc.payoff(bp, np.log(S)) == pytest.approx(5.0, rel=1e-13)
    gp = inputs.basket(3, 100.0, 105.0, 0.05, 0.0, 0.2, 0.0, 1.0, 9, inputs.PUT_GEO)
    assert orc.payoff(gp, np.log(S)) == pytest.approx(105.0 - (90 * 110 * 100) ** (1 / 3), rel=1e-13)
    # out of the money is zero, never negative
    assert orc.payoff(mc, np.log(np.array([50.0, 60.0, 70.0]))) == 0.0
    assert orc.payoff(gp, np.log(np.array([150.0, 160.0, 170.0]))) == 0.0


def test_bridge_points_marginal_law(orc, inputs):
    """x_i at t_m is lognormal(ln S0 + (r - delta - sigma^2/2) t_m, sigma^2 t_m);
    assets are correlated by rho."""
    spec = inputs.geometric_put5()
    N = 4000
    for m in (1, 4, 9):
        x = orc.points_cmc(spec, m, N, seed=1)
        t = spec.dates[m - 1]
        for i in range(spec.d):
            mu = math.log(spec.S0[i]) + (spec.r - spec.delta[i] - 0.5 * spec.sigma[i] ** 2) * t
            zs = (np.log(x[i]) - mu) / (spec.sigma[i] * math.sqrt(t))
            assert stats.kstest(zs, "norm").pvalue > 1e-4
        C = np.corrcoef(np.log(x))
        off = C[~np.eye(spec.d, dtype=bool)]
        assert np.all(np.abs(off - 0.3) < 0.06)


def test_bridge_correlation_across_dates(orc, inputs):
    """With independent assets, corr(B_{t_m}, B_{t_{m+1}}) = sqrt(t_m / t_{m+1})."""
    spec = inputs.basket(2, 100.0, 100.0, 0.05, 0.0, 0.2, 0.0, 1.0, 10, inputs.PUT_GEO)
    N = 6000
    for m in (2, 5, 8):
        xa = orc.points_cmc(spec, m, N, seed=4)
        xb = orc.points_cmc(spec, m + 1, N, seed=4)
        ta, tb = spec.dates[m - 1], spec.dates[m]
        for i in range(2):
            rho = np.corrcoef(np.log(xa[i]), np.log(xb[i]))[0, 1]
            assert rho == pytest.approx(math.sqrt(ta / tb), abs=0.02)
        # increments over (t_m, t_{m+1}] have variance sigma^2 (t_{m+1} - t_m)
        inc = np.log(xb[0]) - np.log(xa[0])
        assert inc.var() == pytest.approx(0.04 * (tb - ta), rel=0.06)


def test_lattice_generator_is_max_min_distance(orc):
    for J, q in ((64, 2), (128, 3), (101, 4)):
        a = orc.korobov(J, q)
        gen = [pow(a, i, J) for i in range(q)]
        best = max(pins.korobov_min_dist_bruteforce(J, [pow(b, i, J) for i in range(q)])
                   for b in range(1, J))
        assert pins.korobov_min_dist_bruteforce(J, gen) == best
        # ties go to the smallest generator
        for b in range(1, a):
            assert pins.korobov_min_dist_bruteforce(J, [pow(b, i, J) for i in range(q)]) < best


def test_lattice_points_quantiles(orc, inputs):
    """Each free coordinate is the lognormal quantile of S_{t_m} at (k + 1/2)/J."""
    spec = inputs.geometric_put5()
    J, m = 64, 3
    x = orc.points_iz(spec, m, J)
    assert np.all(x[0] == spec.K)
    t = spec.dates[m - 1]
    a = orc.korobov(J, spec.d - 1)
    for i in range(1, spec.d):
        g = pow(a, i - 1, J)
        u = (((np.arange(J) * g) % J) + 0.5) / J
        mu = math.log(spec.S0[i]) + (spec.r - spec.delta[i] - 0.5 * spec.sigma[i] ** 2) * t
        expect = np.exp(mu + spec.sigma[i] * math.sqrt(t) * stats.norm.ppf(u))
        assert np.allclose(x[i], expect, rtol=1e-12)


def _last_interval(orc, spec, x, n, seed=9):
    rules = orc.empty_rules(spec, orc.CMC)
    m = spec.n_dates - 1
    return orc.continuation(spec, orc.CMC, rules, m, x, n, seed, nthreads=cpu_threads())


def test_last_interval_put_is_black_scholes(orc, inputs):
    spec = inputs.one_asset_put()
    x = np.array([[80.0, 95.0, 100.0, 104.0, 120.0]])
    r = _last_interval(orc, spec, x, 200000)
    tau = spec.dates[-1] - spec.dates[-2]
    for j in range(x.shape[1]):
        ref = pins.bs_put(x[0, j], spec.K, spec.r, 0.0, 0.2, tau)
        assert abs(r["cont"][j] - ref) < 4 * r["se"][j] + 1e-9
    # every path runs exactly one interval
    assert np.all(r["steps"] == 200000)


def test_last_interval_geometric_put_reduction(orc, inputs):
    spec = inputs.geometric_put5()
    rng = np.random.default_rng(2)
    x = 100.0 * np.exp(rng.normal(0, 0.08, size=(5, 6)))
    r = _last_interval(orc, spec, x, 100000)
    tau = spec.dates[-1] - spec.dates[-2]
    for j in range(x.shape[1]):
        ref = pins.geometric_put_european(x[:, j], spec, tau)
        assert abs(r["cont"][j] - ref) < 4 * r["se"][j] + 1e-9


def test_last_interval_max_call_quadrature(orc, inputs):
    spec = inputs.max_call(3, 100.0)
    x = np.array([[90.0, 100.0, 120.0], [100.0, 95.0, 80.0], [110.0, 100.0, 101.0]])
    r = _last_interval(orc, spec, x, 100000)
    tau = spec.dates[-1] - spec.dates[-2]
    for j in range(3):
        ref = pins.max_call_european(x[:, j], spec.K, spec.r, 0.1, 0.2, tau)
        assert abs(r["cont"][j] - ref) < 4 * r["se"][j] + 1e-9


def test_arithmetic_basket_put_one_asset_limit(orc, inputs):
    """With perfectly co-moving identical assets the arithmetic basket put is a
    one-asset put (correlation 1 written as a near-1 SPD matrix)."""
    spec = inputs.basket(3, 100.0, 100.0, 0.05, 0.0, 0.2, 1.0 - 1e-9, 1.0, 10, inputs.PUT_BASKET)
    x = np.full((3, 1), 96.0)
    r = _last_interval(orc, spec, x, 100000)
    ref = pins.bs_put(96.0, 100.0, 0.05, 0.0, 0.2, 0.1)
    assert abs(r["cont"][0] - ref) < 4 * r["se"][0] + 1e-6


def test_continuation_deterministic_and_thread_independent(orc, inputs):
    spec = inputs.geometric_put5()
    x = orc.points_cmc(spec, 5, 7, seed=1)
    rules = orc.empty_rules(spec, orc.CMC)
    a = orc.continuation(spec, orc.CMC, rules, 5, x, 5000, 3, nthreads=1)
    b = orc.continuation(spec, orc.CMC, rules, 5, x, 5000, 3, nthreads=cpu_threads())
    for k in ("cont", "se", "steps", "sum", "sumsq"):
        assert np.array_equal(a[k], b[k])
    c = orc.continuation(spec, orc.CMC, rules, 5, x, 5000, 4, nthreads=2)
    assert not np.array_equal(a["cont"], c["cont"])
