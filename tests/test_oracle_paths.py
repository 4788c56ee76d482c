"""Brute-force pins of the oracle's inner paths: a handful of paths simulated
one by one in NumPy from the model's definitions (risk-neutral log-Euler GBM
over the exercise dates with correlated normals, Sections 2.2 and 3.2; the
payoffs of Sections 2.1 and 3.2; the CMC stopping rule min{t : F_t > 0},
Section 3.2; discounting to the start date) must give the oracle's
continuation sums and step counts.

The random words come from the oracle's Philox (pinned separately against
rocRAND); everything after the words -- the uniform map, Box-Muller, the
counter layout of a step, NumPy's Cholesky factor, the GBM step, the payoff,
the exercise test, discounting and the sums -- is written here again,
independently, so that a dropped term, a wrong sign, a swapped index or a
wrong counter in the oracle's path loop fails one of these cases."""
import math

import numpy as np
import pytest


def brute_force(orc, inputs, spec, rules, m, x, n, seed, j=0):
    """Sum and sum of squares of the discounted payoffs and the executed
    path-steps of paths 0..n-1 started at point x (date m, point index j)."""
    d, NT = spec.d, spec.n_dates
    nblk = (d + 3) // 4
    k1 = (orc.STREAM_INNER << 16) | m
    L = np.linalg.cholesky(spec.rho)
    t = np.concatenate(([0.0], spec.dates))
    lnK = math.log(spec.K)

    def normals(k, p):
        z = []
        for b in range(nblk):
            w = orc.philox(seed, k1, [k * nblk + b, p, j, 0])
            u = (w.astype(np.float64) + 0.5) / 2.0 ** 32
            for h in range(2):
                rad = math.sqrt(-2.0 * math.log(u[2 * h]))
                ang = 2.0 * math.pi * u[2 * h + 1]
                z += [rad * math.cos(ang), rad * math.sin(ang)]
        return np.array(z[:d])

    def payoff(lnS):
        S = np.exp(lnS)
        if spec.payoff == inputs.PUT_BASKET:
            v = spec.K - S.mean()
        elif spec.payoff == inputs.CALL_MAX:
            v = S.max() - spec.K
        elif spec.payoff == inputs.CALL_MIN:
            v = S.min() - spec.K
        else:
            v = spec.K - math.exp(lnS.mean())
        return max(v, 0.0)

    def exercise(k, lnS, pay):
        if pay <= 0.0:
            return False
        u = lnS - lnK
        g = pay / spec.K
        feats = np.concatenate(([1.0], u, u * u, [g, g * g]))
        return float(rules[k] @ feats) > 0.0

    s1 = s2 = 0.0
    steps = 0
    drift = spec.r - spec.delta - 0.5 * spec.sigma ** 2
    for p in range(n):
        lnS = np.log(x).astype(np.float64)
        for k in range(m + 1, NT + 1):
            dt = t[k] - t[k - 1]
            lnS = lnS + drift * dt + spec.sigma * math.sqrt(dt) * (L @ normals(k, p))
            pay = payoff(lnS)
            if k == NT or exercise(k, lnS, pay):
                v = math.exp(-spec.r * (t[k] - t[m])) * pay
                s1 += v
                s2 += v * v
                steps += k - m
                break
    return s1, s2, steps


def some_rules(rng, spec):
    """Rule rows that exercise a fair share of in-the-money paths: F = a + b g
    with a < 0 < b, so that deep in-the-money states stop, plus small random
    weights on the other features."""
    d = spec.d
    rows = rng.normal(0.0, 0.05, size=(spec.n_dates + 1, 2 * d + 3))
    rows[:, 0] = -0.02
    rows[:, 1 + 2 * d] = 1.0
    return rows


CASES = [
    # d, payoff, S0, rho, dates, start date
    (1, "PUT_BASKET", 95.0, 0.0, 6, 0),
    (2, "CALL_MAX", 105.0, 0.3, 5, 1),
    (3, "CALL_MIN", 110.0, 0.2, 4, 0),
    (5, "PUT_GEO", 98.0, 0.3, 10, 3),
    (6, "PUT_BASKET", 97.0, 0.5, 3, 1),
]


@pytest.mark.parametrize("d,payoff,S0,rho,nd,m", CASES)
def test_paths_match_brute_force(orc, inputs, d, payoff, S0, rho, nd, m):
    rng = np.random.default_rng(100 + d)
    T = 3.0 if payoff in ("CALL_MAX", "CALL_MIN") else 1.0
    delta = 0.1 if payoff in ("CALL_MAX", "CALL_MIN") else 0.0
    spec = inputs.basket(d, S0, 100.0, 0.05, delta, rng.uniform(0.15, 0.35, d), rho, T, nd,
                         getattr(inputs, payoff))
    rules = some_rules(rng, spec)
    x = (S0 * np.exp(rng.normal(0.0, 0.1, size=(d, 3)))).astype(np.float64)
    n, seed = 7, 11
    ref = orc.continuation(spec, orc.CMC, rules, m, x, n, seed, nthreads=1)
    stopped_early = False
    for j in range(x.shape[1]):
        s1, s2, steps = brute_force(orc, inputs, spec, rules, m, x[:, j], n, seed, j)
        assert ref["sum"][j] == pytest.approx(s1, rel=1e-12, abs=1e-12 * spec.K)
        assert ref["sumsq"][j] == pytest.approx(s2, rel=1e-12, abs=1e-12 * spec.K ** 2)
        assert ref["steps"][j] == steps
        assert ref["cont"][j] == pytest.approx(s1 / n, rel=1e-12, abs=1e-12 * spec.K)
        stopped_early |= steps < n * (spec.n_dates - m)
    # the rules stop some paths before maturity, so the exercise branch is exercised
    assert stopped_early


def test_paths_depend_on_point_index_and_date(orc, inputs):
    """The counters carry the point index and the key carries the date: the
    same point under another index or start date draws other paths."""
    spec = inputs.basket(3, 100.0, 100.0, 0.05, 0.0, 0.2, 0.3, 1.0, 6, inputs.PUT_GEO)
    rules = orc.empty_rules(spec, orc.CMC)
    x = np.full((3, 1), 100.0)
    a = orc.continuation(spec, orc.CMC, rules, 1, x, 5, 3, nthreads=1, ids=[0])
    b = orc.continuation(spec, orc.CMC, rules, 1, x, 5, 3, nthreads=1, ids=[1])
    c = orc.continuation(spec, orc.CMC, rules, 2, x, 5, 3, nthreads=1, ids=[0])
    assert a["sum"][0] != b["sum"][0]
    assert a["sum"][0] != c["sum"][0]
    s1, _, _ = brute_force(orc, inputs, spec, rules, 1, x[:, 0], 5, 3, j=1)
    assert b["sum"][0] == pytest.approx(s1, rel=1e-12)
