"""Pins of the oracle's AdaBoost-stump classifier (CMC [class], Section 3.2).

* brute force: on tiny training sets every round is re-run from the
  definitions (features, bins, fixed-point weights, all stumps enumerated,
  AdaBoost update) and must pick the same stumps with the same errors;
* the Freund-Schapire bound: the cost-weighted training error of sign F is at
  most the product of 2 sqrt(eps_t (1 - eps_t));
* a rule learned from labels that switch at a known price switches within one
  bin of it;
* whole prices against the CRR tree, the reduced geometric tree and Table 4.
"""
import json
import math
from pathlib import Path

import numpy as np
import pytest

import pins
from conftest import cpu_threads

NT = cpu_threads()
GOLDEN = Path(__file__).resolve().parent / "golden"
B = 64


_exp = np.vectorize(math.exp)      # the C library's exp and log, as the oracle calls them
_log = np.vectorize(math.log)


def _psi_payoff(spec, x):
    """Features and payoff from the log-prices, summed asset by asset."""
    lx = _log(x)
    u = lx - math.log(spec.K)
    acc = np.zeros(x.shape[1])
    if spec.payoff == 1:
        acc = _exp(lx[0])
        for i in range(1, spec.d):
            acc = np.maximum(acc, _exp(lx[i]))
        pay = acc - spec.K
    elif spec.payoff == 2:
        for i in range(spec.d):
            acc = acc + lx[i]
        pay = spec.K - _exp(acc / spec.d)
    else:
        for i in range(spec.d):
            acc = acc + _exp(lx[i])
        pay = spec.K - acc / spec.d
    pay = np.maximum(pay, 0.0)
    return np.vstack([u, pay / spec.K]), pay


def _brute_force_boost(spec, x, cont, rounds):
    """Every stump enumerated, every round; plain loops over the definitions."""
    psi, pay = _psi_payoff(spec, x)
    itm = pay > 0
    psi, beta = psi[:, itm], (pay - cont)[itm]
    y = np.where(beta > 0, 1, -1)
    w = np.abs(beta)
    nf, nI = psi.shape
    lo, hi = psi.min(axis=1), psi.max(axis=1)
    bins = np.zeros((nf, nI), dtype=int)
    for f in range(nf):
        if hi[f] > lo[f]:
            inv = B / (hi[f] - lo[f])
            bins[f] = np.clip(np.floor((psi[f] - lo[f]) * inv), 0, B - 1).astype(int)
    shift = 50 - math.frexp(nI * w.max())[1]
    out = []
    for _ in range(rounds):
        W = np.array([int(np.rint(math.ldexp(v, shift))) for v in w], dtype=np.int64)
        total = int(W.sum())
        best = None
        for f in range(nf):
            for k in range(B):
                if k == 0 and f > 0:
                    continue
                for s in (1, -1):
                    h = np.where(bins[f] >= k, s, -s)
                    err = int(W[h != y].sum())
                    if best is None or err < best[0]:
                        best = (err, f, k, s)
        err, f, k, s = best
        if 2 * err >= total:
            break
        eps = err / total
        out.append((f, k, s, eps))
        if err == 0:
            break
        h = np.where(bins[f] >= k, s, -s)
        w = np.where(h != y, w / (2.0 * eps), w / (2.0 * (1.0 - eps)))
    return out, lo, hi


@pytest.mark.parametrize("case", ["put2", "maxcall3", "geo1"])
def test_boosting_rounds_match_brute_force(orc, inputs, case):
    rng = np.random.default_rng({"put2": 1, "maxcall3": 2, "geo1": 3}[case])
    if case == "put2":
        spec = inputs.basket(2, 100.0, 100.0, 0.05, 0.0, [0.2, 0.3], 0.3, 1.0, 5, inputs.PUT_BASKET)
    elif case == "maxcall3":
        spec = inputs.max_call(3, 100.0)
    else:
        spec = inputs.one_asset_put()
    N = 60
    x = 100.0 * np.exp(rng.normal(0.0, 0.25, (spec.d, N)))
    _, pay = _psi_payoff(spec, x)
    cont = np.maximum(pay + rng.normal(0.0, 3.0, N), 0.0)      # noisy labels: many rounds
    rounds = 12
    row, tr = orc.fit_ada(spec, x, cont, rounds=rounds, trace=True)
    want, lo, hi = _brute_force_boost(spec, x, cont, rounds)
    assert np.array_equal(tr["lo"], lo) and np.array_equal(tr["hi"], hi)
    assert len(tr["feature"]) == len(want) >= 3
    for t, (f, k, s, eps) in enumerate(want):
        assert (tr["feature"][t], tr["bin"][t], tr["sign"][t]) == (f, k, s), t
        assert tr["eps"][t] == eps, t
        assert tr["alpha"][t] == pytest.approx(0.5 * math.log((1 - eps) / eps), rel=1e-14)


def _evaluate_row(spec, row, x):
    """Score of the folded row: base plus, per feature, the running sum at the
    number of its (ascending) thresholds the feature value reaches."""
    psi, pay = _psi_payoff(spec, x)
    nf = spec.d + 1
    F = np.full(x.shape[1], row[0])
    at = 1 + nf
    for f in range(nf):
        c = int(row[1 + f])
        th, run = row[at:at + c], row[at + c:at + 2 * c]
        assert np.all(np.diff(th) >= 0)
        k = (psi[f][:, None] >= th[None, :]).sum(axis=1)
        F += np.where(k > 0, run[np.maximum(k - 1, 0)], 0.0)
        at += 2 * c
    return F, pay


def test_folded_row_equals_the_stump_sum(orc, inputs):
    """The folded row scores every point as base + sum_t alpha_t h_t(x)
    written out stump by stump from the trace."""
    spec = inputs.basket(2, 100.0, 100.0, 0.05, 0.0, [0.2, 0.3], 0.3, 1.0, 5, inputs.PUT_BASKET)
    rng = np.random.default_rng(8)
    x = 100.0 * np.exp(rng.normal(0.0, 0.2, (2, 400)))
    _, pay = _psi_payoff(spec, x)
    cont = np.maximum(pay + rng.normal(0.0, 2.0, 400), 0.0)
    row, tr = orc.fit_ada(spec, x, cont, rounds=30, trace=True)
    probe = 100.0 * np.exp(rng.normal(0.0, 0.25, (2, 3000)))
    F, _ = _evaluate_row(spec, row, probe)
    psi, _ = _psi_payoff(spec, probe)
    direct = np.zeros(probe.shape[1])
    for f, k, s, a in zip(tr["feature"], tr["bin"], tr["sign"], tr["alpha"]):
        theta = -np.inf if k == 0 else tr["lo"][f] + k * ((tr["hi"][f] - tr["lo"][f]) / 64)
        direct += a * np.where(psi[f] >= theta, s, -s)
    assert np.allclose(F, direct, atol=1e-9)


def test_training_error_within_adaboost_bound(orc, inputs):
    """Freund & Schapire: the weighted training error of sign(sum alpha_t h_t)
    is at most prod_t 2 sqrt(eps_t (1 - eps_t)) under the initial weights."""
    spec = inputs.geometric_put5()
    m = 5
    x = orc.points_cmc(spec, m, 800, 3)
    cont = orc.continuation(spec, orc.CMC, orc.empty_rules(spec, orc.CMC), m, x, 200, 3, nthreads=NT)["cont"]
    row, tr = orc.fit_ada(spec, x, cont, rounds=40, trace=True)
    F, pay = _evaluate_row(spec, row, x)
    itm = pay > 0
    beta = (pay - cont)[itm]
    c = np.abs(beta)
    wrong = np.sign(F[itm]) != np.where(beta > 0, 1.0, -1.0)
    err = c[wrong].sum() / c.sum()
    bound = float(np.prod(2.0 * np.sqrt(tr["eps"] * (1.0 - tr["eps"]))))
    assert len(tr["eps"]) == 40 and np.all(tr["eps"] < 0.5)
    assert err <= bound + 1e-12
    assert err < 0.2


def test_rule_switches_at_the_label_boundary(orc, inputs):
    """Labels exercise iff S < 92 (cost |92 - S|): the learned rule on the
    one-asset put switches within one bin of 92."""
    spec = inputs.one_asset_put()
    rng = np.random.default_rng(5)
    x = np.sort(100.0 * np.exp(rng.normal(0.0, 0.12, (1, 400))), axis=1)
    pay = np.maximum(spec.K - x[0], 0.0)
    cont = pay - (92.0 - x[0])
    row, tr = orc.fit_ada(spec, x, cont, rounds=8, trace=True)
    grid = np.linspace(70.0, 99.9, 3000).reshape(1, -1)
    F, _ = _evaluate_row(spec, row, grid)
    ex = F > 0
    assert ex[0] and not ex[-1]
    switch = grid[0, np.argmax(~ex)]
    bin_width = math.exp(tr["hi"][0]) / math.exp(tr["lo"][0])    # generous: ratio of the range's ends
    width_price = 100.0 * (tr["hi"][0] - tr["lo"][0]) / B
    assert abs(switch - 92.0) <= width_price + 0.05, (switch, bin_width)
    assert np.all(np.diff(ex.astype(int)) <= 0)                  # one switch


def test_degenerate_training_sets_never_exercise(orc, inputs):
    spec = inputs.one_asset_put()
    x = np.full((1, 10), 120.0)                                  # out of the money
    row = orc.fit_ada(spec, x, np.zeros(10))
    assert np.all(row == 0.0)
    x = np.full((1, 10), 90.0)
    row = orc.fit_ada(spec, x, np.full(10, 10.0))               # Phi - C = 0 everywhere: no cost
    assert np.all(row == 0.0)


@pytest.fixture(scope="module")
def trees():
    berm = pins.crr_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0, 2000, n_dates=10)
    return {"put1": berm}


def test_ada_one_asset_put_against_tree(orc, inputs, trees):
    spec = inputs.one_asset_put()
    r = orc.price(spec, orc.CMC_ADA, 1000, 500, 200000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - trees["put1"]) <= 3 * se + 0.01 * trees["put1"]
    assert r["price"] <= trees["put1"] + 3 * se
    assert r["price"] > pins.bs_put(100.0, 100.0, 0.05, 0.0, 0.2, 1.0) + 10 * se


def test_ada_geometric_put5_against_reduced_tree(orc, inputs):
    spec = inputs.geometric_put5()
    G0, sG, dG = pins.geometric_reduction(spec)
    tree = pins.crr_put(G0, 100.0, 0.05, dG, sG, 1.0, 2000, n_dates=10)
    r = orc.price(spec, orc.CMC_ADA, 2000, 400, 200000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - tree) <= 3 * se + 0.01 * tree
    assert r["price"] <= tree + 3 * se


def test_ada_max_call_d3_against_paper_table4(orc, inputs):
    gold = json.loads((GOLDEN / "paper_tables.json").read_text())["table4_cmc"]["rows"]
    row = [g for g in gold if g["S0"] == 100][0]
    spec = inputs.max_call(3, 100.0)
    r = orc.price(spec, orc.CMC_ADA, 2000, 300, 200000, 1, nthreads=NT)
    se = r["std_err"]
    assert abs(r["price"] - row["binomial"]) <= 3 * se + 0.01 * row["binomial"]
    euro = pins.max_call_european(spec.S0, 100.0, 0.05, 0.1, 0.2, 3.0)
    assert r["price"] > euro + 10 * se
