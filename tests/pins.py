"""Closed forms and brute-force references that pin the oracle.

Each routine is a textbook result written independently of the oracle:
Black-Scholes-Merton, the Cox-Ross-Rubinstein tree (European, Bermudan,
American), the reduction of a geometric-average basket to one lognormal asset,
the European max-call on independent assets by one-dimensional quadrature,
and the logistic-regression maximum likelihood solved by a generic optimiser.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize, stats


def bs_put(S0, K, r, q, sigma, T):
    if sigma == 0.0 or T == 0.0:
        return max(K * math.exp(-r * T) - S0 * math.exp(-q * T), 0.0)
    sq = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r - q + 0.5 * sigma * sigma) * T) / sq
    d2 = d1 - sq
    return K * math.exp(-r * T) * stats.norm.cdf(-d2) - S0 * math.exp(-q * T) * stats.norm.cdf(-d1)


def bs_call(S0, K, r, q, sigma, T):
    sq = sigma * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r - q + 0.5 * sigma * sigma) * T) / sq
    d2 = d1 - sq
    return S0 * math.exp(-q * T) * stats.norm.cdf(d1) - K * math.exp(-r * T) * stats.norm.cdf(d2)


def crr_put(S0, K, r, q, sigma, T, steps, n_dates=None, american=False, want_boundary=False):
    """CRR binomial put.  n_dates=None and american=False: European.
    n_dates=k: Bermudan with exercise at t_m = m T / k, m = 1..k (t_0 excluded).
    Returns the price and, if asked, the critical price at each exercise step
    (largest node price at which exercise is optimal)."""
    dt = T / steps
    u = math.exp(sigma * math.sqrt(dt))
    dn = 1.0 / u
    p = (math.exp((r - q) * dt) - dn) / (u - dn)
    disc = math.exp(-r * dt)
    j = np.arange(steps + 1)
    S = S0 * u ** j * dn ** (steps - j)
    V = np.maximum(K - S, 0.0)
    ex_steps = set()
    if n_dates is not None:
        assert steps % n_dates == 0
        ex_steps = {m * steps // n_dates for m in range(1, n_dates)}
    boundary = {}
    for i in range(steps - 1, -1, -1):
        V = disc * (p * V[1:] + (1 - p) * V[:-1])
        if (american and i > 0) or i in ex_steps:
            j = np.arange(i + 1)
            S = S0 * u ** j * dn ** (i - j)
            intrinsic = np.maximum(K - S, 0.0)
            ex = (intrinsic >= V) & (intrinsic > 0)
            if want_boundary:
                boundary[i] = float(S[ex].max()) if ex.any() else 0.0
            V = np.maximum(V, intrinsic)
    if want_boundary:
        return float(V[0]), boundary
    return float(V[0])


def max_call2_tree(S0, K, r, delta, sigma, T, steps, n_dates, want_boundary=False, kind="max"):
    """Bermudan call on the maximum (kind="max") or the minimum (kind="min")
    of two independent assets: the product of two CRR trees (four branches per
    step), exercise at t_m = m T / n_dates, m = 1..n_dates.  With
    want_boundary, for every exercise step i and asset a the critical prices
    of asset a against the other asset's node prices: boundary[i][a] = (other
    prices, critical prices), the smallest price of asset a at which exercise
    becomes optimal, above the other asset for the max-call and below it for
    the min-call, by linear interpolation in ln S_a of exercise value minus
    continuation value."""
    best = np.maximum if kind == "max" else np.minimum
    assert steps % n_dates == 0
    dt = T / steps
    u = [math.exp(s * math.sqrt(dt)) for s in sigma]
    p = [(math.exp((r - q) * dt) - 1.0 / uu) / (uu - 1.0 / uu) for q, uu in zip(delta, u)]
    disc = math.exp(-r * dt)

    def prices(i):
        k = np.arange(i + 1)
        return [S0[a] * u[a] ** (2.0 * k - i) for a in range(2)]

    Sa, Sb = prices(steps)
    V = np.maximum(best(Sa[:, None], Sb[None, :]) - K, 0.0)
    ex_steps = {m * steps // n_dates for m in range(1, n_dates)}
    boundary = {}
    for i in range(steps - 1, -1, -1):
        pa, pb = p
        V = disc * (pa * pb * V[1:, 1:] + pa * (1 - pb) * V[1:, :-1]
                    + (1 - pa) * pb * V[:-1, 1:] + (1 - pa) * (1 - pb) * V[:-1, :-1])
        if i in ex_steps:
            Sa, Sb = prices(i)
            pay = np.maximum(best(Sa[:, None], Sb[None, :]) - K, 0.0)
            if want_boundary:
                g = pay - V
                out = {}
                for a in range(2):
                    ga = g if a == 0 else g.T          # rows: asset a, columns: the other
                    own, other = (Sa, Sb) if a == 0 else (Sb, Sa)
                    xs, ys = [], []
                    for c in range(len(other)):
                        col = ga[:, c]
                        for k in range(1, len(own)):
                            inside = own[k - 1] > other[c] if kind == "max" else own[k] < other[c]
                            if inside and col[k - 1] <= 0.0 < col[k]:
                                w = col[k - 1] / (col[k - 1] - col[k])
                                ys.append(math.exp((1 - w) * math.log(own[k - 1]) + w * math.log(own[k])))
                                xs.append(other[c])
                                break
                    out[a] = (np.array(xs), np.array(ys))
                boundary[i] = out
            V = np.maximum(V, pay)
    if want_boundary:
        return float(V[0, 0]), boundary
    return float(V[0, 0])


def geometric_reduction(spec):
    """The geometric average of d correlated GBMs is one GBM:
    sigma_G^2 = sum_ij rho_ij sigma_i sigma_j / d^2,
    delta_G  = mean(delta_i + sigma_i^2 / 2) - sigma_G^2 / 2,
    G_0      = (prod S0_i)^(1/d)."""
    d = spec.d
    sig = np.asarray(spec.sigma)
    var = float(sig @ np.asarray(spec.rho) @ sig) / (d * d)
    dG = float(np.mean(np.asarray(spec.delta) + 0.5 * sig ** 2)) - 0.5 * var
    G0 = float(np.exp(np.mean(np.log(spec.S0))))
    return G0, math.sqrt(var), dG


def geometric_put_european(x, spec, tau):
    """European geometric put from point x (vector of d prices) with maturity tau."""
    G0 = float(np.exp(np.mean(np.log(x))))
    _, sG, dG = geometric_reduction(spec)
    return bs_put(G0, spec.K, spec.r, dG, sG, tau)


def max_call_european(x, K, r, delta, sigma, tau):
    """European call on the maximum of independent GBMs, by quadrature of
    E[(M - K)^+] = int_K^inf (1 - prod_i F_i(y)) dy, F_i the lognormal CDFs."""
    x = np.asarray(x, dtype=float)
    delta = np.broadcast_to(delta, x.shape)
    sigma = np.broadcast_to(sigma, x.shape)
    mu = np.log(x) + (r - delta - 0.5 * sigma ** 2) * tau
    sd = sigma * math.sqrt(tau)

    def tail(y):
        return 1.0 - float(np.prod(stats.norm.cdf((math.log(y) - mu) / sd)))

    hi = float(np.max(np.exp(mu + 12 * sd)))
    val, _ = integrate.quad(tail, K, hi, limit=400, epsabs=1e-10, epsrel=1e-10)
    return math.exp(-r * tau) * val


def min_call_european(x, K, r, delta, sigma, tau):
    """European call on the minimum of independent GBMs, by quadrature of
    E[(m - K)^+] = int_K^inf prod_i (1 - F_i(y)) dy, F_i the lognormal CDFs."""
    x = np.asarray(x, dtype=float)
    delta = np.broadcast_to(delta, x.shape)
    sigma = np.broadcast_to(sigma, x.shape)
    mu = np.log(x) + (r - delta - 0.5 * sigma ** 2) * tau
    sd = sigma * math.sqrt(tau)

    def tail(y):
        return float(np.prod(stats.norm.sf((math.log(y) - mu) / sd)))

    hi = float(np.min(np.exp(mu + 12 * sd)))
    val, _ = integrate.quad(tail, K, hi, limit=400, epsabs=1e-10, epsrel=1e-10)
    return math.exp(-r * tau) * val


def korobov_min_dist_bruteforce(J, gen):
    """Minimal squared toroidal distance over all point pairs (in units 1/J)."""
    j = np.arange(J)
    pts = np.stack([(j * g) % J for g in gen], axis=1)
    best = None
    for a in range(J):
        diff = np.abs(pts[a + 1:] - pts[a])
        diff = np.minimum(diff, J - diff)
        if len(diff):
            m = int((diff ** 2).sum(axis=1).min())
            best = m if best is None else min(best, m)
    return best


def logistic_mle(Phi, e):
    """Maximiser of sum_j [e_j log pi_j + (1 - e_j) log(1 - pi_j)] with
    pi_j = 1 / (1 + exp(-2 Phi_j . w)), by BFGS on standardised columns."""
    mu = Phi[:, 1:].mean(axis=0)
    sd = Phi[:, 1:].std(axis=0)
    Z = np.column_stack([np.ones(len(Phi)), (Phi[:, 1:] - mu) / sd])

    def nll(g):
        F2 = 2.0 * (Z @ g)
        return float(np.sum(np.logaddexp(0.0, F2) - e * F2))

    def grad(g):
        pi = 1.0 / (1.0 + np.exp(-2.0 * (Z @ g)))
        return 2.0 * Z.T @ (pi - e)

    res = optimize.minimize(nll, np.zeros(Z.shape[1]), jac=grad, method="BFGS",
                            options={"gtol": 1e-12, "maxiter": 10000})
    g = res.x
    w = np.empty_like(g)
    w[1:] = g[1:] / sd
    w[0] = g[0] - float(np.sum(g[1:] * mu / sd))
    return w
