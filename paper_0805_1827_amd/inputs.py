"""Seeded synthetic option specifications.

Input generation only: this module holds none of the pricing method's
arithmetic.  Both the GPU library's callers and the CPU oracle's tests draw
their specs from here.  The option families are those of the paper's
experiments (max-call on d assets, Section 2.2 and Section 3.2, Tables 1-4)
and the basket/geometric puts used as checkable variants.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PUT_BASKET, CALL_MAX, PUT_GEO, CALL_MIN = 0, 1, 2, 3
PAYOFF_NAMES = {PUT_BASKET: "basket_put", CALL_MAX: "max_call", PUT_GEO: "geometric_put", CALL_MIN: "min_call"}


@dataclass
class OptionSpec:
    """d-asset Bermudan option under risk-neutral GBM."""
    d: int
    S0: np.ndarray
    delta: np.ndarray
    sigma: np.ndarray
    rho: np.ndarray          # d x d correlation
    K: float
    r: float
    T: float
    dates: np.ndarray        # t_1 < ... < t_NT = T
    payoff: int
    meta: dict = field(default_factory=dict)

    @property
    def n_dates(self) -> int:
        return int(len(self.dates))


def equal_dates(T: float, n_dates: int) -> np.ndarray:
    """t_m = m T / N_T, m = 1..N_T (t_0 = 0 is not an exercise date)."""
    return T * np.arange(1, n_dates + 1, dtype=np.float64) / n_dates


def basket(d: int, S0, K: float, r: float, delta, sigma, rho, T: float, n_dates: int,
           payoff: int) -> OptionSpec:
    S0 = np.broadcast_to(np.asarray(S0, dtype=np.float64), (d,)).copy()
    delta = np.broadcast_to(np.asarray(delta, dtype=np.float64), (d,)).copy()
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (d,)).copy()
    if np.isscalar(rho):
        R = np.full((d, d), float(rho))
        np.fill_diagonal(R, 1.0)
    else:
        R = np.asarray(rho, dtype=np.float64).reshape(d, d).copy()
    return OptionSpec(d, S0, delta, sigma, R, float(K), float(r), float(T),
                      equal_dates(T, n_dates), int(payoff))


def one_asset_put(n_dates: int = 10, T: float = 1.0, r: float = 0.05, sigma: float = 0.2,
                  S0: float = 100.0, K: float = 100.0) -> OptionSpec:
    """1-asset Bermudan put, S0 = K = 100, r = 0.05, sigma = 0.2, T = 1, 10 dates."""
    return basket(1, S0, K, r, 0.0, sigma, 1.0, T, n_dates, PUT_BASKET)


def geometric_put5(n_dates: int = 10) -> OptionSpec:
    """5-asset geometric-average Bermudan put, pairwise rho = 0.3, T = 1."""
    return basket(5, 100.0, 100.0, 0.05, 0.0, 0.2, 0.3, 1.0, n_dates, PUT_GEO)


def max_call(d: int, S0: float, n_dates: int = 9, T: float = 3.0) -> OptionSpec:
    """Max-call of Section 2.2 / Section 3.2: K = 100, r = 0.05, delta = 0.1,
    sigma = 0.2, independent assets, T = 3, 9 dates."""
    return basket(d, S0, 100.0, 0.05, 0.1, 0.2, 0.0, T, n_dates, CALL_MAX)


def min_call(d: int, S0, sigma=0.2, n_dates: int = 9, T: float = 3.0, delta: float = 0.1) -> OptionSpec:
    """Call on the minimum of d independent assets with the max-call's market
    block: K = 100, r = 0.05, T = 3, 9 dates."""
    return basket(d, S0, 100.0, 0.05, delta, sigma, 0.0, T, n_dates, CALL_MIN)


def wishart_corr(d: int, rng: np.random.Generator) -> np.ndarray:
    """Normalised Wishart(d, d+2) draw: W = G G^T, G in R^{d x (d+2)} iid N(0,1),
    rho = D^{-1/2} W D^{-1/2} with D = diag W."""
    G = rng.standard_normal((d, d + 2))
    W = G @ G.T
    s = 1.0 / np.sqrt(np.diag(W))
    R = W * s[:, None] * s[None, :]
    R = 0.5 * (R + R.T)
    np.fill_diagonal(R, 1.0)
    return R


def random_option(seed: int, d_range=(1, 20), dates_range=(4, 50),
                  n_choices=(1024, 4096, 16384)) -> OptionSpec:
    """One option of the uneven batch: d, date count, inner paths, vols,
    Wishart correlation and payoff drawn from a per-option seed.  Unset market
    parameters: S0 = K = 100, r = 0.05; puts T = 1 and delta = 0; max-calls
    T = 3 and delta = 0.1."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(d_range[0], d_range[1] + 1))
    n_dates = int(rng.integers(dates_range[0], dates_range[1] + 1))
    n = int(rng.choice(np.asarray(n_choices)))
    sigma = rng.uniform(0.1, 0.4, size=d)
    rho = wishart_corr(d, rng)
    payoff = int(rng.choice(np.asarray([PUT_BASKET, CALL_MAX, PUT_GEO])))
    if payoff == CALL_MAX:
        T, delta = 3.0, 0.1
    else:
        T, delta = 1.0, 0.0
    spec = basket(d, 100.0, 100.0, 0.05, delta, sigma, rho, T, n_dates, payoff)
    spec.meta = {"seed": int(seed), "n": n}
    return spec


def uneven_batch(count: int = 256, first_seed: int = 0) -> list[OptionSpec]:
    """The uneven-instance batch: options with seeds first_seed..first_seed+count-1."""
    return [random_option(s) for s in range(first_seed, first_seed + count)]


def serving_catalogue(size: int = 64, seed: int = 1000) -> list[OptionSpec]:
    """Catalogue of request specs for the serving loop: d in 1..40, 4..50 dates,
    n in {2k, 8k, 32k}."""
    return [random_option(seed + i, d_range=(1, 40), n_choices=(2048, 8192, 32768))
            for i in range(size)]


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate on [0, duration)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(t)
    return np.asarray(out)
