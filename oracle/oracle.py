"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports this
module.  Specs are duck-typed (attributes d, S0, delta, sigma, rho, K, r, T,
dates, payoff) so that this wrapper imports nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "liboracle.so"

PUT_BASKET, CALL_MAX, PUT_GEO, CALL_MIN = 0, 1, 2, 3
SEARCH_PLAIN, SEARCH_SECANT = 0, 1
CMC, IZ, CMC_ADA = 0, 1, 2
ADA_BINS, ADA_TMAX = 64, 64
ADA_ROUNDS = 64          # default AdaBoost rounds
STREAM_OUTER, STREAM_INNER, STREAM_FINAL = 1, 2, 3


def build(force: bool = True) -> Path:
    """Compile liboracle.so with gcc (FP64, no contraction)."""
    if LIB_PATH.exists() and not force:
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-pthread", str(HERE / "oracle.c"), "-o", str(LIB_PATH) + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(str(LIB_PATH) + ".tmp", LIB_PATH)
    return LIB_PATH


class _Spec(C.Structure):
    _fields_ = [("d", C.c_int32), ("S0", C.POINTER(C.c_double)), ("delta", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("K", C.c_double), ("r", C.c_double), ("T", C.c_double),
                ("n_dates", C.c_int32), ("dates", C.POINTER(C.c_double)), ("payoff", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            build()
        L = C.CDLL(str(LIB_PATH))
        dp, i64p, i32p, u32p = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32), C.POINTER(C.c_uint32))
        sp = C.POINTER(_Spec)
        L.orc_rule_width.argtypes = [C.c_int, C.c_int]
        L.orc_iz_regions.argtypes = [sp]
        L.orc_rule_width_spec.argtypes = [sp, C.c_int]
        L.orc_philox.argtypes = [C.c_uint32, C.c_uint32, u32p, u32p]
        L.orc_philox.restype = None
        L.orc_normal_block.argtypes = [C.c_uint32, C.c_uint32, u32p, dp]
        L.orc_normal_block.restype = None
        L.orc_cholesky.argtypes = [C.c_int, dp, dp]
        L.orc_payoff.argtypes = [sp, dp]
        L.orc_payoff.restype = C.c_double
        L.orc_points_cmc.argtypes = [sp, C.c_int, C.c_int64, C.c_uint32, dp]
        L.orc_korobov.argtypes = [C.c_int64, C.c_int]
        L.orc_korobov.restype = C.c_int64
        L.orc_points_iz.argtypes = [sp, C.c_int, C.c_int, C.c_int64, dp]
        L.orc_continuation.argtypes = [sp, C.c_int, dp, C.c_int, dp, C.c_int64, u32p, C.c_int64,
                                       C.c_uint32, C.c_int, C.c_int, dp, dp, i64p, dp, dp]
        L.orc_fit_cmc.argtypes = [sp, dp, dp, C.c_int64, C.c_int, dp]
        L.orc_fit_ada.argtypes = [sp, dp, dp, C.c_int64, C.c_int, dp, i32p, i32p, i32p, i32p, dp, dp, dp, dp]
        L.orc_iz_search.argtypes = [sp, dp, C.c_int, C.c_int, dp, C.c_int64, C.c_int64, C.c_uint32,
                                    C.c_double, C.c_int, C.c_int, C.c_int, dp, i32p, i64p]
        L.orc_fit_iz.argtypes = [sp, C.c_int, dp, dp, C.c_int64, dp]
        L.orc_price.argtypes = [sp, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_uint32,
                                C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _SpecHolder:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, spec):
        d = int(spec.d)
        self.S0 = np.ascontiguousarray(spec.S0, dtype=np.float64).reshape(d)
        self.delta = np.ascontiguousarray(spec.delta, dtype=np.float64).reshape(d)
        self.sigma = np.ascontiguousarray(spec.sigma, dtype=np.float64).reshape(d)
        self.rho = np.ascontiguousarray(spec.rho, dtype=np.float64).reshape(d * d)
        self.dates = np.ascontiguousarray(spec.dates, dtype=np.float64)
        self.c = _Spec(d, _dp(self.S0), _dp(self.delta), _dp(self.sigma), _dp(self.rho),
                       float(spec.K), float(spec.r), float(spec.T), len(self.dates),
                       _dp(self.dates), int(spec.payoff))
        self.d = d
        self.n_dates = len(self.dates)

    @property
    def ptr(self):
        return C.byref(self.c)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def rule_width(method: int, d: int) -> int:
    """Coefficients of one CMC rule or of one I&Z region's boundary."""
    return int(lib().orc_rule_width(method, d))


def iz_regions(spec) -> int:
    return int(lib().orc_iz_regions(_SpecHolder(spec).ptr))


def row_width(spec, method: int) -> int:
    """Width of a rule row: every I&Z region's boundary block side by side."""
    return int(lib().orc_rule_width_spec(_SpecHolder(spec).ptr, method))


def philox(k0: int, k1: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF,
                     c.ctypes.data_as(C.POINTER(C.c_uint32)), out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def normal_block(k0: int, k1: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    out = np.zeros(4, dtype=np.float64)
    lib().orc_normal_block(k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF,
                           c.ctypes.data_as(C.POINTER(C.c_uint32)), _dp(out))
    return out


def cholesky(rho: np.ndarray) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    d = rho.shape[0]
    L = np.zeros((d, d))
    rc = lib().orc_cholesky(d, _dp(rho), _dp(L))
    if rc != 0:
        raise ValueError("correlation matrix is not positive definite")
    return L


def payoff(spec, logS) -> float:
    h = _SpecHolder(spec)
    v = np.ascontiguousarray(logS, dtype=np.float64)
    return float(lib().orc_payoff(h.ptr, _dp(v)))


def points_cmc(spec, m: int, N: int, seed: int) -> np.ndarray:
    h = _SpecHolder(spec)
    x = np.zeros((h.d, N))
    _check(lib().orc_points_cmc(h.ptr, m, N, seed, _dp(x)), "points_cmc")
    return x


def korobov(J: int, q: int) -> int:
    return int(lib().orc_korobov(J, q))


def points_iz(spec, m: int, J: int, region: int = 0) -> np.ndarray:
    h = _SpecHolder(spec)
    x = np.zeros((h.d, J))
    _check(lib().orc_points_iz(h.ptr, m, region, J, _dp(x)), "points_iz")
    return x


def empty_rules(spec, method: int) -> np.ndarray:
    return np.zeros((len(spec.dates) + 1, row_width(spec, method)))


def continuation(spec, method: int, rules, m: int, x: np.ndarray, n: int, seed: int,
                 stream: int = STREAM_INNER, nthreads: int = 0, ids=None) -> dict:
    """ids: optional point indices used in the random-number counters."""
    h = _SpecHolder(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    N = x.shape[1]
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32).reshape(N)
        idp = ids.ctypes.data_as(C.POINTER(C.c_uint32))
    rules = np.ascontiguousarray(rules, dtype=np.float64)
    cont, se, sm, sq = (np.zeros(N) for _ in range(4))
    steps = np.zeros(N, dtype=np.int64)
    _check(lib().orc_continuation(h.ptr, method, _dp(rules), m, _dp(x), N, idp, n, seed, stream,
                                  nthreads, _dp(cont), _dp(se),
                                  steps.ctypes.data_as(C.POINTER(C.c_int64)), _dp(sm), _dp(sq)),
           "continuation")
    return {"cont": cont, "se": se, "steps": steps, "sum": sm, "sumsq": sq}


def final_price(spec, method: int, rules, n_final: int, seed: int, nthreads: int = 0) -> dict:
    x0 = np.ascontiguousarray(spec.S0, dtype=np.float64).reshape(-1, 1)
    r = continuation(spec, method, rules, 0, x0, n_final, seed, STREAM_FINAL, nthreads)
    s, q = r["sum"][0], r["sumsq"][0]
    price = s / n_final
    var = max((q - s * s / n_final) / (n_final - 1), 0.0)
    se = float(np.sqrt(var / n_final))
    return {"price": price, "variance": var, "std_err": se, "ci95": 1.96 * se,
            "final_steps": int(r["steps"][0])}


def fit_cmc(spec, x: np.ndarray, cont: np.ndarray, rounds: int = 8) -> np.ndarray:
    h = _SpecHolder(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    cont = np.ascontiguousarray(cont, dtype=np.float64)
    w = np.zeros(rule_width(CMC, h.d))
    _check(lib().orc_fit_cmc(h.ptr, _dp(x), _dp(cont), x.shape[1], rounds, _dp(w)), "fit_cmc")
    return w


def iz_search(spec, rules, m: int, x: np.ndarray, n: int, seed: int, eps: float = 0.01,
              max_iter: int = 100, nthreads: int = 0, region: int = 0, mode: int = SEARCH_PLAIN) -> dict:
    h = _SpecHolder(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    J = x.shape[1]
    rules = np.ascontiguousarray(rules, dtype=np.float64)
    s = np.zeros(J)
    it = np.zeros(J, dtype=np.int32)
    st = C.c_int64(0)
    _check(lib().orc_iz_search(h.ptr, _dp(rules), m, region, _dp(x), J, n, seed, eps, max_iter, mode, nthreads,
                               _dp(s), it.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(st)),
           "iz_search")
    return {"s": s, "iters": it, "steps": int(st.value)}


def fit_iz(spec, x: np.ndarray, sstar: np.ndarray, region: int = 0) -> np.ndarray:
    h = _SpecHolder(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    sstar = np.ascontiguousarray(sstar, dtype=np.float64)
    b = np.zeros(rule_width(IZ, h.d))
    _check(lib().orc_fit_iz(h.ptr, region, _dp(x), _dp(sstar), x.shape[1], _dp(b)), "fit_iz")
    return b


def fit_ada(spec, x: np.ndarray, cont: np.ndarray, rounds: int = ADA_ROUNDS, trace: bool = False):
    """AdaBoost-stump rule row; with trace, also the stumps and feature ranges."""
    h = _SpecHolder(spec)
    x = np.ascontiguousarray(x, dtype=np.float64)
    cont = np.ascontiguousarray(cont, dtype=np.float64)
    row = np.zeros(rule_width(CMC_ADA, h.d))
    nf = h.d + 1
    T = np.zeros(1, dtype=np.int32)
    feat, k, sg = (np.zeros(ADA_TMAX, dtype=np.int32) for _ in range(3))
    eps, alpha = np.zeros(ADA_TMAX), np.zeros(ADA_TMAX)
    lo, hi = np.zeros(nf), np.zeros(nf)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    _check(lib().orc_fit_ada(h.ptr, _dp(x), _dp(cont), x.shape[1], rounds, _dp(row), ip(T), ip(feat), ip(k),
                             ip(sg), _dp(eps), _dp(alpha), _dp(lo), _dp(hi)), "fit_ada")
    if not trace:
        return row
    t = int(T[0])
    return row, {"feature": feat[:t].copy(), "bin": k[:t].copy(), "sign": sg[:t].copy(), "eps": eps[:t].copy(),
                 "alpha": alpha[:t].copy(), "lo": lo, "hi": hi}


def price(spec, method: int, N: int, n: int, n_final: int, seed: int, rounds: int = 0,
          eps: float = 0.01, max_iter: int = 100, nthreads: int = 0, search_mode: int = SEARCH_PLAIN) -> dict:
    """rounds: boosting rounds (0: 8 for CMC, 64 for CMC_ADA)."""
    if rounds <= 0:
        rounds = ADA_ROUNDS if method == CMC_ADA else 8
    h = _SpecHolder(spec)
    rules = np.zeros((h.n_dates + 1, row_width(spec, method)))
    res = np.zeros(8)
    _check(lib().orc_price(h.ptr, method, N, n, n_final, seed, rounds, eps, max_iter, search_mode, nthreads,
                           _dp(rules), _dp(res)), "price")
    return {"price": res[0], "variance": res[1], "std_err": res[2], "ci95": res[3],
            "inner_path_steps": int(res[4]), "final_path_steps": int(res[5]),
            "iz_unconverged": int(res[6]), "iz_iterations": int(res[7]), "rules": rules}
