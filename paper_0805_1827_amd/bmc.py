"""ctypes binding of libbmc.so (the gfx950 nested continuation-value Monte Carlo).

Argument marshalling only: every computation runs in the HIP library.  Device
arrays are torch CUDA (HIP) tensors; the context issues work on the torch
stream current at creation.  Function names follow include/bmc.h.
Importing this module fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import sys
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libbmc.so"

OK, EINVAL, ENOTSPD, ENOMEM, EDEVICE, EUNSUPPORTED, ENOCONV, EBUSY, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7, -8
PUT_BASKET, CALL_MAX, PUT_GEO, CALL_MIN = 0, 1, 2, 3
SEARCH_PLAIN, SEARCH_SECANT = 0, 1
CMC, IZ, CMC_ADA = 0, 1, 2
FP64, FP32, FP32_KAHAN = 0, 1, 2
STREAM_OUTER, STREAM_INNER, STREAM_FINAL = 1, 2, 3
D_MAX, NT_MAX = 64, 512

# every symbol include/bmc.h declares
SYMBOLS = [
    "bmc_version", "bmc_last_error", "bmc_ctx_create", "bmc_ctx_destroy", "bmc_sync", "bmc_price",
    "bmc_rules_create", "bmc_rules_destroy", "bmc_rules_width", "bmc_rules_set", "bmc_rules_get",
    "bmc_rules_export", "bmc_rules_import", "bmc_sample_points", "bmc_estimate_continuation",
    "bmc_fit_rule", "bmc_iz_search", "bmc_final_price", "bmc_philox", "bmc_normals", "bmc_price_batch",
    "bmc_tuning_set", "bmc_tuning_get", "bmc_server_create", "bmc_server_destroy", "bmc_server_submit",
    "bmc_server_poll", "bmc_server_wait", "bmc_server_cancel", "bmc_server_stats_get", "bmc_ctx_set_graphs",
    "bmc_ctx_graph_stats",
    "bmc_autotune", "bmc_iz_regions", "bmc_estimate_continuation_noalloc",
]


class BmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"bmc status {status}: {message}")
        self.status = status


class bmc_spec(C.Structure):
    _fields_ = [("d", C.c_int32), ("S0", C.POINTER(C.c_double)), ("delta", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("K", C.c_double), ("r", C.c_double), ("T", C.c_double),
                ("n_dates", C.c_int32), ("dates", C.POINTER(C.c_double)), ("payoff", C.c_int32)]


class bmc_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("N", C.c_int64), ("n", C.c_int64),
                ("n_final", C.c_int64), ("seed", C.c_uint64), ("cls_rounds", C.c_int32),
                ("iz_max_iter", C.c_int32), ("iz_eps", C.c_double), ("iz_search", C.c_int32)]


class bmc_result(C.Structure):
    _fields_ = [("price", C.c_double), ("variance", C.c_double), ("std_err", C.c_double),
                ("ci95", C.c_double), ("inner_path_steps", C.c_int64),
                ("final_path_steps", C.c_int64), ("iz_unconverged", C.c_int64),
                ("iz_iterations", C.c_int64), ("seconds", C.c_double),
                ("calc_seconds", C.c_double), ("fit_seconds", C.c_double),
                ("final_seconds", C.c_double), ("refine_seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class bmc_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_inflight", C.c_int32), ("rule_cache", C.c_int32)]


class bmc_server_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "rejected", "completed", "failed", "cache_hits",
                                          "cache_misses", "cached_rules", "rounds", "inner_path_steps",
                                          "final_path_steps", "queued", "inflight", "hbm_in_use",
                                          "hbm_peak")] + [("busy_seconds", C.c_double), ("canceled", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Loads libbmc.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0805_1827_amd.build` "
                          "(or __graft_entry__.build())")
    L = C.CDLL(str(LIB_PATH))
    vp, dp, u32p, i32p, i64p = C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p
    sp = C.POINTER(bmc_spec)
    L.bmc_version.restype = C.c_int32
    L.bmc_last_error.restype = C.c_char_p
    L.bmc_ctx_create.argtypes = [C.c_int32, vp, C.POINTER(vp)]
    L.bmc_ctx_destroy.argtypes = [vp]
    L.bmc_ctx_destroy.restype = None
    L.bmc_sync.argtypes = [vp]
    L.bmc_price.argtypes = [vp, sp, C.POINTER(bmc_opts), C.POINTER(vp), C.POINTER(bmc_result)]
    L.bmc_price_batch.argtypes = [vp, C.c_int32, sp, C.POINTER(bmc_opts), C.POINTER(vp), C.POINTER(bmc_result)]
    L.bmc_tuning_set.argtypes = [vp, C.c_int32, C.c_int32, C.c_int64, C.c_int32]
    L.bmc_tuning_get.argtypes = [vp, C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.POINTER(C.c_int32)]
    L.bmc_autotune.argtypes = [vp, sp, C.c_int32, C.c_int64, C.c_int64, C.POINTER(C.c_int32)]
    L.bmc_ctx_set_graphs.argtypes = [vp, C.c_int32]
    L.bmc_ctx_graph_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.bmc_server_create.argtypes = [vp, C.POINTER(bmc_server_opts), C.POINTER(vp)]
    L.bmc_server_destroy.argtypes = [vp]
    L.bmc_server_destroy.restype = None
    L.bmc_server_submit.argtypes = [vp, sp, C.POINTER(bmc_opts), C.POINTER(C.c_uint64)]
    L.bmc_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(bmc_result)]
    L.bmc_server_cancel.argtypes = [vp, C.c_uint64]
    L.bmc_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(bmc_result)]
    L.bmc_server_stats_get.argtypes = [vp, C.POINTER(bmc_server_stats)]
    L.bmc_rules_create.argtypes = [vp, sp, C.c_int32, C.POINTER(vp)]
    L.bmc_rules_destroy.argtypes = [vp]
    L.bmc_rules_destroy.restype = None
    L.bmc_rules_width.argtypes = [vp]
    L.bmc_rules_width.restype = C.c_int32
    L.bmc_rules_set.argtypes = [vp, C.c_int32, dp]
    L.bmc_rules_get.argtypes = [vp, C.c_int32, dp]
    L.bmc_rules_export.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.bmc_rules_import.argtypes = [vp, vp, C.c_size_t, C.POINTER(vp)]
    L.bmc_iz_regions.argtypes = [sp]
    L.bmc_iz_regions.restype = C.c_int32
    L.bmc_sample_points.argtypes = [vp, sp, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, vp]
    L.bmc_estimate_continuation.argtypes = [vp, sp, vp, C.c_int32, vp, C.c_int64, C.c_int64, C.c_uint64,
                                            C.c_int32, vp, vp, vp]
    L.bmc_estimate_continuation_noalloc.argtypes = [vp, sp, vp, C.c_int32, vp, C.c_int64, C.c_int64,
                                                    C.c_uint64, C.c_int32, vp, vp, vp]
    L.bmc_fit_rule.argtypes = [vp, sp, vp, C.c_int32, C.c_int32, vp, vp, C.c_int64, C.c_int32]
    L.bmc_iz_search.argtypes = [vp, sp, vp, C.c_int32, C.c_int32, vp, C.c_int64, C.c_int64, C.c_uint64,
                                C.c_int32, C.c_double, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_int64)]
    L.bmc_final_price.argtypes = [vp, sp, vp, C.c_int64, C.c_uint64, C.c_int32, C.POINTER(bmc_result)]
    L.bmc_philox.argtypes = [vp, C.c_uint32, C.c_uint32, vp, C.c_int64, vp]
    L.bmc_normals.argtypes = [vp, C.c_uint32, C.c_uint32, vp, C.c_int64, C.c_int32, vp]
    for name in SYMBOLS:
        fn = getattr(L, name)
        if fn.restype is C.c_int:       # default: statuses are int32
            fn.restype = C.c_int32
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise BmcError(status, load().bmc_last_error().decode(errors="replace"))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Spec:
    """Marshals an option spec (attributes d, S0, delta, sigma, rho, K, r, T,
    dates, payoff) into bmc_spec, keeping the host arrays alive."""

    def __init__(self, spec):
        d = int(spec.d)
        self.d = d
        self.S0 = np.ascontiguousarray(spec.S0, dtype=np.float64).reshape(d)
        self.delta = np.ascontiguousarray(spec.delta, dtype=np.float64).reshape(d)
        self.sigma = np.ascontiguousarray(spec.sigma, dtype=np.float64).reshape(d)
        self.rho = np.ascontiguousarray(spec.rho, dtype=np.float64).reshape(d * d)
        self.dates = np.ascontiguousarray(spec.dates, dtype=np.float64)
        self.n_dates = len(self.dates)
        self.c = bmc_spec(d, _dp(self.S0), _dp(self.delta), _dp(self.sigma), _dp(self.rho),
                          float(spec.K), float(spec.r), float(spec.T), self.n_dates, _dp(self.dates),
                          int(spec.payoff))

    @property
    def ptr(self):
        return C.byref(self.c)


def as_spec(spec) -> Spec:
    return spec if isinstance(spec, Spec) else Spec(spec)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Context:
    """A bmc_ctx bound to a device and a HIP stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        L = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = C.c_void_p()
        _check(L.bmc_ctx_create(device, C.c_void_p(int(stream.cuda_stream)), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().bmc_ctx_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be torn down:
        # a handle still open then is left to the process exit (close()
        # explicitly to release it earlier).
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Rules:
    """Owned bmc_rules handle."""

    def __init__(self, handle: C.c_void_p, n_dates: int):
        self.h = handle
        self.n_dates = n_dates

    @property
    def width(self) -> int:
        return int(load().bmc_rules_width(self.h))

    def close(self):
        if getattr(self, "h", None):
            load().bmc_rules_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be torn down:
        # a handle still open then is left to the process exit (close()
        # explicitly to release it earlier).
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def bmc_ctx_set_graphs(ctx: Context, enable: bool) -> None:
    _check(load().bmc_ctx_set_graphs(ctx.h, 1 if enable else 0))


def bmc_ctx_graph_stats(ctx: Context) -> tuple:
    c, r = C.c_int64(0), C.c_int64(0)
    _check(load().bmc_ctx_graph_stats(ctx.h, C.byref(c), C.byref(r)))
    return int(c.value), int(r.value)


def bmc_version() -> int:
    return int(load().bmc_version())


def bmc_sync(ctx: Context):
    _check(load().bmc_sync(ctx.h))


def bmc_price(ctx: Context, spec, method: int = CMC, precision: int = FP64, N: int = 500, n: int = 500,
              n_final: int = 100000, seed: int = 1, cls_rounds: int = 0, iz_max_iter: int = 0,
              iz_eps: float = 0.0, want_rules: bool = False, iz_search: int = SEARCH_PLAIN):
    s = as_spec(spec)
    o = bmc_opts(method, precision, N, n, n_final, seed, cls_rounds, iz_max_iter, iz_eps, iz_search)
    res = bmc_result()
    rh = C.c_void_p()
    _check(load().bmc_price(ctx.h, s.ptr, C.byref(o), C.byref(rh) if want_rules else None, C.byref(res)))
    out = res.as_dict()
    if want_rules:
        return out, Rules(rh, s.n_dates)
    return out


def bmc_price_batch(ctx: Context, specs, opts, want_rules: bool = False):
    """Prices many options in shared launches.  specs: option specs; opts:
    one dict per option with keys of bmc_price (method, precision, N, n,
    n_final, seed, cls_rounds).  Returns the list of result dicts (and the
    list of Rules with want_rules)."""
    ss = [as_spec(s) for s in specs]
    count = len(ss)
    if count != len(opts):
        raise ValueError("specs and opts differ in length")
    sarr = (bmc_spec * count)(*[s.c for s in ss])
    oarr = (bmc_opts * count)()
    for i, o in enumerate(opts):
        oarr[i] = bmc_opts(o.get("method", CMC), o.get("precision", FP64), o.get("N", 500), o.get("n", 500),
                           o.get("n_final", 100000), o.get("seed", 1), o.get("cls_rounds", 0),
                           o.get("iz_max_iter", 0), o.get("iz_eps", 0.0), o.get("iz_search", SEARCH_PLAIN))
    res = (bmc_result * count)()
    rh = (C.c_void_p * count)()
    _check(load().bmc_price_batch(ctx.h, count, sarr, oarr, rh if want_rules else None, res))
    out = [r.as_dict() for r in res]
    if want_rules:
        return out, [Rules(C.c_void_p(rh[i]), ss[i].n_dates) for i in range(count)]
    return out


def bmc_tuning_set(ctx: Context, d: int = 0, precision: int = -1, n: int = 0, ppt: int = 0) -> None:
    _check(load().bmc_tuning_set(ctx.h, d, precision, n, ppt))


def bmc_tuning_get(ctx: Context, d: int, precision: int, N: int, n: int) -> int:
    v = C.c_int32(0)
    _check(load().bmc_tuning_get(ctx.h, d, precision, N, n, C.byref(v)))
    return int(v.value)


class Server:
    """A bmc_server: continuous-batching request loop on ctx's device."""

    def __init__(self, ctx: Context, hbm_budget: int = 0, max_inflight: int = 0, rule_cache: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        o = bmc_server_opts(hbm_budget, max_inflight, rule_cache)
        _check(load().bmc_server_create(ctx.h, C.byref(o), C.byref(h)))
        self.h = h

    def submit(self, spec, method: int = CMC, precision: int = FP64, N: int = 256, n: int = 1024,
               n_final: int = 16384, seed: int = 1, cls_rounds: int = 0) -> int:
        s = as_spec(spec)
        o = bmc_opts(method, precision, N, n, n_final, seed, cls_rounds, 0, 0.0)
        t = C.c_uint64(0)
        _check(load().bmc_server_submit(self.h, s.ptr, C.byref(o), C.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        """The result dict, or None while the request is pending."""
        res = bmc_result()
        st = load().bmc_server_poll(self.h, ticket, C.byref(res))
        if st == EBUSY:
            return None
        _check(st)
        return res.as_dict()

    def wait(self, ticket: int, timeout: float = -1.0):
        res = bmc_result()
        st = load().bmc_server_wait(self.h, ticket, timeout, C.byref(res))
        if st == EBUSY:
            return None
        _check(st)
        return res.as_dict()

    def cancel(self, ticket: int) -> None:
        """Cancels a queued or running request (BmcError EINVAL if it has
        already finished); its poll and wait then raise ECANCELED."""
        _check(load().bmc_server_cancel(self.h, ticket))

    def stats(self) -> dict:
        s = bmc_server_stats()
        _check(load().bmc_server_stats_get(self.h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "h", None):
            load().bmc_server_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be torn down:
        # a handle still open then is left to the process exit (close()
        # explicitly to release it earlier).
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def bmc_autotune(ctx: Context, spec, precision: int, N: int, n: int) -> int:
    s = as_spec(spec)
    v = C.c_int32(0)
    _check(load().bmc_autotune(ctx.h, s.ptr, precision, N, n, C.byref(v)))
    return int(v.value)


def bmc_rules_create(ctx: Context, spec, method: int) -> Rules:
    s = as_spec(spec)
    h = C.c_void_p()
    _check(load().bmc_rules_create(ctx.h, s.ptr, method, C.byref(h)))
    return Rules(h, s.n_dates)


def bmc_rules_set(rules: Rules, date: int, w) -> None:
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (rules.width,):
        raise ValueError(f"rule row must have {rules.width} entries")
    _check(load().bmc_rules_set(rules.h, date, _dp(w)))


def bmc_rules_width(rules: Rules) -> int:
    return int(load().bmc_rules_width(rules.h))


def bmc_rules_get(rules: Rules, date: int) -> np.ndarray:
    w = np.zeros(rules.width)
    _check(load().bmc_rules_get(rules.h, date, _dp(w)))
    return w


def rules_table(rules: Rules) -> np.ndarray:
    """All rows (0..N_T) as a host array."""
    return np.stack([bmc_rules_get(rules, k) for k in range(rules.n_dates + 1)])


def set_rules_table(rules: Rules, table: np.ndarray) -> None:
    for k in range(1, rules.n_dates):
        bmc_rules_set(rules, k, table[k])


def bmc_rules_export(rules: Rules) -> bytes:
    L = load()
    n = C.c_size_t(0)
    _check(L.bmc_rules_export(rules.h, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(L.bmc_rules_export(rules.h, buf, C.byref(n)))
    return buf.raw[: n.value]


def bmc_rules_import(ctx: Context, data: bytes) -> Rules:
    h = C.c_void_p()
    buf = C.create_string_buffer(data, len(data))
    _check(load().bmc_rules_import(ctx.h, buf, len(data), C.byref(h)))
    n_dates = int(np.frombuffer(data[:32], dtype=np.int32)[4])
    return Rules(h, n_dates)


def _dev_zeros(shape, dtype, ctx: Context):
    import torch
    return torch.zeros(shape, dtype=dtype, device=f"cuda:{ctx.device}")


def bmc_iz_regions(spec) -> int:
    return int(load().bmc_iz_regions(as_spec(spec).ptr))


def bmc_sample_points(ctx: Context, spec, method: int, date: int, N: int, seed: int, region: int = 0):
    import torch
    s = as_spec(spec)
    x = _dev_zeros((s.d, N), torch.float64, ctx)
    _check(load().bmc_sample_points(ctx.h, s.ptr, method, date, region, N, seed, _ptr(x)))
    return x


def bmc_estimate_continuation(ctx: Context, spec, rules: Rules, date: int, x, n: int, seed: int,
                              precision: int = FP64):
    import torch
    s = as_spec(spec)
    x = x.contiguous()
    N = int(x.shape[1])
    cont = _dev_zeros(N, torch.float64, ctx)
    se = _dev_zeros(N, torch.float64, ctx)
    steps = _dev_zeros(N, torch.int64, ctx)
    _check(load().bmc_estimate_continuation(ctx.h, s.ptr, rules.h, date, _ptr(x), N, n, seed, precision,
                                            _ptr(cont), _ptr(se), _ptr(steps)))
    return cont, se, steps


def bmc_estimate_continuation_noalloc(ctx: Context, spec, rules: Rules, date: int, x, cont, std_err, steps,
                                      n: int, seed: int, precision: int = FP64) -> None:
    """bmc_estimate_continuation into caller-made device tensors cont [N],
    std_err [N] (float64) and steps [N] (int64, or None), with no device
    allocation in the call."""
    s = as_spec(spec)
    N = int(x.shape[1])
    _check(load().bmc_estimate_continuation_noalloc(ctx.h, s.ptr, rules.h, date, _ptr(x), N, n, seed, precision,
                                                    _ptr(cont), _ptr(std_err), _ptr(steps)))


def bmc_fit_rule(ctx: Context, spec, rules: Rules, date: int, x, values=None, rounds: int = 0,
                 region: int = 0) -> None:
    s = as_spec(spec)
    x = x.contiguous()
    _check(load().bmc_fit_rule(ctx.h, s.ptr, rules.h, date, region, _ptr(x),
                               _ptr(values.contiguous()) if values is not None else None,
                               int(x.shape[1]), rounds))


def bmc_iz_search(ctx: Context, spec, rules: Rules, date: int, x, n: int, seed: int,
                  precision: int = FP64, eps: float = 0.01, max_iter: int = 100, region: int = 0,
                  mode: int = 0):
    import torch
    s = as_spec(spec)
    x = x.contiguous()
    J = int(x.shape[1])
    s_out = _dev_zeros(J, torch.float64, ctx)
    iters = _dev_zeros(J, torch.int32, ctx)
    steps = C.c_int64(0)
    _check(load().bmc_iz_search(ctx.h, s.ptr, rules.h, date, region, _ptr(x), J, n, seed, precision, eps,
                                max_iter, mode, _ptr(s_out), _ptr(iters), C.byref(steps)))
    return s_out, iters, int(steps.value)


def bmc_final_price(ctx: Context, spec, rules: Rules, n_final: int, seed: int,
                    precision: int = FP64) -> dict:
    s = as_spec(spec)
    res = bmc_result()
    _check(load().bmc_final_price(ctx.h, s.ptr, rules.h, n_final, seed, precision, C.byref(res)))
    return res.as_dict()


def bmc_philox(ctx: Context, k0: int, k1: int, ctr):
    """ctr: int32/uint32-valued torch tensor [M, 4] on the device."""
    import torch
    ctr = ctr.contiguous()
    M = int(ctr.shape[0])
    out = _dev_zeros((M, 4), torch.int32, ctx)
    _check(load().bmc_philox(ctx.h, k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF, _ptr(ctr), M, _ptr(out)))
    return out


def bmc_normals(ctx: Context, k0: int, k1: int, ctr, precision: int = FP64):
    import torch
    ctr = ctr.contiguous()
    M = int(ctr.shape[0])
    out = _dev_zeros((M, 4), torch.float64, ctx)
    _check(load().bmc_normals(ctx.h, k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF, _ptr(ctr), M, precision, _ptr(out)))
    return out
