#!/usr/bin/env python3
"""Benchmark of the nested continuation-value Monte Carlo on one MI355X.

One step = one whole pricing pass of the 5-asset geometric-average Bermudan
put (S0_i = K = 100, r = 0.05, sigma_i = 0.2, pairwise rho = 0.3, T = 1,
10 dates) by the CMC pricer with N = 4096 training points per date,
n = 4096 inner paths per point and 1e6 final-pricing paths: sample points,
continuation estimates (the hot kernel), labels and boosting fit at every
date, then final pricing.  Inputs are synthetic and generated on the device.

Prints ONE JSON line: inner path-steps per second of the FP32 form (float
stepping, double accumulation), with the plain FP64 form, prices and their
distance in standard errors, per-step latency percentiles, the hot kernel's
VALU roofline and the CPU oracle's rate on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

# MI355X VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, in FP32-FMA
# issue slots per second (= 78.6 TFLOP/s of unpacked FP32 FMA).
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9

# Issue cost of one lane-operation of each class, in FP32-FMA slots, measured
# on gfx950 by paper_0805_1827_amd/calib/valu_rates.hip (8 independent chains
# of one instruction class per lane, 8 waves per SIMD on all 256 CUs):
# 2-input integer/logic 0.6, three-input xor (v_bitop3_b32) 0.64, v_mad_u64_u32
# (32x32->64 multiply) 1.15, FP32 transcendental (v_log/v_exp/v_sin/v_cos/v_sqrt)
# 1.9, FP32 FMA/add/mul 1.0.
COST = {"int": 0.6, "xor3": 0.64, "mul64": 1.15, "trans": 1.9, "f32": 1.0}


# FP32 dense matrix-core peak of MI355X (TFLOP/s).
PEAK_MFMA_F32 = 157.3e12


def uses_mfma(d: int) -> bool:
    """FP32 kernels for d >= 25 run the correlation on the matrix cores."""
    return d >= 25


def mfma_flops_per_step(d: int) -> float:
    """Algorithmic flops of the correlation product A (s z) per path-step."""
    return float(d * (d + 1))


def philox_block_slots(cost=None) -> float:
    """One Philox4x32-10 block: 10 rounds of 2 wide multiplies and 2
    three-input xors (high half ^ counter word ^ key; the key schedule is
    uniform across the wavefront, i.e. scalar)."""
    c = cost or COST
    return 10 * (2 * c["mul64"] + 2 * c["xor3"])


def bm_pair_slots_fp32() -> float:
    """One Box-Muller pair in FP32: 2 word->float conversions and 2 scalings,
    log2, a multiply, sqrt, sin, cos, 2 multiplies."""
    c = COST
    return 4 * c["f32"] + c["trans"] + c["f32"] + c["trans"] + 2 * c["trans"] + 2 * c["f32"]


def rng_units(d: int, layout: bool) -> tuple[float, float]:
    """Philox blocks and Box-Muller pairs per path-step: d/4 and d/2 for the
    d random words a path-step consumes (the algorithmic count); with layout,
    the ceil(d/4) blocks and ceil(d/2) pairs the kernel draws (it spends
    whole blocks per step, so that each step's counter is addressable on its
    own)."""
    if layout:
        return float((d + 3) // 4), float((d + 1) // 2)
    return d / 4.0, d / 2.0


def slots_per_step_fp32(d: int, payoff: int, method: int, layout: bool = False) -> float:
    """Algorithmic VALU issue slots of one inner path-step (FP32 form).

    Random numbers: d/4 Philox blocks and d/2 Box-Muller pairs (rng_units).
    Step: sqrt(dt) z (d), the lower-triangular correlation d(d+1)/2 FMAs, the
    drift d FMAs.  Payoff: max-call / geometric one exp plus d+3 simple ops;
    arithmetic basket d exps plus d+3.  CMC rule: d subtractions, 2d FMAs, 4
    more for g and the comparison; I&Z boundary: q + q(q+1)/2 FMAs and
    q(q+1)/2 products (q = d-1).  Per path (amortised over its steps and left
    out): the FP64 accumulation of the payoff.  For d > 8 the correlation
    runs on the matrix cores and is left out of the VALU count (reported as
    matrix-core flops, mfma_flops_per_step).
    """
    blocks, pairs = rng_units(d, layout)
    philox = blocks * philox_block_slots()
    bm = pairs * bm_pair_slots_fp32()
    corr = 0 if uses_mfma(d) else d * (d + 1) / 2
    step = (d + corr + d) * COST["f32"]
    if payoff == 0:
        pay = d * COST["trans"] + (d + 3) * COST["f32"]
    else:
        pay = COST["trans"] + (d + 3) * COST["f32"]
    if method == 0:
        rule = (3 * d + 4) * COST["f32"]
    else:
        q = d - 1
        rule = (1 + q + q * (q + 1)) * COST["f32"]
    return philox + bm + step + pay + rule


# FP64 form: issue cost of each operation class in FP64-FMA slots (one FP64
# FMA per lane; MI355X issues 256 CUs x 4 SIMDs x 16 lanes of them per clock,
# 78.6 TFLOP/s at 2.4 GHz).  Integer classes are the FP32 calibration's
# figures rescaled by the FP64 FMA's own cost (1.112 FP32 slots); the normal
# map's ln u, sin/cos(2 pi u) and sqrt are the kernel's own functions
# (log_u32, sincos_2pi_u32, sqrt_pos) and exp the device library's, net
# costs measured on gfx950 by paper_0805_1827_amd/calib/valu_rates.hip.
COST64 = {"f64": 1.0, "int": 0.606 / 1.112, "xor3": 0.636 / 1.112, "mul64": 1.145 / 1.112,
          "log": 31.6, "exp": 18.5, "sqrt": 13.5, "sincospi": 30.6, "cvt_pair": 1.5}


def slots_per_step_fp64(d: int, payoff: int, method: int, layout: bool = False) -> float:
    """Algorithmic VALU issue slots of one inner path-step of the FP64 form,
    in FP64-FMA slots: the FP32 form's operation list with FP64 arithmetic,
    the library's own FP64 normal map (log of a word, sine and cosine of a
    turn fraction, square root; measured net of their word conversions) and
    the device library's FP64 exp."""
    c = COST64
    blocks, pairs = rng_units(d, layout)
    philox = blocks * philox_block_slots(c)
    # ln u_a (with its word conversion), -2x, sqrt, sin and cos of 2 pi u_b, 2 products
    bm = pairs * (c["log"] + 1 + c["sqrt"] + c["sincospi"] + 2)
    step = d + d * (d + 1) / 2 + d
    if payoff == 0:
        pay = d * c["exp"] + (d + 3)
    else:
        pay = c["exp"] + (d + 3)
    if method == 0:
        rule = 3 * d + 4
    else:
        q = d - 1
        rule = 1 + q + q * (q + 1)
    return philox + bm + step + pay + rule


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=float), q))


TRAFFIC_FILE = ROOT / "profiles" / "k_cont_geo5_fp32_traffic.json"
KERNEL_SOURCES = ("cont_kernel.hpp", "device.hpp", "cont_args.hpp")


def measured_traffic():
    """HBM bytes per date launch of the continuation kernel from the committed
    FETCH_SIZE / WRITE_SIZE runs (scaled by a copy kernel), or None when the
    kernel's sources have changed since those counters were taken."""
    import hashlib
    if not TRAFFIC_FILE.exists():
        return None
    rec = json.loads(TRAFFIC_FILE.read_text())
    csrc = ROOT / "paper_0805_1827_amd" / "csrc"
    h = hashlib.sha256(b"".join((csrc / f).read_bytes() for f in KERNEL_SOURCES)).hexdigest()
    return rec["hbm_bytes_per_launch"] if rec.get("src_sha256") == h else None


def cpu_threads() -> int:
    """Host threads of the oracle baseline: every core of the affinity mask,
    capped by OMP_NUM_THREADS when the machine sets it (the CPU share of one
    GPU on a shared host)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(spec, N, n, seed, target_seconds: float) -> dict:
    """The FP64 oracle timed on this host: the inner-path continuation
    estimates of a subset of the CMC training points, at every date, with the
    same draws as the GPU run, under exercise rules the oracle learns itself
    (its own CMC pricer at N = n = 256)."""
    from oracle import oracle as orc
    threads = cpu_threads()
    rules = orc.price(spec, orc.CMC, 256, 256, 2, seed, nthreads=threads)["rules"]
    pts = {m: orc.points_cmc(spec, m, N, seed) for m in range(1, spec.n_dates)}

    def run(k):
        steps = 0
        t0 = time.perf_counter()
        for m in range(1, spec.n_dates):
            ids = np.arange(k, dtype=np.uint32)
            r = orc.continuation(spec, orc.CMC, rules, m, pts[m][:, :k], n, seed, nthreads=threads, ids=ids)
            steps += int(r["steps"].sum())
        return steps, time.perf_counter() - t0

    k = max(threads, 16)
    steps, dt = run(k)
    if dt < target_seconds:
        k = int(min(N, max(k, k * target_seconds / max(dt, 1e-3))))
        steps, dt = run(k)
    return {"value": steps / dt, "unit": "path-steps/s", "cores": threads,
            "affinity_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"continuation estimates of {k} of the {N} training points at each of the "
                      f"{spec.n_dates - 1} dates, n = {n} inner paths, FP64, rules learned by the oracle "
                      f"at N = n = 256 ({steps} path-steps in {dt:.1f} s)"}


def batch_form(ctx, bmc, inputs, count: int, N: int, n_final: int) -> dict:
    """The uneven-instance batch (count options: d in 1..20, 4..50 dates, n in
    {1k, 4k, 16k}, Wishart correlations, three payoffs, seeds 0..count-1),
    priced by bmc_price_batch in FP32 and FP64, with the FP32 slot roofline
    over the batch's executed path-steps and the FP32-FP64 price distance."""
    import torch
    specs = inputs.uneven_batch(count)

    def opts(prec):
        return [dict(method=bmc.CMC, precision=prec, N=N, n=s.meta["n"], n_final=n_final, seed=s.meta["seed"])
                for s in specs]

    bmc.bmc_price_batch(ctx, specs[:4], opts(bmc.FP32)[:4])   # warm-up (module load, buffers)
    out = {}
    rules64 = None
    for name, prec in (("fp32", bmc.FP32), ("fp64", bmc.FP64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if prec == bmc.FP64:
            res, rules64 = bmc.bmc_price_batch(ctx, specs, opts(prec), want_rules=True)
        else:
            res = bmc.bmc_price_batch(ctx, specs, opts(prec))
        dt = time.perf_counter() - t0
        out[name] = (res, dt)
    # FP32 final pricing under the FP64 rules (same rules, precision alone)
    same = []
    for s, rl, r in zip(specs, rules64, out["fp64"][0]):
        f = bmc.bmc_final_price(ctx, s, rl, n_final, s.meta["seed"], bmc.FP32)
        same.append(abs(f["price"] - r["price"]) / r["std_err"])
        rl.close()
    same = np.array(same)
    # the same sweep captured as a HIP graph, then replayed
    gctx = bmc.Context(0)
    try:
        bmc.bmc_ctx_set_graphs(gctx, True)
        bmc.bmc_price_batch(gctx, specs, opts(bmc.FP32))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rg = bmc.bmc_price_batch(gctx, specs, opts(bmc.FP32))
        t_graph = time.perf_counter() - t0
        graph_stats = bmc.bmc_ctx_graph_stats(gctx)
    finally:
        gctx.close()
    r32, t32 = out["fp32"]
    r64, t64 = out["fp64"]
    assert all(a["price"] == b["price"] for a, b in zip(rg, r32)), "graph replay differs from direct launches"
    steps32 = sum(r["inner_path_steps"] for r in r32)
    steps64 = sum(r["inner_path_steps"] for r in r64)
    slots = sum(slots_per_step_fp32(s.d, s.payoff, bmc.CMC) * r["inner_path_steps"] for s, r in zip(specs, r32))
    mflops = sum(mfma_flops_per_step(s.d) * r["inner_path_steps"] for s, r in zip(specs, r32) if uses_mfma(s.d))
    calc = r32[0]["calc_seconds"]
    dist = np.array([abs(a["price"] - b["price"]) / b["std_err"] for a, b in zip(r32, r64)])
    return {"workload": f"{count} uneven options (d 1-20, 4-50 dates, n in 1k/4k/16k, Wishart rho, "
                        f"3 payoffs, seeds 0-{count - 1}), CMC, N={N}, n_final={n_final}",
            "fp32": {"value": steps32 / t32, "seconds": t32, "inner_path_steps": steps32,
                     "phase_s": {"calc": calc, "fit": r32[0]["fit_seconds"], "final": r32[0]["final_seconds"]}},
            "fp64": {"value": steps64 / t64, "seconds": t64, "inner_path_steps": steps64},
            "fp32_graph_replay": {"value": steps32 / t_graph, "seconds": t_graph,
                                  "captures_replays": list(graph_stats)},
            "unit": "path-steps/s",
            "fp32_valu_slot_frac_of_peak": slots / calc / PEAK_SLOTS,
            # matrix-core correlation only from d = 25 on (none in this mix)
            **({"fp32_mfma_tflops": mflops / calc / 1e12, "fp32_mfma_frac_of_peak": mflops / calc / PEAK_MFMA_F32}
               if mflops > 0 else {}),
            "fp32_vs_fp64_price_in_std_err": {"median": float(np.median(dist)), "max": float(dist.max()),
                                              "frac_within_0.1": float(np.mean(dist <= 0.1))},
            "fp32_final_under_fp64_rules_in_std_err": {"median": float(np.median(same)), "max": float(same.max()),
                                                       "frac_within_0.1": float(np.mean(same <= 0.1))}}


def serving_form(ctx, bmc, inputs, duration: float, rate: float, precision: int, N: int = 256,
                 seed: int = 7) -> dict:
    """The serving loop under Poisson arrivals: requests draw from a seeded
    catalogue of 64 specs (d in 1..40, 4..50 dates, n in {2k, 8k, 32k},
    Wishart correlations, three payoffs), learn with N points on a rule-cache
    miss and price with n_final = 16 n.  Latency = completion - submission."""
    cat = inputs.serving_catalogue(64)
    rng = np.random.default_rng(seed)
    arrivals = inputs.poisson_arrivals(rate, duration, seed)
    picks = rng.integers(0, len(cat), size=len(arrivals))
    srv = bmc.Server(ctx, hbm_budget=16 << 30)
    tickets = []
    t0 = time.perf_counter()
    try:
        for t_arr, k in zip(arrivals, picks):
            now = time.perf_counter() - t0
            if t_arr > now:
                time.sleep(t_arr - now)
            s = cat[k]
            n = s.meta["n"]
            tickets.append(srv.submit(s, method=bmc.CMC, precision=precision, N=N, n=n, n_final=16 * n,
                                      seed=1000 + int(k)))
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    lat = np.array([r["seconds"] for r in res])
    # after the cold-cache learning burst: requests arriving in the last two thirds of the window
    late = lat[np.asarray(arrivals) >= duration / 3.0]
    steps = st["inner_path_steps"] + st["final_path_steps"]
    return {"requests": len(res), "offered_rate": len(res) / duration, "served_rate": len(res) / wall,
            "wall_s": wall, "cache_hit_rate": st["cache_hits"] / max(1, len(res)),
            "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99)),
                           "max": 1e3 * float(lat.max())},
            "latency_ms_last_two_thirds": {"p50": 1e3 * float(np.percentile(late, 50)),
                                           "p99": 1e3 * float(np.percentile(late, 99)),
                                           "max": 1e3 * float(late.max())} if late.size else None,
            "cache_misses": st["cache_misses"],
            "path_steps_per_s": steps / wall, "inner_path_steps": st["inner_path_steps"],
            "final_path_steps": st["final_path_steps"], "rounds": st["rounds"],
            "busy_frac": st["busy_seconds"] / wall, "hbm_peak_bytes": st["hbm_peak"]}


def saturation_form(ctx, bmc, inputs, precision: int, N: int = 256) -> dict:
    """Learning-bound rate: the 64 catalogue specs submitted at once, cold cache."""
    cat = inputs.serving_catalogue(64)
    srv = bmc.Server(ctx, hbm_budget=16 << 30)
    t0 = time.perf_counter()
    try:
        tickets = [srv.submit(s, method=bmc.CMC, precision=precision, N=N, n=s.meta["n"],
                              n_final=16 * s.meta["n"], seed=2000 + i) for i, s in enumerate(cat)]
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    steps = st["inner_path_steps"] + st["final_path_steps"]
    return {"requests": len(res), "requests_per_s": len(res) / wall, "wall_s": wall,
            "path_steps_per_s": steps / wall, "inner_path_steps": st["inner_path_steps"]}


# Binomial references of the max-call of Table 1 (d = 3, K = 100, r = 0.05,
# delta = 0.1, sigma = 0.2, rho = 0, T = 3, 9 dates) and the running times the
# paper reports for its I&Z pricer on 16 processors (Tables 2 and 3, S0 = 90).
IZ_BINOMIAL = {90: 11.29, 100: 18.69, 110: 27.58}
IZ_PAPER_MINUTES = {("J", 128): 4.6, ("J", 256): 8.1, ("J", 1024): 29.5,
                    ("N1", 5000): 4.6, ("N1", 10000): 6.9, ("N1", 100000): 35.7}


def iz_form(ctx, bmc, inputs, reps: int = 3) -> dict:
    """I&Z on the three-asset max-call: the Table 1 prices (S0 = 90, 100, 110;
    J = 128 lattice points, N_1 = 5000 inner paths, N = 1e6 final paths) in
    both precisions, and the J and N_1 sweeps of Tables 2-3 at S0 = 90.  Each
    configuration is priced reps times (same seed); the median wall time is
    reported."""
    def one(S0, J, N1, prec, search=bmc.SEARCH_PLAIN):
        spec = inputs.max_call(3, float(S0))
        kw = dict(N=J, n=N1, n_final=1_000_000, seed=1, iz_search=search)
        bmc.bmc_price(ctx, spec, bmc.IZ, prec, **kw)   # warm
        runs = [bmc.bmc_price(ctx, spec, bmc.IZ, prec, **kw) for _ in range(reps)]
        r = runs[-1]
        wall = float(np.median([x["seconds"] for x in runs]))
        calc = float(np.median([x["calc_seconds"] for x in runs]))
        research = float(np.median([x["refine_seconds"] for x in runs]))
        return {"S0": S0, "J": J, "N1": N1, "price": r["price"], "std_err": r["std_err"],
                "error_vs_binomial": IZ_BINOMIAL[S0] - r["price"], "ms": 1e3 * wall, "calc_ms": 1e3 * calc,
                "near_tie_fp64_search_ms": 1e3 * research,
                "inner_path_steps": r["inner_path_steps"],
                "inner_path_steps_per_s": r["inner_path_steps"] / calc,
                "iterations_per_point": r["iz_iterations"] / (3 * (spec.n_dates - 1) * J),
                "unconverged": r["iz_unconverged"]}

    out = {"workload": "call on the max of 3 assets (Table 1 parameters), I&Z with 3 exercise regions, "
                       "eps = 0.01, seed 1",
           "table1_fp32": [one(S0, 128, 5000, bmc.FP32) for S0 in (90, 100, 110)],
           "table1_fp64": [one(S0, 128, 5000, bmc.FP64) for S0 in (90, 100, 110)],
           "table1_fp32_secant": [one(S0, 128, 5000, bmc.FP32, bmc.SEARCH_SECANT) for S0 in (90, 100, 110)]}
    sweep = []
    for key, J, N1 in (("J", 128, 5000), ("J", 256, 5000), ("J", 1024, 5000), ("N1", 128, 10000),
                       ("N1", 128, 100000)):
        row = one(90, J, N1, bmc.FP32)
        row["paper_minutes_16_procs"] = IZ_PAPER_MINUTES[(key, J if key == "J" else N1)]
        sweep.append(row)
    out["sweeps_fp32"] = sweep
    return out


def maxcall5_form(ctx, bmc, inputs) -> dict:
    """The five-asset max-call (K = 100, r = 0.05, delta = 0.1, sigma = 0.2,
    independent assets, T = 3, 9 dates; S0 = 90, 100, 110), CMC at
    N = n = 16384 with 1e6 final paths: FP32 stepping with compensated FP64
    sums beside the FP64 form on the same GPU, whose continuation estimates
    the tests hold to the oracle at 1e-10 relative."""
    rows = []
    for S0 in (90, 100, 110):
        spec = inputs.max_call(5, float(S0))
        kw = dict(N=16384, n=16384, n_final=1_000_000, seed=1)
        bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32_KAHAN, **kw)   # warm
        a = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32_KAHAN, **kw)
        b = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, **kw)
        rows.append({"S0": S0, "price_fp32_kahan": a["price"], "price_fp64": b["price"],
                     "std_err": b["std_err"], "fp32_error_in_std_err": abs(a["price"] - b["price"]) / b["std_err"],
                     "ms_fp32_kahan": 1e3 * a["seconds"], "ms_fp64": 1e3 * b["seconds"],
                     "inner_path_steps": a["inner_path_steps"],
                     "inner_path_steps_per_s_fp32_kahan": a["inner_path_steps"] / a["calc_seconds"],
                     "inner_path_steps_per_s_fp64": b["inner_path_steps"] / b["calc_seconds"],
                     "asset_steps_per_s_fp32_kahan": 5 * a["inner_path_steps"] / a["calc_seconds"],
                     "valu_frac_fp32_kahan": slots_per_step_fp32(5, spec.payoff, bmc.CMC) * a["inner_path_steps"]
                     / a["calc_seconds"] / PEAK_SLOTS,
                     "valu_frac_fp64": slots_per_step_fp64(5, spec.payoff, bmc.CMC) * b["inner_path_steps"]
                     / b["calc_seconds"] / PEAK_SLOTS})
    return {"workload": "call on the max of 5 independent assets, CMC, N=n=16384, 9 dates, 1e6 final paths, "
                        "seed 1", "runs": rows}


def mincall_form(ctx, bmc, inputs) -> dict:
    """Calls on the minimum of 2 and 3 independent assets (S0 = 100, K = 100,
    r = 0.05, delta = 0.1, sigma = 0.2, T = 3, 9 dates): I&Z with d exercise
    regions (J = 128, N_1 = 5000; plain and secant searches) and CMC
    (N = n = 4096), 1e6 final paths, FP32 beside FP64 on the same GPU."""
    rows = []
    for d in (2, 3):
        spec = inputs.min_call(d, 100.0)
        for name, method, kw in (
                ("iz_plain", bmc.IZ, dict(N=128, n=5000, iz_search=bmc.SEARCH_PLAIN)),
                ("iz_secant", bmc.IZ, dict(N=128, n=5000, iz_search=bmc.SEARCH_SECANT)),
                ("cmc", bmc.CMC, dict(N=4096, n=4096))):
            kw = dict(kw, n_final=1_000_000, seed=1)
            bmc.bmc_price(ctx, spec, method, bmc.FP32, **kw)   # warm
            a = bmc.bmc_price(ctx, spec, method, bmc.FP32, **kw)
            b = bmc.bmc_price(ctx, spec, method, bmc.FP64, **kw)
            rows.append({"d": d, "method": name, "price_fp32": a["price"], "price_fp64": b["price"],
                         "std_err": b["std_err"], "fp32_error_in_std_err": abs(a["price"] - b["price"]) / b["std_err"],
                         "ms_fp32": 1e3 * a["seconds"], "ms_fp64": 1e3 * b["seconds"],
                         "inner_path_steps_per_s_fp32": a["inner_path_steps"] / a["calc_seconds"],
                         "iz_iterations": a["iz_iterations"]})
    return {"workload": "call on the min of 2 and 3 independent assets, I&Z (J=128, N_1=5000) and CMC "
                        "(N=n=4096), 1e6 final paths, seed 1", "runs": rows}


# 2000-step CRR values of the Bermudan puts (10 dates, exercise at t_1..T):
# the 1-asset put (S0 = K = 100, r = 0.05, sigma = 0.2, T = 1) and the
# 5-asset geometric put reduced to one GBM (sigma_G^2 = 0.0176,
# delta_G = 0.0112); the oracle's pins recompute both.
CRR_PUT1 = 6.0334
CRR_GEO5 = 3.832
# Table 4: binomial values of the 3-asset max-call (S0 = 90, 100, 110) and the
# paper's CMC prices with 5000 training points, 500 inner paths, 1e6 final paths.
TABLE4_BINOMIAL = {90: 11.29, 100: 18.69, 110: 27.58}
TABLE4_PAPER_CMC = {90: 11.295, 100: 18.706, 110: 27.604}


def put1_form(ctx, bmc, inputs, reps: int = 3) -> dict:
    """The 1-asset Bermudan put (S0 = K = 100, r = 0.05, sigma = 0.2, T = 1,
    10 dates), CMC with N = n = 500, 1e5 final paths, seed 1, against the
    2000-step binomial tree."""
    spec = inputs.one_asset_put()
    kw = dict(N=500, n=500, n_final=100_000, seed=1)
    out = {"workload": "1-asset Bermudan put, CMC, N=n=500, 10 dates, 1e5 final paths, seed 1",
           "tree_price": CRR_PUT1}
    for name, prec in (("fp64", bmc.FP64), ("fp32", bmc.FP32)):
        bmc.bmc_price(ctx, spec, bmc.CMC, prec, **kw)
        runs = [bmc.bmc_price(ctx, spec, bmc.CMC, prec, **kw) for _ in range(reps)]
        r = runs[-1]
        out[name] = {"price": r["price"], "std_err": r["std_err"], "error_vs_tree": r["price"] - CRR_PUT1,
                     "error_in_std_err": (r["price"] - CRR_PUT1) / r["std_err"],
                     "ms": 1e3 * float(np.median([x["seconds"] for x in runs])),
                     "inner_path_steps": r["inner_path_steps"]}
    out["fp32_vs_fp64_in_std_err"] = abs(out["fp32"]["price"] - out["fp64"]["price"]) / out["fp64"]["std_err"]
    return out


def table4_form(ctx, bmc, inputs) -> dict:
    """Table 4's CMC setting: the 3-asset max-call (K = 100, r = 0.05,
    delta = 0.1, sigma = 0.2, independent, T = 3, 9 dates) with 5000 training
    points per date, 500 inner paths and 1e6 final paths, S0 = 90, 100, 110,
    in FP64 and FP32, against the binomial column."""
    rows = []
    for S0 in (90, 100, 110):
        spec = inputs.max_call(3, float(S0))
        kw = dict(N=5000, n=500, n_final=1_000_000, seed=1)
        bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32, **kw)
        a = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP32, **kw)
        b = bmc.bmc_price(ctx, spec, bmc.CMC, bmc.FP64, **kw)
        rows.append({"S0": S0, "price_fp64": b["price"], "ci95_fp64": b["ci95"],
                     "error_vs_binomial_fp64": TABLE4_BINOMIAL[S0] - b["price"],
                     "price_fp32": a["price"], "fp32_error_in_std_err": abs(a["price"] - b["price"]) / b["std_err"],
                     "paper_cmc_price": TABLE4_PAPER_CMC[S0], "binomial": TABLE4_BINOMIAL[S0],
                     "ms_fp32": 1e3 * a["seconds"], "ms_fp64": 1e3 * b["seconds"],
                     "inner_path_steps": a["inner_path_steps"]})
    return {"workload": "call on the max of 3 assets (Table 4), CMC, N=5000 training points, n=500 inner paths, "
                        "9 dates, 1e6 final paths, seed 1", "runs": rows}


def geo5_iz_form(ctx, bmc, inputs) -> dict:
    """The headline option (5-asset geometric put) priced by I&Z with
    J = N = 4096 lattice points per date and n = 4096 inner paths, 1e6 final
    paths, FP32 and FP64, against the reduced binomial tree."""
    spec = inputs.geometric_put5()
    kw = dict(N=4096, n=4096, n_final=1_000_000, seed=1)
    out = {"workload": "5-asset geometric-average Bermudan put, I&Z, J=n=4096, 10 dates, 1e6 final paths, seed 1",
           "tree_price": CRR_GEO5}
    for name, prec in (("fp32", bmc.FP32), ("fp64", bmc.FP64)):
        bmc.bmc_price(ctx, spec, bmc.IZ, prec, **kw)
        r = bmc.bmc_price(ctx, spec, bmc.IZ, prec, **kw)
        out[name] = {"price": r["price"], "std_err": r["std_err"], "error_vs_tree": r["price"] - CRR_GEO5,
                     "ms": 1e3 * r["seconds"], "calc_ms": 1e3 * r["calc_seconds"],
                     "inner_path_steps": r["inner_path_steps"],
                     "inner_path_steps_per_s": r["inner_path_steps"] / r["calc_seconds"],
                     "iterations_per_point": r["iz_iterations"] / ((spec.n_dates - 1) * 4096),
                     "unconverged": r["iz_unconverged"]}
    out["fp32_vs_fp64_in_std_err"] = abs(out["fp32"]["price"] - out["fp64"]["price"]) / out["fp64"]["std_err"]
    return out


_T0 = time.perf_counter()


def note(msg: str) -> None:
    """Progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg} ({time.perf_counter() - _T0:.1f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=4096)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--n-final", type=int, default=1_000_000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline (0 disables it)")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-autotune", action="store_true", help="heuristic launch shapes for the headline")
    ap.add_argument("--ppt", type=int, default=0,
                    help="paths per lane of the FP32 headline's date launches instead of the autotuner's "
                         "(profiling runs that must repeat one launch shape)")
    ap.add_argument("--batch", type=int, default=256, help="options in the batched form (0 disables it)")
    ap.add_argument("--batch-N", type=int, default=256)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival window of the serving form (0 disables it)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrival rate of the serving form (1/s)")
    ap.add_argument("--no-iz", action="store_true", help="skip the I&Z max-call form (Tables 1-3)")
    ap.add_argument("--no-ada", action="store_true", help="skip the AdaBoost-stump line")
    ap.add_argument("--no-maxcall5", action="store_true", help="skip the five-asset max-call line")
    ap.add_argument("--no-mincall", action="store_true", help="skip the min-call line")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1-asset put, Table 4 and I&Z geometric-put lines")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the pricer runs on a single device and has no "
              "multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0805_1827_amd import bmc, inputs

    spec = inputs.geometric_put5()
    ctx = bmc.Context(0)
    kw = dict(N=args.N, n=args.n, n_final=args.n_final, seed=args.seed)
    # launch shapes of the headline workload from the autotuner (training
    # continuation and final pricing, both precisions)
    tuning = {}
    if not args.no_autotune:
        for name, prec in (("fp32", bmc.FP32), ("fp64", bmc.FP64)):
            tuning[name] = {"ppt": bmc.bmc_autotune(ctx, spec, prec, args.N, args.n),
                            "final_ppt": bmc.bmc_autotune(ctx, spec, prec, 1, args.n_final)}
    if args.ppt > 0:
        bmc.bmc_tuning_set(ctx, d=spec.d, precision=bmc.FP32, n=args.n, ppt=args.ppt)
        tuning.setdefault("fp32", {})["ppt"] = args.ppt

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            bmc.bmc_price(ctx, spec, bmc.CMC, prec, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [bmc.bmc_price(ctx, spec, bmc.CMC, prec, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    note("launch shapes tuned")
    res32, t32 = timed(bmc.FP32, args.steps, args.warmup)
    note("FP32 prices timed")
    fp64_steps = args.fp64_steps if args.fp64_steps is not None else max(2, args.steps // 2)
    if fp64_steps > 0:
        res64, t64 = timed(bmc.FP64, fp64_steps, 1)
        note("FP64 prices timed")
    else:   # profiling runs of the FP32 form only
        res64, t64, fp64_steps = res32, t32, args.steps

    inner32 = sum(r["inner_path_steps"] for r in res32)
    inner64 = sum(r["inner_path_steps"] for r in res64)
    calc32 = sum(r["calc_seconds"] for r in res32)
    calc64 = sum(r["calc_seconds"] for r in res64)
    launches32 = args.steps * (spec.n_dates - 1)
    p32, p64 = res32[-1], res64[-1]
    se = p64["std_err"]

    slots = slots_per_step_fp32(spec.d, spec.payoff, bmc.CMC)
    slots_layout = slots_per_step_fp32(spec.d, spec.payoff, bmc.CMC, layout=True)
    achieved = slots * inner32 / calc32
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS, "traffic": measured_traffic(),
                "kernel": "k_cont<5, float> (continuation, FP32 stepping)",
                "slots_per_path_step": slots,
                "slots_per_path_step_as_drawn": slots_layout,
                "frac_as_drawn": slots_layout * inner32 / calc32 / PEAK_SLOTS,
                "avg_launch_ms": 1e3 * calc32 / launches32, "launches": launches32}
    slots64 = slots_per_step_fp64(spec.d, spec.payoff, bmc.CMC)
    roofline64 = {"bound": "alu", "achieved": slots64 * inner64 / calc64 / 1e12, "peak": PEAK_SLOTS / 1e12,
                  "unit": "T fp64-slot/s", "frac": slots64 * inner64 / calc64 / PEAK_SLOTS,
                  "kernel": "k_cont<5, double> (continuation, FP64)", "slots_per_path_step": slots64,
                  "avg_launch_ms": 1e3 * calc64 / (fp64_steps * (spec.n_dates - 1))}

    out = {
        "metric": "inner path-steps/s (FP32 stepping, FP64 accumulation)",
        "value": inner32 / t32,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "5-asset geometric-average Bermudan put, CMC, N=n=4096, 10 dates, "
                               "1e6 final paths, seed 1",
                   "d": spec.d, "dates": spec.n_dates, "N": args.N, "n": args.n, "n_final": args.n_final,
                   "method": "CMC"},
        "kernel_path_steps_per_s": inner32 / calc32,
        "asset_steps_per_s": spec.d * inner32 / t32,
        "nominal_inner_path_steps_per_price": sum(args.N * args.n * (spec.n_dates - m)
                                                  for m in range(1, spec.n_dates)),
        "fp64": {"value": inner64 / t64, "ms_per_step": 1e3 * t64 / fp64_steps,
                 "kernel_path_steps_per_s": inner64 / calc64, "asset_steps_per_s": spec.d * inner64 / t64,
                 "steps": fp64_steps, "roofline": roofline64},
        "fp32_over_fp64": (inner32 / t32) / (inner64 / t64),
        "price_fp32": p32["price"], "price_fp64": p64["price"], "std_err": se,
        "fp32_error_in_std_err": abs(p32["price"] - p64["price"]) / se,
        "latency_ms": {"p50": 1e3 * percentile([r["seconds"] for r in res32], 50),
                       "p99": 1e3 * percentile([r["seconds"] for r in res32], 99)},
        "phase_ms": {"calc": 1e3 * calc32 / args.steps,
                     "refine": 1e3 * sum(r["refine_seconds"] for r in res32) / args.steps,
                     "fit": 1e3 * sum(r["fit_seconds"] for r in res32) / args.steps,
                     "final": 1e3 * sum(r["final_seconds"] for r in res32) / args.steps},
        "inner_path_steps_per_price": inner32 // args.steps,
        "launch_shapes": tuning or "heuristic",
        "roofline": roofline,
    }
    if args.batch > 0:
        bctx = bmc.Context(0)
        out["batch"] = batch_form(bctx, bmc, inputs, args.batch, args.batch_N, 100_000)
        note("batch done")
        bctx.close()
    # the same workload with the AdaBoost-stump classifier (64 rounds)
    ada = [] if args.no_ada else [bmc.bmc_price(ctx, spec, bmc.CMC_ADA, bmc.FP32, **kw) for _ in range(3)]
    out["cmc_adaboost"] = None if args.no_ada else {
        "workload": "as the headline, CMC with AdaBoost stumps (64 rounds, 64 bins) instead of LogitBoost",
        "ms_per_price": 1e3 * float(np.median([r["seconds"] for r in ada])),
        "fit_ms_per_price": 1e3 * float(np.median([r["fit_seconds"] for r in ada])),
        "calc_ms_per_price": 1e3 * float(np.median([r["calc_seconds"] for r in ada])),
        "inner_path_steps_per_s": ada[-1]["inner_path_steps"] / float(np.median([r["calc_seconds"] for r in ada])),
        "price": ada[-1]["price"], "std_err": ada[-1]["std_err"],
        "logitboost_price": p32["price"]}
    if not args.no_ada:
        note("AdaBoost done")
    if not args.no_maxcall5:
        out["maxcall5"] = maxcall5_form(ctx, bmc, inputs)
        note("five-asset max-call done")
    if not args.no_iz:
        out["iz"] = iz_form(ctx, bmc, inputs)
        note("I&Z done")
    if not args.no_mincall:
        out["mincall"] = mincall_form(ctx, bmc, inputs)
        note("min-call done")
    if not args.no_configs:
        out["put1"] = put1_form(ctx, bmc, inputs)
        out["table4_cmc"] = table4_form(ctx, bmc, inputs)
        out["geo5_iz"] = geo5_iz_form(ctx, bmc, inputs)
        note("1-asset put, Table 4 and I&Z geometric put done")
    if args.serve_seconds > 0:
        out["serving"] = {
            "workload": f"Poisson arrivals at {args.serve_rate:g}/s for {args.serve_seconds:g} s from a catalogue "
                        "of 64 specs (d 1-40, 4-50 dates, n in 2k/8k/32k); CMC, N=256 on a rule-cache miss, "
                        "n_final=16n",
            "fp32": serving_form(ctx, bmc, inputs, args.serve_seconds, args.serve_rate, bmc.FP32),
            "fp64": serving_form(ctx, bmc, inputs, args.serve_seconds, args.serve_rate, bmc.FP64),
            "saturation_fp32": saturation_form(ctx, bmc, inputs, bmc.FP32),
            "saturation_fp64": saturation_form(ctx, bmc, inputs, bmc.FP64)}
        note("serving done")
    ctx.close()   # before the interpreter (and the HIP runtime) shuts down
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(spec, args.N, args.n, args.seed, args.cpu_seconds)
        note("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
