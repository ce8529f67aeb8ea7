#!/usr/bin/env python3
"""Benchmark of the staggered CG hot path on one MI355X.

A step is one complete solve of A x = b (A = m^2 - D_eo D_oe) on the
16^3 x 32 lattice with exp(i 0.3 H) links, m = 0.01, one complex Gaussian
right-hand side, to true relative residual 1e-8, with fp32 inner CG and fp64
reliable updates, timed from b resident in HBM to x resident in HBM with the
fp64 true residual verified. Prints one JSON line on stdout (progress goes
to stderr).

Beside the headline it reports: the dominant kernel's achieved bandwidth
against the 8 TB/s HBM peak (HIP events on the launch stream, inside the
timed solves), plain fp64 CG and fp16-storage mixed CG on the same system
(time-to-1e-8), the A-apply bandwidth per precision on the 32^3 x 64
lattice, and the fp64 CPU oracle timed on this host as a baseline.
"""

from __future__ import annotations

import argparse
import functools
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 solve & solves/s, mixed vs FP64 CG; A-apply HBM GB/s; p99 lat"
WORKLOAD = "c2_16x16x16x32"
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_MB = 256          # MI355X last-level (MALL) cache


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_NAMES = ("hop_stage1", "hop_stage2", "update")


def kernel_bytes(which, inner, vh, costs, r12):
    """Algorithmic bytes of one launch of a CG-iteration kernel (as the solver runs it)."""
    if which == 0:
        return vh * costs.hop_bytes_per_site(inner, 1, lazy=True, r12=r12)
    if which == 1:
        return vh * costs.hop_bytes_per_site(inner, 2, lazy=True, r12=r12)
    return vh * costs.update_bytes_per_site(inner, inner != "f64")


COPY_FLOATS = 64 << 20  # calibration copy: 256 MiB each way
TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "c2_16x16x16x32_iteration_kernels_hbm_traffic.md")


KERNEL_SOURCES = ("common.h", "launch.h", "kern.h", "hop.hip", "blas.hip", "layout.hip")


def csrc_digest():
    """sha256 over the device-code sources (names and contents) of the kernels."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1111_0125_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def kernel_names(tune, inner, npairs=4):
    """Symbol names of the three iteration kernels for a tuned shape (one RHS)."""
    p = {"f64": 0, "f32": 1, "f16s": 2}[inner]
    nt = "true" if tune["nt"] else "false"
    op = 2 if inner == "f64" else 3
    return [f"void stag::k_hop<{p}, {tune['S1']}, 1, 0, {nt}, {npairs}>(stag::HopArgs)",
            f"void stag::k_hop<{p}, {tune['S2']}, 1, 2, {nt}, {npairs}>(stag::HopArgs)",
            f"void stag::k_vec<{p}, 1, {op}>(stag::VecArgs)"]


def measured_traffic(kernel, links):
    """HBM bytes per launch of `kernel` from the committed counter summary, when
    it was taken on these sources with these links; else None."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            txt = f.read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("kernel_src_sha256") != csrc_digest() or blob.get("links") != links:
        return None
    k = blob.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


A_SHAPES = [(S, nt, sw) for nt in (1, 0) for sw in (1, 0) for S in (1, 2, 4)]
A_TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                 "a_apply_32x32x32x64_hbm_traffic.md")


def summary_blob(path):
    """The JSON block of a committed counter summary, or None."""
    try:
        with open(path) as f:
            txt = f.read()
        return json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None


def a_leg_traffic(leg, shape):
    """HBM bytes per A application of leg `leg` in launch shape `shape` from the
    committed 32^3x64 counter summary, when it was taken on these sources; else None."""
    blob = summary_blob(A_TRAFFIC_SUMMARY)
    if not blob or blob.get("kernel_src_sha256") != csrc_digest():
        return None
    key = f"{leg} S={shape['S1']} nt={shape['nt']} swizzle={shape['swizzle']}"
    v = blob.get("legs", {}).get(key)
    return None if v is None else v.get("hbm_bytes_per_A")


def a_apply_leg(stag, torch, costs, ctx, g, leg, prec, v, mass, reps, improved=False, r12=False,
                sweep_reps=10, order=None):
    """A on one gauge copy: every launch shape (lanes per site S for both stages,
    non-temporal link loads, XCD-aware block order) timed over `sweep_reps`
    back-to-back applications after 3 warm-ups, then the fastest three times
    over `reps` (the median is reported), between torch events on the stream
    the library launches on. `order`
    collects (leg, shape, applications) in launch order for the counter
    summary."""
    vh = g.vh
    stream = torch.cuda.current_stream()
    fi = ctx.field(g, 0, prec, 1).load(v)
    fo = ctx.field(g, 0, prec, 1)

    def run(shape, k):
        S, nt, sw = shape
        stag.stag_tune_set(ctx, prec, 1, vh, S1=S, S2=S, nt=nt, swizzle=sw, improved=improved)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            stag.stag_apply_A(ctx, g, [mass], fi, fo, stream=stream)
        e0.record(stream)
        for _ in range(k):
            stag.stag_apply_A(ctx, g, [mass], fi, fo, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if order is not None:
            order.append({"leg": leg, "S": S, "nt": nt, "swizzle": sw, "applications": 3 + k})
        return e0.elapsed_time(e1) / k

    sweep = {f"S={S} nt={nt} swizzle={sw}": round(run((S, nt, sw), sweep_reps) * 1e3, 2)
             for S, nt, sw in A_SHAPES}
    best = min(A_SHAPES, key=lambda t: sweep[f"S={t[0]} nt={t[1]} swizzle={t[2]}"])
    trials = sorted(run(best, reps) for _ in range(3))
    ms = trials[1]  # the median of three
    fi.destroy()
    fo.destroy()
    byts = vh * costs.a_bytes_per_site(prec, r12=r12, improved=improved)
    gbs = byts / (ms * 1e-3) / 1e9
    paper_b = vh * costs.paper_a_bytes_per_site(prec, r12=r12, improved=improved)
    shape = {"S1": best[0], "S2": best[0], "nt": best[1], "swizzle": best[2]}
    out = {"us_per_A": round(ms * 1e3, 2), "trials_us_per_A": [round(t * 1e3, 2) for t in trials],
           "GB/s": round(gbs, 1),
           "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
           # every neighbour read counted, as the paper counts (Sec.2)
           "paper_convention_GB/s": round(paper_b / (ms * 1e-3) / 1e9, 1),
           "GFLOP/s": round(vh * costs.a_flops_per_site(improved=improved) / (ms * 1e-3) / 1e9, 1),
           "bytes_per_A": byts, "shape": shape, "sweep_us_per_A": sweep}
    t = a_leg_traffic(leg, shape)
    out["traffic_bytes_per_A"] = t
    out["traffic_ratio"] = None if t is None else round(t / byts, 4)
    log("A-apply 32^3x64", leg, {k: out[k] for k in ("us_per_A", "GB/s", "frac_of_8TBs", "shape",
                                                    "traffic_ratio")})
    return out


@functools.lru_cache(maxsize=1)
def c3_inputs(synth):
    name = "c3_32x32x32x64"
    log("generating", name, "links ...")
    return synth.config_links(name), synth.config_rhs(name)


def improved_32(stag, torch, costs, synth, reps=30, solves=True, order=None):
    """The improved operator (fat links + three-hop long links) on 32^3 x 64:
    fields from the Haar links of the 32^3 x 64 workload (fat = 9/8 U plus
    0.05 complex normal noise, long = -1/24 U U U), A-apply bandwidth per
    precision (each in its fastest launch shape) and time to 1e-10 at m = 0.01,
    fp32-inner mixed CG against plain fp64 CG."""
    name = "c3_32x32x32x64"
    cfg = synth.CONFIGS[name]
    L, m, tol = cfg["L"], 0.01, 1e-10
    U, b = c3_inputs(synth)
    log("improved: building fat and long links")
    fat, lng = synth.naik_links(U, fat_noise=0.05, seed=cfg["gauge_seed"] + 100)
    out = {"lattice": list(L), "mass": m, "tol": tol,
           "fields": "fat = 9/8 U + 0.05 N(0,1) complex, long = -1/24 U(x) U(x+mu) U(x+2mu)"}
    v = synth.gaussian_rhs(L, 1, cfg["rhs_seed"])
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, fat, precisions=("f64", "f32", "f16s"), long=lng)
        del fat, lng
        for prec in ("f64", "f32", "f16s"):
            out["A_" + prec] = a_apply_leg(stag, torch, costs, ctx, g, "improved_" + prec, prec, v,
                                           m, reps, improved=True, order=order)
        for prec in (("f32", "f64") if solves else ()):
            stag.stag_tune(ctx, g, prec, 1)  # the solver's iteration kernels
        fb = ctx.field(g, 0, "f64", 1).load(b)
        fx = ctx.field(g, 0, "f64", 1)
        for inner in (("f32", "f64") if solves else ()):
            p = stag.cg_params(tol=tol, inner=inner)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s0 = st[0]
            out["solve_" + inner] = {"time_to_tol_s": round(dt, 4), "status": rc,
                                     "iters": s0["iters"], "reliable_updates": s0["reliable_updates"],
                                     "true_rel_res": s0["true_rel_res"],
                                     "us_per_iteration": round(dt * 1e6 / max(s0["iters"], 1), 2)}
            log("improved solve", inner, out["solve_" + inner])
    if solves and out["solve_f64"]["status"] == 0 and out["solve_f32"]["status"] == 0:
        out["speedup_f32_vs_f64"] = round(out["solve_f64"]["time_to_tol_s"] /
                                          out["solve_f32"]["time_to_tol_s"], 3)
    return out


def timed_solves(stag, torch, ctx, g, mass, fb, fx, params, k):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(k):
        rc, st = stag.stag_cg_solve(ctx, g, [mass], fb, fx, params)
        if rc != 0:
            raise RuntimeError(f"solve failed: rc={rc} {st}")
        last = st[0]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / k, last


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """GB/s of a plain elementwise read-and-write kernel (torch.mul, nbytes
    each way): the streaming rate this chip reaches in practice, for scale."""
    x = torch.ones(nbytes // 4, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(x, 2.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes / (e0.elapsed_time(e1) * 1e-3 / reps) / 1e9
    del x, y
    return round(gbs, 1)


def a_apply_bandwidth(stag, torch, costs, synth, reps=50, order=None):
    """GB/s of A = both hop stages on the 32^3 x 64 lattice, per precision,
    full and 12-parameter links, each in its fastest launch shape, timed with
    torch events on the stream the library launches on."""
    name = "c3_32x32x32x64"
    cfg = synth.CONFIGS[name]
    L = cfg["L"]
    U, _ = c3_inputs(synth)
    v = synth.gaussian_rhs(L, 1, cfg["rhs_seed"])
    out = {}
    for r12 in (False, True):
        with stag.Context(0) as ctx:
            precs = ("f64", "f32", "f16s")
            g = ctx.gauge(L, U, precisions=precs, r12=r12)
            for prec in precs:
                key = prec + ("_r12" if r12 else "")
                out[key] = a_apply_leg(stag, torch, costs, ctx, g, key, prec, v, cfg["mass"], reps,
                                       r12=r12, order=order)
    return out


def c3_solves(stag, torch, synth, costs):
    """32^3x64 Haar, m = 0.005, 1e-10: mixed CG with fp16+scale and with
    fp32 inner iterations, and plain fp64 CG; time-to-tolerance each, and the
    mixed solutions' distance from the fp64 one (every solve meets the same
    true residual, so they may differ by up to about kappa * tol)."""
    name = "c3_32x32x32x64"
    cfg = synth.CONFIGS[name]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U, b = c3_inputs(synth)
    out = {"lattice": list(L), "mass": m, "tol": tol, "links": "12-parameter"}
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=True)
        fb = ctx.field(g, 0, "f64", 1).load(b)
        fx = ctx.field(g, 0, "f64", 1)
        xs = {}
        for inner in ("f16s", "f32", "f64"):
            stag.stag_tune(ctx, g, inner, 1)
            p = stag.cg_params(tol=tol, inner=inner)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s0 = st[0]
            xs[inner] = fx.store()[0]
            out[inner] = {"time_to_tol_s": round(dt, 4), "status": rc, "iters": s0["iters"],
                          "reliable_updates": s0["reliable_updates"], "restarts": s0["restarts"],
                          "true_rel_res": s0["true_rel_res"], "inner_final": s0["inner_final"],
                          "us_per_iteration": round(dt * 1e6 / max(s0["iters"], 1), 2)}
            log("c3", inner, out[inner])
        import numpy as np
        x64 = xs.pop("f64")
        n64 = float(np.linalg.norm(x64))
        for inner, x in xs.items():
            out[inner]["rel_err_vs_f64_solution"] = float(np.linalg.norm(x - x64)) / n64
        del xs, x64
        # the same links at m = 0.1 and 1e-8, a system fp16 storage can refine
        # (kappa u16 near 1): where its lower traffic per iteration pays
        wc = {"mass": 0.1, "tol": 1e-8}
        for inner in ("f16s", "f32", "f64"):
            p = stag.cg_params(tol=1e-8, inner=inner)
            stag.stag_cg_solve(ctx, g, [0.1], fb, fx, p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st = stag.stag_cg_solve(ctx, g, [0.1], fb, fx, p)
            torch.cuda.synchronize()
            wc[inner] = {"time_to_tol_s": round(time.perf_counter() - t0, 4), "status": rc,
                         "iters": st[0]["iters"], "inner_final": st[0]["inner_final"],
                         "true_rel_res": st[0]["true_rel_res"]}
        if all(wc[k]["status"] == 0 for k in ("f16s", "f32", "f64")):
            wc["speedup_f16s_vs_f32"] = round(wc["f32"]["time_to_tol_s"] / wc["f16s"]["time_to_tol_s"], 3)
            wc["speedup_f16s_vs_f64"] = round(wc["f64"]["time_to_tol_s"] / wc["f16s"]["time_to_tol_s"], 3)
        out["m0.1_tol1e-8"] = wc
        log("c3 links at m = 0.1", wc)
    if out["f64"]["status"] == 0:
        for inner in ("f16s", "f32"):
            if out[inner]["status"] == 0:
                out[f"speedup_{inner}_vs_f64"] = round(out["f64"]["time_to_tol_s"] /
                                                       out[inner]["time_to_tol_s"], 3)
    return out


def batched_c4(stag, torch, synth):
    """24^3 x 48, exp(i 0.5 H) links, m = 0.01, 12 right-hand sides to 1e-8:
    one block solve (links loaded once per site for all 12) against one
    single-RHS solve repeated 12 times, mixed and plain fp64."""
    name = "c4_24x24x24x48"
    cfg = synth.CONFIGS[name]
    L, m, tol, n = cfg["L"], cfg["mass"], cfg["tol"], cfg["nrhs"]
    log("generating", name)
    U = synth.config_links(name)
    b = synth.config_rhs(name)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"), r12=True)
        # the solver runs 12 right-hand sides as kernels of 8 and 4
        for k in (8, 4, 1):
            stag.stag_tune(ctx, g, "f32", k)
        fb = ctx.field(g, 0, "f64", n).load(b)
        fx = ctx.field(g, 0, "f64", n)
        p = stag.cg_params(tol=tol, inner="f32")
        stag.stag_cg_solve(ctx, g, [m] * n, fb, fx, p)  # warm-up (graphs, workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = stag.stag_cg_solve(ctx, g, [m] * n, fb, fx, p)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        f1 = ctx.field(g, 0, "f64", 1).load(b[:1])
        x1 = ctx.field(g, 0, "f64", 1)
        stag.stag_cg_solve(ctx, g, [m], f1, x1, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc1, st1 = stag.stag_cg_solve(ctx, g, [m], f1, x1, p)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t0
        p64 = stag.cg_params(tol=tol, inner="f64")
        stag.stag_tune(ctx, g, "f64", 1)
        stag.stag_cg_solve(ctx, g, [m], f1, x1, p64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stag.stag_cg_solve(ctx, g, [m], f1, x1, p64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
    out = {"nrhs": n, "block_solve_s": round(tb, 4), "solves_per_s": round(n / tb, 3),
           "time_to_1e-8_per_rhs_s": round(tb / n, 5),
           "single_solve_s": round(t1, 4), "sequential_12_s_est": round(12 * t1, 4),
           "block_speedup": round(12 * t1 / tb, 3),
           "single_fp64_solve_s": round(t64, 4), "sequential_12_fp64_s_est": round(12 * t64, 4),
           "block_speedup_vs_fp64": round(12 * t64 / tb, 3), "status": rc,
           "max_iters": max(s["iters"] for s in st),
           "max_true_rel_res": max(s["true_rel_res"] for s in st)}
    log("batched", out)
    return out


def c1_gpu(stag, torch, synth, solves=20):
    """The 4^4 workload (Haar links, m = 0.1, 1e-10) on the GPU: the
    one-workgroup solver in fp64 (Fig.1) and with fp32 inner iterations
    (Sec.3.2), median over `solves` solves from b resident in HBM."""
    import statistics
    name = "c1_4x4x4x4"
    cfg = synth.CONFIGS[name]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U, b = synth.config_links(name), synth.config_rhs(name)
    out = {"lattice": list(L), "mass": m, "tol": tol, "solver": "one workgroup per right-hand side"}
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"))
        fb = ctx.field(g, 0, "f64", 1).load(b)
        fx = ctx.field(g, 0, "f64", 1)
        for inner in ("f64", "f32"):
            p = stag.cg_params(tol=tol, inner=inner)
            stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
            ts = []
            for _ in range(solves):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            out[inner] = {"time_to_1e-10_ms": round(statistics.median(ts) * 1e3, 3), "status": rc,
                          "iters": st[0]["iters"], "true_rel_res": st[0]["true_rel_res"]}
    log("c1 4^4", out)
    return out


# Requests per second the full serving stream below drains at when offered
# more than it can take (80 requests at 2/s on one MI355X, fp32 inner):
# the capacity its default arrival rate is set against.
SERVE_CAPACITY_RPS = 1.27


def serving(stag, synth, n_requests=40, rate=None, full=False, seed=2011):
    """A Poisson stream of solve requests over resident gauge fields,
    continuously batched per gauge; solves/s and submit-to-finish latency.
    full (the benchmark's default): the four resident Haar fields 8^4,
    16^3x32, 24^3x48, 32^3x64 (gauge seeds 15-18), masses {0.005, 0.01,
    0.05, 0.1}, tolerances {1e-6, 1e-8, 1e-10}, 1-8 right-hand sides, at
    half the stream's measured capacity unless `rate` is given. Otherwise a
    light stream over 8^4 and 16^3x32 with smooth links."""
    import numpy as np
    if full:
        sizes = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
        masses = [0.005, 0.01, 0.05, 0.1]
        log("serving: generating", sizes)
        links = [synth.haar_links(L, 15 + i) for i, L in enumerate(sizes)]
    else:
        sizes = [(8, 8, 8, 8), (16, 16, 16, 32)]
        masses = [0.01, 0.02, 0.05, 0.1]
        log("serving: generating", sizes)
        # the same smooth-link recipe as the 16^3 x 32 workload (exp(i 0.3 H))
        links = [synth.exp_ih_links(L, 15 + i, 0.3) for i, L in enumerate(sizes)]
    tols = [1e-6, 1e-8, 1e-10]
    rate = rate or (50.0 if not full else 0.5 * SERVE_CAPACITY_RPS)
    reqs = synth.request_stream(seed, n_requests, rate, sizes, masses, tols, max_nrhs=8)
    lat, nrhs_done = [], 0
    lat_by = {i: [] for i in range(len(sizes))}
    with stag.Context(0) as ctx:
        gauges = [ctx.gauge(L, U, precisions=("f64", "f32"), r12=True) for L, U in zip(sizes, links)]
        del links
        pending = {}
        t0 = time.perf_counter()
        t_log = t0
        i = 0
        while i < len(reqs) or pending:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["t"] <= now:
                q = reqs[i]
                L = sizes[q["lattice"]]
                b = synth.gaussian_rhs(L, q["nrhs"], q["rhs_seed"])
                tid = stag.stag_solver_submit(ctx, gauges[q["lattice"]], q["mass"], b, q["tol"], "f32")
                pending[tid] = (q["nrhs"], gauges[q["lattice"]].vh, q["lattice"])
                i += 1
            for tid in list(pending):
                nr, vh, li = pending[tid]
                r = stag.stag_solver_poll(ctx, tid, nr, vh, want_x=False)
                if r is not None:
                    rc, _, st, latency = r
                    if rc != 0:
                        raise RuntimeError(f"serving request failed: {rc} {st}")
                    lat.append(latency)
                    lat_by[li].append(latency)
                    nrhs_done += nr
                    del pending[tid]
            if time.perf_counter() - t_log > 15.0:
                t_log = time.perf_counter()
                log(f"serving: {len(lat)} of {len(reqs)} requests done, {len(pending)} pending")
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
    lat = np.array(lat)
    out = {"requests": len(reqs), "rhs": nrhs_done, "wall_s": round(wall, 3),
           "solves_per_s": round(nrhs_done / wall, 3), "requests_per_s": round(len(reqs) / wall, 3),
           "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
           "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
           "arrival_rate_per_s": rate,
           "rho_vs_capacity": (round(rate / SERVE_CAPACITY_RPS, 3) if full else None),
           "capacity_requests_per_s": SERVE_CAPACITY_RPS if full else None,
           "lattices": ["x".join(map(str, L)) for L in sizes],
           "links": "Haar" if full else "exp(i 0.3 H)",
           "p50_p99_by_lattice_s": {"x".join(map(str, sizes[i])): [
               round(float(np.percentile(v, 50)), 4), round(float(np.percentile(v, 99)), 4)]
               for i, v in lat_by.items() if v},
           "masses": masses, "tols": tols, "inner": "f32"}
    log("serving", out)
    return out


def cpu_baseline(synth, L, U, b, mass, gpu_fp64_iters, target_s):
    """The fp64 C oracle's Fig.1 CG on the same system, timed on this host
    for a bounded number of iterations and scaled to a full solve."""
    from oracle import c as oc
    oc.lib()
    t0 = time.perf_counter()
    oc.cg_fixed(U, b, L, mass, 5)
    per_iter = (time.perf_counter() - t0) / 5
    n = max(10, min(int(target_s / per_iter), gpu_fp64_iters))
    log(f"cpu baseline: {n} oracle iterations (~{n * per_iter:.1f} s) ...")
    t0 = time.perf_counter()
    oc.cg_fixed(U, b, L, mass, n)
    per_iter = (time.perf_counter() - t0) / n
    solve_s = per_iter * gpu_fp64_iters
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": 1.0 / solve_s, "unit": "solves/s", "cores": oc.threads(), "kind": "oracle",
        "host_cpus": os.cpu_count(), "cpu_model": model,
        "sample": (f"{n} Fig.1 fp64 CG iterations of the C+OpenMP oracle on the same 16^3x32 "
                   f"system, scaled to the {gpu_fp64_iters} iterations a full 1e-8 fp64 solve "
                   f"takes ({per_iter * 1e3:.2f} ms/iteration)"),
        "ms_per_iteration": per_iter * 1e3,
    }


def cpu_a_apply(synth, costs):
    """The C oracle's fp64 A (Eq.2-3 over Eq.5, full links) on the host cores:
    median of 10 applications on 4^4 and 16^3x32, of 3 on 32^3x64, with the
    same compulsory bytes per even site as the GPU's fp64 A; and the oracle's
    full Fig.1 CG on 4^4 (m = 0.1, 1e-10)."""
    import statistics
    from oracle import c as oc
    out = {}
    for name, reps in (("c1_4x4x4x4", 10), ("c2_16x16x16x32", 10), ("c3_32x32x32x64", 3)):
        cfg = synth.CONFIGS[name]
        L, m = cfg["L"], cfg["mass"]
        U, b = synth.config_links(name), synth.config_rhs(name)[0]
        oc.apply_A(U, b, L, m)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oc.apply_A(U, b, L, m)
            ts.append(time.perf_counter() - t0)
        t = statistics.median(ts)
        nbytes = b.shape[0] * costs.a_bytes_per_site("f64")
        out[name] = {"ms_per_A": round(t * 1e3, 3), "GB/s": round(nbytes / t / 1e9, 2), "reps": reps}
        if name == "c1_4x4x4x4":
            t0 = time.perf_counter()
            _, st = oc.cg(U, b, L, m, cfg["tol"])
            out[name]["cg_to_tol_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
            out[name]["cg_iters"] = st["iters"]
        del U, b
    log("cpu A", out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", default="f32", choices=["f32", "f16s"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the fp64 / f16s comparison solves and the 32^3x64 A-apply")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-light", action="store_true",
                    help="light serving stream (8^4 and 16^3x32, smooth links) instead of the "
                         "stream over all four Haar lattices")
    ap.add_argument("--serve-requests", type=int, default=80)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="request arrival rate per second (default: half the measured capacity "
                         "of the full stream; 50 light)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only tune and launch the iteration kernels (as timed for the roofline), "
                         "then a 256 MiB copy kernel: the program that hardware-counter runs profile")
    ap.add_argument("--a-apply-only", action="store_true",
                    help="only the 32^3x64 A applications (Eq.5 full and 12-parameter links, and "
                         "the improved operator), autotuned: the program the A-apply kernel "
                         "profiles trace")
    ap.add_argument("--block-kernels-only", action="store_true",
                    help="only tune and time the block iteration kernels of the 24^3x48 workload "
                         "for 4, 8 and 12 right-hand sides, then a 256 MiB copy kernel: the program "
                         "the block-kernel profiles run")
    ap.add_argument("--c3-solves-only", action="store_true",
                    help="only the 32^3x64 Haar solves at m = 0.1 to 1e-8 (fp32 and fp16+scale "
                         "inner, 12-parameter links), a warm-up and a timed solve each: the program "
                         "the in-solve kernel trace of the large lattice runs")
    ap.add_argument("--full-links", action="store_true",
                    help="store the gauge copies in full (18 reals per link) instead of 12 parameters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus}: the library solves on one GPU; "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import tempfile

    # persistent launch-shape table (stag_tune reads it before timing shapes)
    os.environ.setdefault("STAG_TUNE_CACHE", os.path.join(tempfile.gettempdir(),
                                                          "stag_tune_cache.txt"))
    import torch

    import paper_1111_0125_amd as stag
    import synth
    from paper_1111_0125_amd import costs

    if args.a_apply_only:
        torch.cuda.init()
        order = []
        out = {"a_apply_32x32x32x64": a_apply_bandwidth(stag, torch, costs, synth, order=order),
               "improved_32x32x32x64": improved_32(stag, torch, costs, synth, solves=False,
                                                   order=order),
               "copy_kernel_GB/s": copy_bandwidth(torch),
               # what the counter summary needs to attribute dispatches: every
               # (leg, shape) in launch order, each application two hop kernels,
               # then the 1 GiB copy kernel (3 + 20 launches)
               "launch_order": order, "copy_bytes_each_way": 1 << 30,
               "kernel_src_sha256": csrc_digest()}
        print(json.dumps(out), flush=True)
        return

    if args.c3_solves_only:
        torch.cuda.init()
        name = "c3_32x32x32x64"
        L = synth.CONFIGS[name]["L"]
        U, b = c3_inputs(synth)
        m, tol = 0.1, 1e-8
        out = {"c3_solves_only": True, "workload": name, "lattice": list(L), "mass": m, "tol": tol,
               "links": "r12", "solves": {}}
        with stag.Context(0) as ctx:
            g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=True)
            out["vh"] = g.vh
            fb = ctx.field(g, 0, "f64", 1).load(b)
            fx = ctx.field(g, 0, "f64", 1)
            tune64 = stag.stag_tune(ctx, g, "f64", 1)[0]
            for inner in ("f32", "f16s"):
                tune = stag.stag_tune(ctx, g, inner, 1)[0]
                p = stag.cg_params(tol=tol, inner=inner)
                stag.stag_cg_solve(ctx, g, [m], fb, fx, p)  # warm-up: graphs, workspace
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
                torch.cuda.synchronize()
                out["solves"][inner] = {"tune": tune, "tune_f64": tune64, "status": rc,
                                        "ms": round((time.perf_counter() - t0) * 1e3, 3),
                                        "iters": st[0]["iters"],
                                        "reliable_updates": st[0]["reliable_updates"],
                                        "inner_final": st[0]["inner_final"]}
        out["kernel_src_sha256"] = csrc_digest()
        print(json.dumps(out), flush=True)
        return

    if args.block_kernels_only:
        torch.cuda.init()
        os.environ.pop("STAG_TUNE_CACHE", None)  # every shape is timed (and counted)
        name = "c4_24x24x24x48"
        c4 = synth.CONFIGS[name]
        with stag.Context(0) as ctx:
            g = ctx.gauge(c4["L"], synth.config_links(name), precisions=("f64", "f32"), r12=True)
            out = {"block_kernels_only": True, "workload": name, "inner": "f32", "links": "r12",
                   "vh": g.vh, "tune": {}, "us": {}, "kernel_src_sha256": csrc_digest()}
            for n in (4, 8, 12):
                out["tune"][n], _ = stag.stag_tune(ctx, g, "f32", n)
                out["us"][n] = stag.stag_time_kernels(ctx, g, "f32", n, reps=20)
                log("block kernels", n, out["tune"][n], out["us"][n])
        nf = COPY_FLOATS
        xs = torch.ones(nf, device="cuda")
        ys = torch.empty_like(xs)
        for _ in range(3):
            torch.mul(xs, 2.0, out=ys)
        torch.cuda.synchronize()
        out.update({"copy_bytes_read": nf * 4, "copy_bytes_written": nf * 4})
        print(json.dumps(out), flush=True)
        return

    cfg = synth.CONFIGS[WORKLOAD]
    L, mass, tol = cfg["L"], cfg["mass"], cfg["tol"]
    log("inputs", WORKLOAD)
    U = synth.config_links(WORKLOAD)
    b = synth.config_rhs(WORKLOAD)
    torch.cuda.init()
    if args.kernels_only:
        # the counter runs time every launch shape: no shapes from a table
        os.environ.pop("STAG_TUNE_CACHE", None)
    ctx = stag.Context(0)
    r12 = not args.full_links
    g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=r12)
    vh = g.vh
    tunes = {p: stag.stag_tune(ctx, g, p, 1)[0] for p in ("f64", "f32", "f16s")}
    loaded, measured = stag.stag_tune_counts(ctx)
    log("tuned", tunes, "loaded from the table:", loaded, "measured:", measured)
    inner = args.inner
    if args.kernels_only:
        us = stag.stag_time_kernels(ctx, g, inner, 1, reps=20)
        n = COPY_FLOATS
        xs = torch.ones(n, device="cuda")
        ys = torch.empty_like(xs)
        for _ in range(3):
            torch.mul(xs, 2.0, out=ys)  # reads and writes n * 4 bytes
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "tune": tunes[inner], "us": us,
                          "kernel_names": kernel_names(tunes[inner], inner),
                          "inner": inner, "links": "r12" if r12 else "full", "vh": vh,
                          "copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
                          "kernel_src_sha256": csrc_digest()}), flush=True)
        return
    fb = ctx.field(g, 0, "f64", 1).load(b)
    fx = ctx.field(g, 0, "f64", 1)
    params = stag.cg_params(tol=tol, inner=inner)

    for _ in range(args.warmup):
        rc, st = stag.stag_cg_solve(ctx, g, [mass], fb, fx, params)
        log("warmup", rc, st[0])

    # ---- timed region: K whole solves (graph replays), b and x resident in HBM
    sec, last = timed_solves(stag, torch, ctx, g, mass, fb, fx, params, args.steps)
    log("timed", args.steps, "solves:", round(sec * 1e3, 3), "ms each;", last)

    # the same kernels inside a solve: one more solve with its kernels launched
    # eagerly, events recorded at each kernel's start and end (the graph
    # replays of the timed region cannot be bracketed kernel by kernel)
    stag.stag_timing_enable(ctx, True)
    stag.stag_cg_solve(ctx, g, [mass], fb, fx, params)
    in_solve = {name: stag.stag_timing_read(ctx, kk) for name, kk in
                (("hop_stage1", stag.K_HOP1), ("hop_stage2", stag.K_HOP2), ("update", stag.K_UPDATE))}
    stag.stag_timing_enable(ctx, False)

    # ---- the iteration's kernels, launched exactly as in the solve and in its
    # order, timed between HIP events on the library's stream
    us = stag.stag_time_kernels(ctx, g, inner, 1, reps=200)
    kinds = {}
    for k, name in enumerate(KERNEL_NAMES):
        byts = kernel_bytes(k, inner, vh, costs, r12)
        kinds[name] = {"avg_us": round(us[k], 3), "bytes_per_launch": byts,
                       "GB/s": round(byts / (us[k] * 1e-6) / 1e9, 1)}
    dom = max(kinds, key=lambda k: kinds[k]["avg_us"])
    d = kinds[dom]
    dom_name = kernel_names(tunes[inner], inner)[KERNEL_NAMES.index(dom)]
    traffic = measured_traffic(dom_name, "r12" if r12 else "full")
    roofline = {"bound": "hbm", "achieved": d["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["GB/s"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel_symbol": dom_name,
                "kernel": (f"{dom} ({inner}, 16^3x32, {'12-parameter' if r12 else 'full'}"
                           f" links, S1={tunes[inner]['S1']} S2={tunes[inner]['S2']} "
                           f"nt={tunes[inner]['nt']} swizzle={tunes[inner]['swizzle']})"),
                "avg_us": d["avg_us"],
                "bytes_per_launch": d["bytes_per_launch"]}
    # what one iteration touches: both parities' links and the inner vectors
    # (r, d, t, A d in the inner precision, y in fp32); on this lattice it fits
    # in the 256 MB Infinity Cache, so 8 TB/s is a conservative ceiling here
    link_b = (costs.LINK_BYTES_R12 if r12 else costs.LINK_BYTES)[inner]
    ws = vh * (2 * (8 * link_b + costs.SITE_SCALE_BYTES[inner])
               + 4 * costs.SPINOR_BYTES[inner] + costs.SPINOR_BYTES["f32"])
    roofline["iteration_working_set_MB"] = round(ws / 1e6, 1)
    roofline["infinity_cache_MB"] = INFINITY_CACHE_MB
    n_in, ms_in = in_solve[dom]
    in_us = ms_in * 1e3 / max(n_in, 1)
    roofline["in_solve"] = {"launches": n_in, "avg_us": round(in_us, 3),
                            "GB/s": round(d["bytes_per_launch"] / (in_us * 1e-6) / 1e9, 1),
                            "frac": round(d["bytes_per_launch"] / (in_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                            "how": "one solve with its kernels launched eagerly (no graph), "
                                   "events recorded at each kernel's start and end; mean over all "
                                   "of its launches of the kernel (inactive-slot launches included)"}
    iters = last["iters"]
    per_iter_us = sec * 1e6 / max(iters, 1)
    log("kernels", kinds, "per-iteration wall", round(per_iter_us, 2), "us")

    result = {
        "metric": METRIC,
        "value": round(1.0 / sec, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{inner}+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"16^3x32 lattice, exp(i*0.3*H) links (seed {cfg['gauge_seed']}), "
                         f"m={mass}, 1 complex Gaussian RHS (seed {cfg['rhs_seed']}), "
                         f"true residual {tol:g}, {inner}-inner CG + fp64 reliable updates"),
            "lattice": list(L), "mass": mass, "tol": tol, "inner": inner, "nrhs": 1,
            "links": "12-parameter (third row rebuilt)" if r12 else "full",
        },
        "roofline": roofline,
        "solve": {"iters": iters, "reliable_updates": last["reliable_updates"],
                  "true_rel_res": last["true_rel_res"], "time_to_1e-8_ms": round(sec * 1e3, 3),
                  "us_per_iteration": round(per_iter_us, 3),
                  "kernel_us_per_iteration": round(sum(us), 3),
                  "bytes_per_iteration": costs.cg_iteration_bytes_per_site(
                      inner, True, r12=r12) * vh},
        "kernels": kinds,
        "tune": tunes,
        "tune_table": {"path": os.environ.get("STAG_TUNE_CACHE"), "loaded": loaded,
                       "measured": measured},
    }

    fp64_iters = None
    if not args.no_extras:
        p64 = stag.cg_params(tol=tol, inner="f64")
        stag.stag_cg_solve(ctx, g, [mass], fb, fx, p64)
        s64, st64 = timed_solves(stag, torch, ctx, g, mass, fb, fx, p64, 2)
        fp64_iters = st64["iters"]
        result["fp64_cg"] = {"time_to_1e-8_ms": round(s64 * 1e3, 3), "iters": st64["iters"],
                             "true_rel_res": st64["true_rel_res"],
                             "solves_per_s": round(1 / s64, 3)}
        result["speedup_mixed_vs_fp64"] = round(s64 / sec, 3)
        # the plain iterative refinement of Fig.2 (direction restarted at each
        # update) on the same system, against the Eq.6 carry-over above
        prs = stag.cg_params(tol=tol, inner=inner, mixed_variant="restart")
        stag.stag_cg_solve(ctx, g, [mass], fb, fx, prs)
        srs, strs = timed_solves(stag, torch, ctx, g, mass, fb, fx, prs, 2)
        result["fig2_restart_variant"] = {"time_to_1e-8_ms": round(srs * 1e3, 3),
                                          "iters": strs["iters"],
                                          "updates": strs["reliable_updates"],
                                          "true_rel_res": strs["true_rel_res"],
                                          "iters_vs_eq6_carry": round(strs["iters"] / max(iters, 1), 3)}
        # the two update methods of Sec.3.2 alone (capped at 4x the iterations
        # of the scheme that applies both)
        abl = {}
        for var in ("reliable", "fold_only"):
            pv = stag.cg_params(tol=tol, inner=inner, mixed_variant=var, max_iter=4 * iters)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, stv = stag.stag_cg_solve(ctx, g, [mass], fb, fx, pv)
            torch.cuda.synchronize()
            abl[var] = {"status": rc, "iters": stv[0]["iters"], "updates": stv[0]["reliable_updates"],
                        "true_rel_res": stv[0]["true_rel_res"],
                        "ms": round((time.perf_counter() - t0) * 1e3, 3)}
        result["update_ablations"] = abl
        p16 = stag.cg_params(tol=tol, inner="f16s")
        stag.stag_cg_solve(ctx, g, [mass], fb, fx, p16)
        s16, st16 = timed_solves(stag, torch, ctx, g, mass, fb, fx, p16, 2)
        result["f16s_mixed"] = {"time_to_1e-8_ms": round(s16 * 1e3, 3), "iters": st16["iters"],
                                "reliable_updates": st16["reliable_updates"],
                                "true_rel_res": st16["true_rel_res"],
                                "solves_per_s": round(1 / s16, 3)}
        log("fp64", result["fp64_cg"], "f16s", result["f16s_mixed"])
    ctx.close()

    if not args.no_extras:
        result["a_apply_32x32x32x64"] = a_apply_bandwidth(stag, torch, costs, synth)
        # for scale: what a plain streaming kernel reaches (1 GiB each way)
        cb = copy_bandwidth(torch)
        result["copy_kernel_GB/s"] = cb
        for v in result["a_apply_32x32x32x64"].values():
            v["frac_of_copy_kernel"] = round(v["GB/s"] / cb, 4)
        result["c3_32x32x32x64_solves"] = c3_solves(stag, torch, synth, costs)
        result["improved_32x32x32x64"] = improved_32(stag, torch, costs, synth)
        for v in result["improved_32x32x32x64"].values():
            if isinstance(v, dict) and "GB/s" in v:
                v["frac_of_copy_kernel"] = round(v["GB/s"] / cb, 4)
        c3_inputs.cache_clear()
        result["batched_24x24x24x48_12rhs"] = batched_c4(stag, torch, synth)
        result["c1_4x4x4x4_gpu"] = c1_gpu(stag, torch, synth)
        result["serving"] = serving(stag, synth, n_requests=args.serve_requests,
                                    rate=args.serve_rate or None, full=not args.serve_light)

    if not args.no_cpu:
        if fp64_iters is None:
            with stag.Context(0) as c2:
                g2 = c2.gauge(L, U, precisions=("f64",))
                fb2 = c2.field(g2, 0, "f64", 1).load(b)
                fx2 = c2.field(g2, 0, "f64", 1)
                _, st = stag.stag_cg_solve(c2, g2, [mass], fb2, fx2, stag.cg_params(tol=tol))
                fp64_iters = st[0]["iters"]
        result["cpu_baseline"] = cpu_baseline(synth, L, U, b[0], mass, fp64_iters, args.cpu_seconds)
        result["cpu_baseline"]["a_apply_fp64"] = cpu_a_apply(synth, costs)
        c1 = result.get("c1_4x4x4x4_gpu")
        if c1:
            c1["cpu_oracle_fp64_cg_ms"] = result["cpu_baseline"]["a_apply_fp64"]["c1_4x4x4x4"].get(
                "cg_to_tol_ms")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
