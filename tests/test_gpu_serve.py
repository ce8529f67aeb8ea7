"""GPU tests of the serving loop (stag_solver_submit / stag_solver_poll):
continuous batching over several resident gauge fields, results checked
against the oracle's true residual and against the same solve run alone."""

import math
import time

import numpy as np
import pytest

import synth
from tests.gpu_common import log, oracle_apply_A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


def wait_all(stag, ctx, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for tid, (nrhs, vh) in tickets.items():
            if tid in out:
                continue
            r = stag.stag_solver_poll(ctx, tid, nrhs, vh)
            if r is not None:
                out[tid] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(tickets) - len(out)} tickets still pending")
        time.sleep(0.002)
    return out


def true_res(U, L, m, b, x):
    Ax = oracle_apply_A(U, x, L, m)
    return [float(np.linalg.norm(b[r] - Ax[r]) / np.linalg.norm(b[r])) for r in range(b.shape[0])]


def test_stream_mixed_requests_alone_equals_mix(stag):
    lattices = [(4, 4, 4, 4), (8, 8, 8, 8), (6, 6, 6, 6)]
    links = [synth.haar_links(L, 100 + i) for i, L in enumerate(lattices)]
    reqs = synth.request_stream(2011, 18, rate=500.0, sizes=lattices,
                                masses=[0.05, 0.1, 0.2], tols=[1e-6, 1e-8, 1e-10], max_nrhs=4)
    precs = ["f32", "f64", "f16s"]
    with stag.Context(0) as ctx:
        stag.stag_solver_config(ctx, slots_per_batch=8)
        gauges = [ctx.gauge(L, U, precisions=("f64", "f32", "f16s")) for L, U in zip(lattices, links)]
        tickets, meta = {}, {}
        t0 = time.time()
        for q in reqs:
            # honour the Poisson arrival times (scaled) so requests join mid-flight
            while time.time() - t0 < q["t"]:
                time.sleep(0.0005)
            i = q["lattice"]
            L = lattices[i]
            b = synth.gaussian_rhs(L, q["nrhs"], q["rhs_seed"])
            inner = precs[q["id"] % 3]
            tid = stag.stag_solver_submit(ctx, gauges[i], q["mass"], b, q["tol"], inner)
            tickets[tid] = (q["nrhs"], gauges[i].vh)
            meta[tid] = (q, b, inner)
        res = wait_all(stag, ctx, tickets)
        lat = sorted(r[3] for r in res.values())
        log("served", len(res), "p50", lat[len(lat) // 2], "max", lat[-1])
        for tid, (rc, x, st, latency) in res.items():
            q, b, inner = meta[tid]
            i = q["lattice"]
            assert rc == 0, (q, st)
            tr = true_res(links[i], lattices[i], q["mass"], b, x)
            assert max(tr) <= q["tol"], (q, tr)
            # the same solve alone, through stag_cg_solve with the serving
            # loop's kernel-per-stage solver (its one-workgroup solver for
            # tiny lattices sums in another order)
            g = gauges[i]
            fb = ctx.field(g, 0, "f64", q["nrhs"]).load(b)
            fx = ctx.field(g, 0, "f64", q["nrhs"])
            rc1, st1 = stag.stag_cg_solve(ctx, g, [q["mass"]] * q["nrhs"], fb, fx,
                                          stag.cg_params(tol=q["tol"], inner=inner,
                                                         small_lattice=False))
            assert rc1 == 0
            x1 = fx.store()
            assert np.array_equal(x1, x), (q, inner, float(np.abs(x1 - x).max()))
            assert [s["iters"] for s in st1] == [s["iters"] for s in st]
            fb.destroy()
            fx.destroy()


def test_admission_waits_for_hbm_budget(stag):
    """With a budget that holds one batch at a time, requests for two
    different gauges queue and all complete."""
    L = (8, 8, 8, 8)
    U1, U2 = synth.haar_links(L, 201), synth.haar_links(L, 202)
    vh = 8 ** 4 // 2
    # gauges (f64 + f32): 2 parities x vh x (1152 + 576) bytes each
    gauge_bytes = 2 * vh * (1152 + 576)
    # one batch of 4 slots (mixed f32): x, r, t, b fp64 + y, rs, d, t, Ad fp32 ~ 4 x 7.5 vh x 48
    batch_bytes = 4 * vh * (4 * 48 + 5 * 24) + 4 * vh * 8 + 4096
    budget = 2 * gauge_bytes + batch_bytes + 8 * vh * 48 + (1 << 20)
    with stag.Context(0, hbm_budget=budget) as ctx:
        stag.stag_solver_config(ctx, slots_per_batch=4)
        g1 = ctx.gauge(L, U1, precisions=("f64", "f32"))
        g2 = ctx.gauge(L, U2, precisions=("f64", "f32"))
        tickets, meta = {}, {}
        for k in range(6):
            g, U = (g1, U1) if k % 2 == 0 else (g2, U2)
            b = synth.gaussian_rhs(L, 2, 300 + k)
            tid = stag.stag_solver_submit(ctx, g, 0.1, b, 1e-8, "f32")
            tickets[tid] = (2, vh)
            meta[tid] = (U, b)
        res = wait_all(stag, ctx, tickets)
        assert ctx.memory_used() <= budget
        for tid, (rc, x, st, latency) in res.items():
            U, b = meta[tid]
            assert rc == 0
            assert max(true_res(U, L, 0.1, b, x)) <= 1e-8


def test_poll_errors(stag):
    L = (4, 4, 4, 4)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, synth.haar_links(L, 5), precisions=("f64", "f32"))
        with pytest.raises(stag.StagError):
            stag.stag_solver_poll(ctx, 12345, 1, g.vh)
        b = synth.gaussian_rhs(L, 1, 6)
        tid = stag.stag_solver_submit(ctx, g, 0.1, b, 1e-8, "f32")
        res = wait_all(stag, ctx, {tid: (1, g.vh)})
        assert res[tid][0] == 0
        with pytest.raises(stag.StagError):
            stag.stag_solver_poll(ctx, tid, 1, g.vh)
        with pytest.raises(stag.StagError):
            stag.stag_solver_submit(ctx, g, -0.1, b, 1e-8, "f32")


def test_destroy_with_pending_tickets(stag):
    L = (8, 8, 8, 8)
    ctx = stag.Context(0)
    g = ctx.gauge(L, synth.haar_links(L, 7), precisions=("f64", "f32"))
    for k in range(4):
        stag.stag_solver_submit(ctx, g, 0.01, synth.gaussian_rhs(L, 2, 400 + k), 1e-10, "f32")
    ctx.close()  # cancels whatever is pending; must return promptly


def test_served_f16s_hard_request_hands_over_to_f32(stag):
    """8^4 Haar links at m = 0.005, tol 1e-10: fp16 storage stalls at its
    precision floor (the oracle's emulation does too: true residual ~0.5
    after three stall updates). Served on a gauge that also holds fp32
    links, each right-hand side hands over to the fp32 batch and reaches its
    fp64 true residual (checked with the oracle's A), with the same bits and
    iteration count as stag_cg_solve's own escalation of the same solve."""
    L, m, tol = (8, 8, 8, 8), 0.005, 1e-10
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 2, 1001)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"))
        tid = stag.stag_solver_submit(ctx, g, m, b, tol, "f16s")
        res = wait_all(stag, ctx, {tid: (2, g.vh)})
        rc, x, st, latency = res[tid]
        log("served f16s", rc, st)
        assert rc == 0, st
        assert all(s["inner_final"] == stag.PREC["f32"] for s in st)
        assert max(true_res(U, L, m, b, x)) <= tol
        fb = ctx.field(g, 0, "f64", 2).load(b)
        fx = ctx.field(g, 0, "f64", 2)
        rc1, st1 = stag.stag_cg_solve(ctx, g, [m, m], fb, fx, stag.cg_params(tol=tol, inner="f16s"))
        log("stag_cg_solve f16s", rc1, st1)
        assert rc1 == 0 and all(s["inner_final"] == stag.PREC["f32"] for s in st1)
        assert np.array_equal(fx.store(), x)
        assert [s["iters"] for s in st1] == [s["iters"] for s in st]


def test_served_f16s_without_f32_copy_reports_stall(stag):
    """The same hard request on a gauge without fp32 links has nowhere to go:
    it ends with ESTALL (and x is the last iterate), not a wrong success."""
    L, m, tol = (8, 8, 8, 8), 0.005, 1e-10
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 1, 1001)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f16s"))
        tid = stag.stag_solver_submit(ctx, g, m, b, tol, "f16s")
        rc, x, st, latency = wait_all(stag, ctx, {tid: (1, g.vh)}, timeout=300.0)[tid]
        log("served f16s, no f32 copy", rc, st)
        assert rc == stag.STAG_ESTALL and st[0]["status"] == stag.STAG_ESTALL
        assert st[0]["inner_final"] == stag.PREC["f16s"]
        assert st[0]["true_rel_res"] > tol


def test_gauge_destroy_refused_while_requests_uncollected(stag):
    """stag_gauge_destroy returns EBUSY while a serving request on the gauge
    is uncollected, leaves the gauge usable, and succeeds once the ticket has
    been polled (its serving batch released with it)."""
    L, m, tol = (8, 8, 8, 8), 0.05, 1e-8
    U = synth.haar_links(L, 17)
    b = synth.gaussian_rhs(L, 1, 18)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"))
        tid = stag.stag_solver_submit(ctx, g, m, b, tol, "f32")
        with pytest.raises(stag.StagError) as ei:
            g.destroy()
        assert ei.value.code == stag.STAG_EBUSY and g.h is not None
        rc, x, st, latency = wait_all(stag, ctx, {tid: (1, g.vh)})[tid]
        assert rc == 0 and max(true_res(U, L, m, b, x)) <= tol
        used = ctx.memory_used()
        g.destroy()
        assert g.h is None and ctx.memory_used() < used
        # the context keeps serving other gauges
        g2 = ctx.gauge(L, U, precisions=("f64", "f32"))
        tid = stag.stag_solver_submit(ctx, g2, m, b, tol, "f32")
        rc2, x2, st2, _ = wait_all(stag, ctx, {tid: (1, g2.vh)})[tid]
        assert rc2 == 0 and np.array_equal(x2, x)
