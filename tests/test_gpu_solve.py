"""GPU CG solves (plain fp64, mixed fp32 / fp16+scale, batched) checked
against the oracle: every solve's fp64 true residual, recomputed by the
oracle's operator, must meet the requested tolerance."""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import dense
from oracle import stag as ostag
from tests.gpu_common import links, log, oracle_apply_A, rel_norm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


@pytest.fixture(scope="module")
def ctx(stag):
    c = stag.Context(0)
    yield c
    c.close()


def true_res(U, L, masses, b, x):
    Ax = oracle_apply_A(U, x, L, masses)
    return [math.sqrt(ostag.norm2(b[r] - Ax[r]) / ostag.norm2(b[r])) for r in range(b.shape[0])]


def solve(stag, ctx, L, U, b, masses, tol, inner="f64", precisions=None, **kw):
    precisions = precisions or (("f64",) if inner == "f64" else ("f64", inner))
    g = ctx.gauge(L, U, precisions=precisions)
    fb = ctx.field(g, 0, "f64", b.shape[0]).load(b)
    fx = ctx.field(g, 0, "f64", b.shape[0])
    rc, st = stag.stag_cg_solve(ctx, g, masses, fb, fx, stag.cg_params(tol=tol, inner=inner, **kw))
    x = fx.store()
    for o in (fb, fx, g):
        o.destroy()
    return rc, st, x


def test_c1_plain_cg_matches_dense(stag, ctx):
    """4^4 Haar, m = 0.1, tol 1e-10: the first workload, against a dense solve."""
    cfg = synth.CONFIGS["c1_4x4x4x4"]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U = synth.config_links("c1_4x4x4x4")
    b = synth.config_rhs("c1_4x4x4x4")
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol)
    log(st)
    assert rc == stag.STAG_OK and st[0]["status"] == 0
    assert true_res(U, L, [m], b, x)[0] <= tol
    A = dense.dense_A_even(U, L, m)
    ev = np.linalg.eigvalsh(A)
    xd = np.linalg.solve(A, b[0].ravel()).reshape(-1, 3)
    assert rel_norm(x[0], xd) <= (ev.max() / ev.min()) * tol
    # iteration count agrees with the oracle's Fig.1 CG within a few percent
    _, ost = ostag.cg(lambda v: ostag.apply_A(U, v, L, m), b[0], tol)
    assert abs(st[0]["iters"] - ost["iters"]) <= 0.05 * ost["iters"] + 5


def test_free_field_solve_matches_fft(stag, ctx):
    L, m, tol = (8, 8, 4, 8), 0.05, 1e-10
    U = synth.unit_links(L)
    b = synth.gaussian_rhs(L, 1, 21)
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol)
    assert rc == 0
    xe = dense.fft_solve(b[0], L, m)
    kappa = (m * m + 16) / (m * m)
    assert rel_norm(x[0], xe) <= kappa * tol


def test_twisted_gauge_rotated_solve(stag, ctx):
    L, m, tol = (8, 8, 8, 8), 0.1, 1e-9
    th = np.array([[0.1, 0.2], [0.3, 0.4], [-0.5, 0.6], [0.7, -0.8]])
    gf = synth.random_gauge(L, 22)
    U = synth.gauge_transform_links(synth.twisted_links(L, th), gf)
    b = synth.gaussian_rhs(L, 1, 23)
    for inner in ("f64", "f32", "f16s"):
        rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner=inner)
        log(inner, st)
        assert rc == 0
        ge = gf.reshape(-1, 3, 3)[ostag.parity(L).reshape(-1) == 0]
        ghb = (np.conj(np.swapaxes(ge, -1, -2)) @ b[0][..., None])[..., 0]
        xe = (ge @ dense.fft_solve(ghb, L, m, th)[..., None])[..., 0]
        kappa = (m * m + 16) / (m * m)
        assert rel_norm(x[0], xe) <= kappa * tol


@pytest.mark.parametrize("inner", ["f32", "f16s"])
def test_mixed_true_residual_and_counts(stag, ctx, inner):
    """Mixed CG reaches the fp64 true residual; iteration count close to the
    oracle's emulation of the same scheme (soft, from the paper's claim that
    the iteration count is preserved)."""
    L, m, tol = (6, 6, 6, 6), 0.03, 1e-8
    U = links(L, "haar", 81)
    b = synth.gaussian_rhs(L, 1, 82)
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner=inner)
    log(inner, st)
    assert rc == 0
    res = true_res(U, L, [m], b, x)[0]
    assert res <= tol
    assert abs(st[0]["true_rel_res"] - res) <= 0.05 * res + 1e-15
    _, est = ostag.mixed_cg(U, L, m, b[0], tol, prec=inner)
    log("emulation", est)
    slack = 0.05 if inner == "f32" else 0.25
    assert abs(st[0]["iters"] - est["iters"]) <= slack * est["iters"] + 10
    assert abs(st[0]["reliable_updates"] - est["updates"]) <= 2 + (0 if inner == "f32" else 4)


def test_fig2_restart_variant_matches_refinement_oracle(stag, ctx):
    """The Fig.2 variant (the direction restarts at every update, the inner
    cycle ends at a delta reduction from its start) against the oracle's
    iterative refinement: same true residual bar, iteration and outer-step
    counts close to the oracle's; and it needs more iterations than the
    Eq.6 carry-over on the same system (the point of Sec.3.2)."""
    L, m, tol = (6, 6, 6, 6), 0.03, 1e-8
    U = links(L, "haar", 81)
    b = synth.gaussian_rhs(L, 1, 82)
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f32", mixed_variant="restart")
    log("restart", st)
    assert rc == 0 and true_res(U, L, [m], b, x)[0] <= tol
    _, est = ostag.refinement_cg(U, L, m, b[0], tol, prec="f32", eps_in=0.1)
    log("oracle refinement", est)
    assert abs(st[0]["iters"] - est["iters"]) <= 0.05 * est["iters"] + 10
    assert abs(st[0]["reliable_updates"] - est["outer"]) <= 2
    rc2, st2, _ = solve(stag, ctx, L, U, b, [m], tol, inner="f32")
    assert rc2 == 0 and st2[0]["iters"] < st[0]["iters"]


@pytest.mark.parametrize("variant", ["carry", "reliable", "fold_only"])
def test_update_ablations_match_oracle(stag, ctx, variant):
    """The Sec.3.2 scheme and its two one-sided ablations on a system where
    fp32 alone cannot reach the tolerance (4^4 Haar, m = 0.1, 1e-10): the
    GPU reproduces the oracle's outcome, iteration count and residual level."""
    L, m, tol = (4, 4, 4, 4), 0.1, 1e-10
    U = links(L, "haar", 11)
    b = synth.gaussian_rhs(L, 1, 111)
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f32", mixed_variant=variant)
    log(variant, rc, st[0])
    upd = {"carry": "both"}.get(variant, variant)
    _, est = ostag.mixed_cg(U, L, m, b[0], tol, prec="f32", update=upd)
    log("oracle", est)
    res = true_res(U, L, [m], b, x)[0]
    assert abs(st[0]["true_rel_res"] - res) <= 1e-3 * res + 1e-14
    if variant == "carry":
        assert rc == 0 and res <= tol
        assert abs(st[0]["iters"] - est["iters"]) <= 0.05 * est["iters"] + 5
    elif variant == "reliable":
        # stalls at fp32's level and runs to the iteration cap, like the oracle
        assert rc == stag.STAG_ENOCONV and est["status"] == "noconv"
        assert st[0]["iters"] == est["iters"]
        assert res > 1e3 * tol and 0.1 < res / est["true_rel_res"] < 10
    else:
        # the iterated residual meets tol, the true one does not
        assert rc == stag.STAG_ENOCONV and est["status"] == "inaccurate"
        assert abs(st[0]["iters"] - est["iters"]) <= 0.05 * est["iters"] + 5
        assert res > 10 * tol and 0.1 < res / est["true_rel_res"] < 10


def test_batched_equals_single(stag, ctx):
    """Each right-hand side of a block solve equals its own single solve."""
    L, tol = (8, 8, 8, 8), 1e-8
    U = links(L, "exp", 31, 0.5)
    n = 5
    b = synth.gaussian_rhs(L, n, 32)
    masses = [0.05, 0.1, 0.02, 0.2, 0.05]
    for inner in ("f64", "f32"):
        rc, st, xb = solve(stag, ctx, L, U, b, masses, tol, inner=inner)
        assert rc == 0
        res = true_res(U, L, masses, b, xb)
        assert max(res) <= tol
        for r in range(n):
            rc1, st1, x1 = solve(stag, ctx, L, U, b[r:r + 1], [masses[r]], tol, inner=inner)
            assert rc1 == 0
            assert st1[0]["iters"] == st[r]["iters"]
            assert np.array_equal(x1[0], xb[r]), (inner, r, rel_norm(x1[0], xb[r]))


def test_largest_block_and_one_more_refused(stag, ctx):
    """The largest block, 16 right-hand sides (kernel groups of 8 and 8, the
    direction as a pass of its own), ragged masses: every one meets the
    oracle's true residual and the first and last equal their single solves
    bit for bit; a 17th right-hand side is refused on the host."""
    L, tol = (8, 8, 8, 8), 1e-8
    U = links(L, "haar", 71)
    n = 16
    b = synth.gaussian_rhs(L, n, 72)
    masses = [0.05 + 0.01 * (r % 5) for r in range(n)]
    rc, st, xb = solve(stag, ctx, L, U, b, masses, tol, inner="f32")
    log("16 RHS", rc, [s_["iters"] for s_ in st])
    assert rc == 0 and max(true_res(U, L, masses, b, xb)) <= tol
    for r in (0, n - 1):
        rc1, st1, x1 = solve(stag, ctx, L, U, b[r:r + 1], [masses[r]], tol, inner="f32")
        assert rc1 == 0 and st1[0]["iters"] == st[r]["iters"]
        assert np.array_equal(x1[0], xb[r])
    g = ctx.gauge(L, U, precisions=("f64",))
    with pytest.raises(stag.StagError):
        ctx.field(g, 0, "f64", n + 1)
    g.destroy()


def test_graph_and_eager_bitwise(stag, ctx):
    L, m, tol = (8, 8, 8, 8), 0.05, 1e-8
    U = links(L, "haar", 41)
    b = synth.gaussian_rhs(L, 1, 42)
    outs = []
    for use_graph in (True, False, True):
        rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f32", use_graph=use_graph, graph_k=8)
        assert rc == 0
        outs.append((st[0]["iters"], x))
    assert outs[0][0] == outs[1][0] == outs[2][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][1], outs[2][1])


@pytest.mark.parametrize("inner", ["f64", "f32", "f16s"])
def test_consecutive_solves_new_rhs_buffers(stag, ctx, inner):
    """One gauge, one solver workspace reused by solves whose right-hand
    sides sit in different (freed and reallocated) buffers: each solve must
    answer its own b (the fix-up kernels inside the cached graphs read b)."""
    L, m, tol = (6, 6, 6, 6), 0.1, 1e-9
    U = links(L, "haar", 71)
    g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"))
    p = stag.cg_params(tol=tol, inner=inner, graph_k=8)
    xs = []
    for seed in (72, 73, 74):
        b = synth.gaussian_rhs(L, 2, seed)
        fb = ctx.field(g, 0, "f64", 2).load(b)
        fx = ctx.field(g, 0, "f64", 2)
        rc, st = stag.stag_cg_solve(ctx, g, [m, m], fb, fx, p)
        x = fx.store()
        fb.destroy()
        fx.destroy()
        assert rc == 0, st
        assert max(true_res(U, L, [m, m], b, x)) <= tol
        xs.append(x)
    # the last solve in a fresh context gives the same bits
    with stag.Context(0) as c2:
        g2 = c2.gauge(L, U, precisions=("f64", "f32", "f16s"))
        b = synth.gaussian_rhs(L, 2, 74)
        fb = c2.field(g2, 0, "f64", 2).load(b)
        fx = c2.field(g2, 0, "f64", 2)
        rc, st = stag.stag_cg_solve(c2, g2, [m, m], fb, fx, p)
        assert rc == 0 and np.array_equal(fx.store(), xs[-1])


@pytest.mark.parametrize("inner", ["f64", "f32", "f16s"])
def test_initial_guess(stag, ctx, inner):
    """use_x0: the exact solution needs no iteration, a perturbed one converges
    to the same tolerance, and b = 0 gives x = 0 whatever x0 was."""
    L, m, tol = (6, 6, 6, 6), 0.1, 1e-10
    U = links(L, "haar", 81)
    b = synth.gaussian_rhs(L, 2, 82)
    b[1] = 0.0
    g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"))
    fb = ctx.field(g, 0, "f64", 2).load(b)
    fx = ctx.field(g, 0, "f64", 2)
    rc, st = stag.stag_cg_solve(ctx, g, [m, m], fb, fx, stag.cg_params(tol=tol, inner=inner))
    assert rc == 0
    x = fx.store()
    assert not np.any(x[1])
    # restart from the converged answer: nothing to do
    rc, st = stag.stag_cg_solve(ctx, g, [m, m], fb, fx, stag.cg_params(tol=tol, inner=inner, use_x0=True))
    assert rc == 0 and st[0]["iters"] == 0 and np.array_equal(fx.store()[0], x[0])
    # from a perturbed guess; the b = 0 slot returns x = 0
    x0 = x + 1e-3 * synth.gaussian_rhs(L, 2, 83)
    fx.load(x0)
    rc, st = stag.stag_cg_solve(ctx, g, [m, m], fb, fx, stag.cg_params(tol=tol, inner=inner, use_x0=True))
    xr = fx.store()
    assert rc == 0 and 0 < st[0]["iters"]
    assert true_res(U, L, [m], b[:1], xr[:1])[0] <= tol
    assert not np.any(xr[1])
    g.destroy()


def test_f16s_escalates_to_f32(stag, ctx):
    """An fp16-storage inner solve that stalls (forced here with a tiny stall
    window) ends in ESTALL without escalation, and with it continues in fp32
    from the current x to the requested true residual."""
    L, m, tol = (8, 8, 8, 8), 0.01, 1e-10
    U = links(L, "haar", 91)
    b = synth.gaussian_rhs(L, 1, 92)
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f16s", precisions=("f64", "f32", "f16s"),
                      stall_iters=3, max_stall=1, escalate=False)
    log("no escalation", rc, st[0])
    assert rc == stag.STAG_ESTALL and st[0]["inner_final"] == stag.PREC["f16s"]
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f16s", precisions=("f64", "f32", "f16s"),
                      stall_iters=3, max_stall=1)
    log("escalated", rc, st[0])
    assert rc == 0 and st[0]["inner_final"] == stag.PREC["f32"]
    assert true_res(U, L, [m], b, x)[0] <= tol
    assert abs(st[0]["true_rel_res"] - true_res(U, L, [m], b, x)[0]) <= 1e-12


def test_zero_rhs_and_nan(stag, ctx):
    L = (4, 4, 4, 4)
    U = links(L, "haar", 51)
    b = np.zeros((2, 128, 3), dtype=np.complex128)
    b[1] = synth.gaussian_rhs(L, 1, 52)[0]
    rc, st, x = solve(stag, ctx, L, U, b, [0.1, 0.1], 1e-9)
    assert rc == 0 and st[0]["iters"] == 0 and not np.any(x[0])
    b[1, 3, 1] = np.nan
    with pytest.raises(stag.StagError):
        solve(stag, ctx, L, U, b, [0.1, 0.1], 1e-9)


def test_max_iter_reports_noconv(stag, ctx):
    L = (8, 8, 8, 8)
    U = links(L, "haar", 61)
    b = synth.gaussian_rhs(L, 1, 62)
    for inner in ("f64", "f32"):
        rc, st, x = solve(stag, ctx, L, U, b, [0.01], 1e-10, inner=inner, max_iter=20)
        assert rc == stag.STAG_ENOCONV and st[0]["status"] == stag.STAG_ENOCONV
        assert st[0]["iters"] <= 20 + 1


@pytest.mark.parametrize("r12", [False, True])
def test_c2_time_to_1e8_fp64_and_mixed(stag, ctx, r12):
    """16^3 x 32, exp(i 0.3 H) links, m = 0.01: plain fp64 CG and fp32-inner
    CG with fp64 reliable updates both reach true residual 1e-8 (true residual
    checked by the C oracle, whose links are never compressed), with full
    links and with the 12-parameter copies the benchmark solves on.
    The fp64 and fp32-inner iteration counts agree with the oracle's Fig.1 CG
    and Sec.3.2 emulation on the same system."""
    name = "c2_16x16x16x32"
    cfg = synth.CONFIGS[name]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U = synth.config_links(name)
    b = synth.config_rhs(name)
    g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=r12)
    fb = ctx.field(g, 0, "f64", 1).load(b)
    fx = ctx.field(g, 0, "f64", 1)
    iters = {}
    for inner in ("f64", "f32", "f16s"):
        rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, stag.cg_params(tol=tol, inner=inner))
        x = fx.store()
        res = true_res(U, L, [m], b, x)[0]
        log(name, "r12" if r12 else "full", inner, st[0], "oracle true res", res)
        assert rc == 0 and res <= tol
        assert abs(st[0]["true_rel_res"] - res) <= 0.05 * res + 1e-14
        iters[inner] = st[0]["iters"]
    ref = _c2_oracle_iters()
    log("oracle iterations", ref)
    for inner in ("f64", "f32"):
        assert abs(iters[inner] - ref[inner]) <= 0.05 * ref[inner] + 5, (inner, iters, ref)


def _c2_oracle_iters():
    """Iterations of the oracle's Fig.1 CG and fp32 Sec.3.2 emulation on the
    16^3 x 32 workload, stored by tests/golden/make_oracle_counts.py (the
    numpy emulation takes minutes at this size)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_counts.json")) as f:
        c = json.load(f)["c2_16x16x16x32"]
    return {"f64": c["fig1_fp64_cg"]["iters"], "f32": c["sec32_fp32_mixed"]["iters"]}


def test_f16s_hands_over_at_first_slow_cycle(stag, ctx):
    """8^4 Haar, m = 0.01, 1e-10: fp16 storage cannot refine this system well
    (the oracle's emulation ends its pass at the first update, whose true
    residual has not halved; plain fp16 refinement takes over 13 000
    iterations). With fp32 links on the gauge the solve hands over there and
    finishes in fp32 to the requested fp64 true residual, in far fewer
    iterations than the fp16 iteration alone needs."""
    L, m, tol = (8, 8, 8, 8), 0.01, 1e-10
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 1, 1001)
    _, est = ostag.mixed_cg(U, L, m, b[0], tol, prec="f16s", max_stall=3, slow_ratio=0.5)
    assert est["status"] == "stall" and est["updates"] == 1
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol, inner="f16s", precisions=("f64", "f32", "f16s"))
    log("f16s with hand-over", rc, st[0], "oracle fp16 pass", est)
    assert rc == 0 and st[0]["inner_final"] == stag.PREC["f32"]
    assert true_res(U, L, [m], b, x)[0] <= tol
    rc32, st32, _ = solve(stag, ctx, L, U, b, [m], tol, inner="f32")
    # the fp16 pass ends near where the oracle's does; the rest is about an fp32 solve
    assert st[0]["iters"] <= st32[0]["iters"] + 1.25 * est["iters"] + 50


def test_f16s_hands_over_when_far_behind_cg(stag, ctx):
    """6^4 Haar, m = 0.02, 1e-8: every fp16 refinement cycle still contracts
    the true residual tenfold, but at about 3x the iterations CG needs (the
    oracle's emulation: 7 131 iterations against fp32's 2 419; its budget ends
    the fp16 pass after about 3 200). The solve hands over to fp32 once it is
    twice behind the CG bound and reaches the tolerance (checked with the
    oracle's fp64 A) in far fewer iterations than fp16 alone; at m = 0.05,
    where fp16 keeps within the bound, the whole solve stays in fp16."""
    L, tol = (6, 6, 6, 6), 1e-8
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 1, 1001)
    precs = ("f64", "f32", "f16s")
    rc, st, x = solve(stag, ctx, L, U, b, [0.02], tol, inner="f16s", precisions=precs)
    log("f16s with hand-over", rc, st[0])
    assert rc == 0 and st[0]["inner_final"] == stag.PREC["f32"]
    assert true_res(U, L, [0.02], b, x)[0] <= tol
    rc16, st16, _ = solve(stag, ctx, L, U, b, [0.02], tol, inner="f16s", precisions=precs,
                          escalate=False)
    log("f16s alone", rc16, st16[0])
    assert rc16 == 0 and st16[0]["inner_final"] == stag.PREC["f16s"]
    assert st16[0]["iters"] > 1.3 * st[0]["iters"]
    rc, st, x = solve(stag, ctx, L, U, b, [0.05], tol, inner="f16s", precisions=precs)
    log("f16s at m = 0.05", rc, st[0])
    assert rc == 0 and st[0]["inner_final"] == stag.PREC["f16s"]
    assert true_res(U, L, [0.05], b, x)[0] <= tol


def test_timing_mode_counts_launches_and_keeps_results(stag, ctx):
    """With kernel timing on, a solve runs eagerly with events at each
    kernel's start and end: the same iterations and bits as the graph solve,
    one stage-1, stage-2 and update launch per iteration (plus the launches
    of flagged slots idling to the end of their segment, and up to two
    blocks of K = 64 iterations enqueued behind the poll that sees
    convergence), and plausible per-launch durations."""
    L, m, tol = (8, 8, 8, 8), 0.05, 1e-8
    U = links(L, "haar", 45)
    b = synth.gaussian_rhs(L, 1, 46)
    g = ctx.gauge(L, U, precisions=("f64", "f32"))
    fb = ctx.field(g, 0, "f64", 1).load(b)
    fx = ctx.field(g, 0, "f64", 1)
    p = stag.cg_params(tol=tol, inner="f32")
    rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
    x_ref = fx.store()
    stag.stag_timing_enable(ctx, True)
    try:
        rc2, st2 = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
        counts = {k: stag.stag_timing_read(ctx, k) for k in (stag.K_HOP1, stag.K_HOP2, stag.K_UPDATE)}
    finally:
        stag.stag_timing_enable(ctx, False)
    log("timed solve", st2[0], counts)
    assert rc == rc2 == 0 and st2[0]["iters"] == st[0]["iters"]
    assert np.array_equal(fx.store(), x_ref)
    n1, n2, nu = (counts[k][0] for k in (stag.K_HOP1, stag.K_HOP2, stag.K_UPDATE))
    assert n1 == n2 == nu and st[0]["iters"] <= n1 <= st[0]["iters"] + 3 * 64
    for n, ms in counts.values():
        assert 0.5 <= ms * 1e3 / n <= 1000.0
    for o in (fb, fx, g):
        o.destroy()
