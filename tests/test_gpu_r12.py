"""12-parameter link storage (two rows per SU(3) link, the third rebuilt in
the kernels, the phases applied from the coordinates) against the CPU
oracle's fp64 operator, which never compresses anything, and, for fp16
storage, against the oracle's model of the compressed fp16 operator."""

import math

import numpy as np
import pytest

import synth
from oracle import stag as ostag
from tests.gpu_common import links, log, oracle_apply_A, oracle_dslash, rel_max

pytestmark = pytest.mark.gpu

LATTICES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 4, 8), (2, 4, 6, 8), (16, 16, 16, 8)]
TOL = {"f64": 1e-12, "f32": 1e-6, "f16s": 1e-3}


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


@pytest.fixture(scope="module")
def ctx(stag):
    c = stag.Context(0)
    yield c
    c.close()


def rel_rms(a, b):
    return float(np.sqrt(np.mean(np.abs(a - b) ** 2) / np.mean(np.abs(b) ** 2)))


def check_f16s_model(got, model, exact, what):
    """fp16 results against the oracle's model of the compressed fp16
    operator: only rare one-unit differences in a stored rounding remain, so
    they sit far closer to the model than to the exact fp64 result (whose
    distance is the link and vector quantisation itself)."""
    e_model, e_exact = rel_rms(got, model), rel_rms(got, exact)
    log(what, "rms vs model", e_model, "vs fp64", e_exact)
    assert e_model < 0.1 * e_exact


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_r12_dslash_and_A(stag, ctx, L, prec):
    U = links(L, "haar", 13)
    g = ctx.gauge(L, U, precisions=(prec,), r12=True)
    for p_in in (0, 1):
        v = synth.gaussian_rhs(L, 2, 14 + p_in)
        fi = ctx.field(g, p_in, prec, 2).load(v)
        fo = ctx.field(g, 1 - p_in, prec, 2)
        stag.stag_dslash(ctx, g, fi, fo)
        got, exact = fo.store(), oracle_dslash(U, v, L, p_in)
        err = rel_max(got, exact)
        log("dslash r12", L, prec, p_in, err)
        assert err <= TOL[prec]
        if prec == "f16s":
            lo = ostag.LowOperator(U, L, 0.0, "f16s", r12=True)
            model = np.stack([ostag.q_f16s(ostag.from_full(
                lo.dslash_full(ostag.to_full(ostag.q_f16s(v[r]), L, p_in)), L, 1 - p_in))
                for r in range(2)])
            check_f16s_model(got, model, exact, f"dslash r12 f16s {L} p_in={p_in}")
    v = synth.gaussian_rhs(L, 3, 16)
    masses = [0.1, 0.05, 0.3]
    fi = ctx.field(g, 0, prec, 3).load(v)
    fo = ctx.field(g, 0, prec, 3)
    stag.stag_apply_A(ctx, g, masses, fi, fo)
    got, exact = fo.store(), oracle_apply_A(U, v, L, masses)
    err = rel_max(got, exact)
    log("A r12", L, prec, err)
    assert err <= TOL[prec]
    if prec == "f16s":
        model = np.stack([ostag.LowOperator(U, L, masses[r], "f16s", r12=True)(v[r]) for r in range(3)])
        check_f16s_model(got, model, exact, f"A r12 f16s {L}")
    g.destroy()


def test_r12_rejects_non_su3(stag, ctx):
    L = (4, 4, 4, 4)
    U = links(L, "haar", 17).copy()
    U[1, 2, 3, 0, 2] *= np.exp(0.3j)  # unitary, det != 1
    with pytest.raises(stag.StagError):
        ctx.gauge(L, U, precisions=("f64",), r12=True)
    U = links(L, "haar", 17).copy()
    U[0, 0, 0, 1, 3, 0, 0] += 1e-6  # not unitary
    with pytest.raises(stag.StagError):
        ctx.gauge(L, U, precisions=("f32",), r12=True)
    # the same links are fine in full storage
    ctx.gauge(L, U, precisions=("f32",)).destroy()


@pytest.mark.parametrize("inner", ["f64", "f32", "f16s"])
def test_r12_solves_and_block_equals_single(stag, ctx, inner):
    """Solves on 12-parameter links reach the fp64 true residual (measured with
    the oracle's full A); a block of right-hand sides gives each one's bits."""
    L, tol = (8, 8, 8, 8), 1e-9
    U = links(L, "exp", 18, 0.3)
    b = synth.gaussian_rhs(L, 3, 19)
    masses = [0.05, 0.1, 0.2]
    g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=True)
    fb = ctx.field(g, 0, "f64", 3).load(b)
    fx = ctx.field(g, 0, "f64", 3)
    rc, st = stag.stag_cg_solve(ctx, g, masses, fb, fx, stag.cg_params(tol=tol, inner=inner))
    log("r12 solve", inner, rc, st[0])
    assert rc == 0
    x = fx.store()
    Ax = oracle_apply_A(U, x, L, masses)
    for r in range(3):
        res = math.sqrt(ostag.norm2(b[r] - Ax[r]) / ostag.norm2(b[r]))
        assert res <= tol
    f1 = ctx.field(g, 0, "f64", 1).load(b[1:2])
    x1 = ctx.field(g, 0, "f64", 1)
    rc1, st1 = stag.stag_cg_solve(ctx, g, masses[1:2], f1, x1, stag.cg_params(tol=tol, inner=inner))
    assert rc1 == 0 and st1[0]["iters"] == st[1]["iters"]
    assert np.array_equal(x1.store()[0], x[1])
    g.destroy()


def _shapes(nrhs):
    for S1 in (1, 2, 4):
        for S2 in (1, 2, 4):
            for nt in ((0, 1) if nrhs == 1 else (1,)):
                for sw in ((0, 1) if nrhs == 1 else (0, 1, 2, 3, 4)):
                    yield S1, S2, nt, sw


@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("r12", [False, True])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_launch_shapes_bitwise_identical(stag, ctx, prec, r12, nrhs):
    """A through every launch shape gives the same bits (one RHS takes
    different load orders by shape: all of a lane's hop pairs requested up
    front when they fit in registers, else the first), with full and
    12-parameter links, and meets the oracle."""
    L = (4, 6, 4, 8)
    U = links(L, "haar", 31)
    g = ctx.gauge(L, U, precisions=(prec,), r12=r12)
    v = synth.gaussian_rhs(L, nrhs, 32)
    masses = [0.1, 0.2][:nrhs]
    fi = ctx.field(g, 0, prec, nrhs).load(v)
    fo = ctx.field(g, 0, prec, nrhs)
    saved = stag.stag_tune_get(ctx, prec, nrhs, g.vh)
    outs = {}
    try:
        for shape in _shapes(nrhs):
            log("shape", prec, r12, nrhs, shape)
            stag.stag_tune_set(ctx, prec, nrhs, g.vh, *shape)
            stag.stag_apply_A(ctx, g, masses, fi, fo)
            outs[shape] = fo.store()
    finally:
        stag.stag_tune_set(ctx, prec, nrhs, g.vh, saved["S1"], saved["S2"], saved["nt"],
                           saved["swizzle"])
    ref = next(iter(outs.values()))
    for k, o in outs.items():
        assert np.array_equal(o, ref), k
    tol = {"f64": 1e-12, "f32": 1e-6, "f16s": 1e-3}[prec]
    assert rel_max(ref, oracle_apply_A(U, v, L, masses)) <= tol
    for o in (fi, fo, g):
        o.destroy()


@pytest.mark.parametrize("inner,r12", [("f32", True), ("f16s", True), ("f16s", False)])
def test_mixed_solve_bitwise_across_shapes(stag, ctx, inner, r12):
    """A mixed solve (deferred direction in stage 1, own-site operand in
    stage 2, fp64 fix-ups) gives the same iterations and bits whatever launch
    shapes the iteration and fix-up kernels take."""
    L = (8, 8, 8, 8)
    U = links(L, "haar", 33)
    b = synth.gaussian_rhs(L, 1, 34)
    m, tol = 0.05, 1e-9
    g = ctx.gauge(L, U, precisions=("f64", inner), r12=r12)
    fb = ctx.field(g, 0, "f64", 1).load(b)
    fx = ctx.field(g, 0, "f64", 1)
    saved = {p: stag.stag_tune_get(ctx, p, 1, g.vh) for p in ("f64", inner)}
    res = []
    try:
        for S in (1, 2, 4):
            for p in ("f64", inner):
                stag.stag_tune_set(ctx, p, 1, g.vh, S, S, S % 2, S // 4)
            rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx,
                                        stag.cg_params(tol=tol, inner=inner, small_lattice=False))
            log(inner, S, st[0]["iters"], st[0]["true_rel_res"])
            assert rc == 0
            res.append((st[0]["iters"], fx.store()))
    finally:
        for p, c in saved.items():
            stag.stag_tune_set(ctx, p, 1, g.vh, c["S1"], c["S2"], c["nt"], c["swizzle"])
    for it, x in res[1:]:
        assert it == res[0][0]
        assert np.array_equal(x, res[0][1])
    Ax = oracle_apply_A(U, res[0][1], L, [m])
    assert math.sqrt(ostag.norm2(b[0] - Ax[0]) / ostag.norm2(b[0])) <= tol
    for o in (fb, fx, g):
        o.destroy()
