"""Batched multi-RHS solves at the 24^3 x 48 configuration: 12 complex
Gaussian right-hand sides solved together (links loaded once per site per
stage for all of them), fp32 inner CG with fp64 reliable updates."""

import math

import numpy as np
import pytest

import synth
from oracle import stag as ostag
from tests.gpu_common import log, oracle_apply_A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


@pytest.mark.parametrize("r12", [False, True])
def test_c4_block_solve_12_rhs(stag, r12):
    """With full links and with the 12-parameter copies the
    benchmark runs on; true residuals from the oracle's uncompressed A."""
    name = "c4_24x24x24x48"
    cfg = synth.CONFIGS[name]
    L, m, tol, n = cfg["L"], cfg["mass"], cfg["tol"], cfg["nrhs"]
    log("generating", name)
    U = synth.config_links(name)
    b = synth.config_rhs(name)
    assert b.shape[0] == n == 12
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"), r12=r12)
        fb = ctx.field(g, 0, "f64", n).load(b)
        fx = ctx.field(g, 0, "f64", n)
        rc, st = stag.stag_cg_solve(ctx, g, [m] * n, fb, fx, stag.cg_params(tol=tol, inner="f32"))
        log("block solve", rc, st[0], "seconds", st[0]["seconds"])
        assert rc == 0
        x = fx.store()
        # every right-hand side: fp64 true residual from the C oracle
        Ax = oracle_apply_A(U, x, L, m)
        res = [math.sqrt(ostag.norm2(b[r] - Ax[r]) / ostag.norm2(b[r])) for r in range(n)]
        log("true residuals", max(res))
        assert max(res) <= tol
        # one right-hand side alone gives the same bits
        j = 5
        f1 = ctx.field(g, 0, "f64", 1).load(b[j:j + 1])
        x1 = ctx.field(g, 0, "f64", 1)
        rc1, st1 = stag.stag_cg_solve(ctx, g, [m], f1, x1, stag.cg_params(tol=tol, inner="f32"))
        assert rc1 == 0 and st1[0]["iters"] == st[j]["iters"]
        assert np.array_equal(x1.store()[0], x[j])


@pytest.mark.parametrize("nrhs", [2, 4, 8, 12])
def test_block_orders_bitwise_identical(stag, nrhs):
    """Every block order (plain, XCD-aware, and XCD-aware in groups of 2, 4
    or 8 t-slices with t fastest) and lane count gives the same bits for a
    block A, on a lattice whose t-slices are whole blocks for every lane count
    (8^4: 256 sites per slice and parity), and meets the oracle."""
    L = (8, 8, 8, 8)
    U = synth.haar_links(L, 41)
    v = synth.gaussian_rhs(L, nrhs, 42)
    masses = [0.05 + 0.01 * r for r in range(nrhs)]
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f32",), r12=True)
        fi = ctx.field(g, 0, "f32", nrhs).load(v)
        fo = ctx.field(g, 0, "f32", nrhs)
        outs = {}
        for S in (1, 2, 4):
            for sw in range(5):
                stag.stag_tune_set(ctx, "f32", nrhs, g.vh, S, S, 1, sw)
                stag.stag_apply_A(ctx, g, masses, fi, fo)
                outs[(S, sw)] = fo.store()
        ref = outs[(1, 0)]
        for k, o in outs.items():
            assert np.array_equal(o, ref), k
        Ax = oracle_apply_A(U, v, L, np.array(masses))
        assert float(np.abs(ref - Ax).max() / np.abs(Ax).max()) <= 1e-6


@pytest.mark.parametrize("n", [8, 16])
def test_block_solve_bitwise_across_block_orders(stag, n):
    """A mixed block solve gives the same iterations and bits in every block
    order, and the bits of a single-RHS solve on this small lattice (whose
    stage 1 forms the direction at every neighbour); each right-hand side
    meets the oracle's true residual. 8 RHS run here as two overlapping
    groups of 4 whose stage 1 forms the direction too, 16 as two groups of 8
    with a direction pass of their own (block hop stages, fp64 fix-ups)."""
    L, m, tol = (8, 8, 8, 8), 0.05, 1e-9
    U = synth.haar_links(L, 43)
    b = synth.gaussian_rhs(L, n, 44)
    res = []
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"), r12=True)
        fb = ctx.field(g, 0, "f64", n).load(b)
        fx = ctx.field(g, 0, "f64", n)
        for sw in range(5):
            for p in ("f64", "f32"):
                for k in (4, 8, 16):  # the kernels of the block and of its groups
                    stag.stag_tune_set(ctx, p, k, g.vh, 1, 1, 1, sw)
            rc, st = stag.stag_cg_solve(ctx, g, [m] * n, fb, fx,
                                        stag.cg_params(tol=tol, inner="f32", small_lattice=False))
            assert rc == 0, st
            res.append(([s["iters"] for s in st], fx.store()))
        f1 = ctx.field(g, 0, "f64", 1).load(b[3:4])
        x1 = ctx.field(g, 0, "f64", 1)
        rc1, st1 = stag.stag_cg_solve(ctx, g, [m], f1, x1,
                                      stag.cg_params(tol=tol, inner="f32", small_lattice=False))
        assert rc1 == 0 and st1[0]["iters"] == res[0][0][3]
        assert np.array_equal(x1.store()[0], res[0][1][3])
    for it, x in res[1:]:
        assert it == res[0][0] and np.array_equal(x, res[0][1])
    Ax = oracle_apply_A(U, res[0][1], L, m)
    r = [math.sqrt(ostag.norm2(b[k] - Ax[k]) / ostag.norm2(b[k])) for k in range(n)]
    assert max(r) <= tol
