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
    """With full links and with the 12-parameter f64 / f32 copies the
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
