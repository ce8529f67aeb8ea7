"""The 32^3 x 64 workload: Haar links, m = 0.005, one complex Gaussian
right-hand side, true residual 1e-10. The corrected mixed-precision CG of
Sec.3.2 with fp16-with-scale storage (fp32 arithmetic) and with fp32, and
plain fp64 CG (Fig.1) for comparison; every answer is checked with the C
oracle's fp64 A."""

import math

import pytest

import synth
from oracle import stag as ostag
from tests.gpu_common import log, oracle_apply_A

pytestmark = pytest.mark.gpu

NAME = "c3_32x32x32x64"


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


@pytest.fixture(scope="module")
def problem():
    cfg = synth.CONFIGS[NAME]
    log("generating", NAME)
    return cfg, synth.config_links(NAME), synth.config_rhs(NAME)


@pytest.mark.parametrize("inner,r12", [("f16s", False), ("f32", False), ("f64", False),
                                       ("f16s", True), ("f32", True), ("f64", True)])
def test_c3_solve_true_residual(stag, problem, inner, r12):
    """With full links and with the 12-parameter copies the benchmark
    solves on; the oracle's A uses the uncompressed links."""
    cfg, U, b = problem
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32", "f16s"), r12=r12)
        fb = ctx.field(g, 0, "f64", 1).load(b)
        fx = ctx.field(g, 0, "f64", 1)
        rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, stag.cg_params(tol=tol, inner=inner))
        log(inner, "r12" if r12 else "full", rc, st[0])
        assert rc == 0, st
        x = fx.store()
    r = b - oracle_apply_A(U, x, L, m)
    res = math.sqrt(ostag.norm2(r[0]) / ostag.norm2(b[0]))
    log(inner, "true residual (oracle A)", res)
    assert res <= tol
    # the library's own fp64 residual agrees with the oracle's
    assert abs(st[0]["true_rel_res"] - res) <= 0.05 * res + 1e-14


@pytest.mark.parametrize("inner", ["f32", "f64"])
def test_c3_improved_solve_true_residual(stag, problem, inner):
    """The improved operator on the same 32^3 x 64 Haar links (fat = 9/8 U +
    0.05 complex normal noise, long = -1/24 U U U), m = 0.01, 1e-10, as the
    benchmark runs it: the answer checked with the C oracle's fp64 A."""
    cfg, U, b = problem
    L, m, tol = cfg["L"], 0.01, 1e-10
    fat, lng = synth.naik_links(U, fat_noise=0.05, seed=cfg["gauge_seed"] + 100)
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, fat, precisions=("f64", "f32"), long=lng)
        fb = ctx.field(g, 0, "f64", 1).load(b)
        fx = ctx.field(g, 0, "f64", 1)
        rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, stag.cg_params(tol=tol, inner=inner))
        log("improved", inner, rc, st[0])
        assert rc == 0, st
        x = fx.store()
    from oracle import c as oc
    r = b[0] - oc.apply_A(fat, x[0], L, m, Ulong=lng)
    res = math.sqrt(ostag.norm2(r) / ostag.norm2(b[0]))
    log(inner, "true residual (oracle A)", res)
    assert res <= tol
    assert abs(st[0]["true_rel_res"] - res) <= 0.05 * res + 1e-14
