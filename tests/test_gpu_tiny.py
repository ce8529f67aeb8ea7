"""GPU parity of the one-workgroup solves of tiny lattices (128 sites per
parity, or up to 648 with several right-hand sides): against the oracle's
solvers and against the kernel-per-stage solver on the same systems."""

import math

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


def solve(stag, ctx, L, U, b, masses, tol, inner="f64", small=True, r12=False, **kw):
    precisions = ("f64",) if inner == "f64" else ("f64", inner)
    g = ctx.gauge(L, U, precisions=precisions, r12=r12)
    fb = ctx.field(g, 0, "f64", b.shape[0]).load(b)
    fx = ctx.field(g, 0, "f64", b.shape[0])
    rc, st = stag.stag_cg_solve(ctx, g, masses, fb, fx,
                                stag.cg_params(tol=tol, inner=inner, small_lattice=small, **kw))
    x = fx.store()
    for o in (fb, fx, g):
        o.destroy()
    return rc, st, x


def true_res(U, L, masses, b, x):
    Ax = oracle_apply_A(U, x, L, masses)
    return [math.sqrt(ostag.norm2(b[r] - Ax[r]) / ostag.norm2(b[r])) for r in range(b.shape[0])]


def test_c1_plain_cg_matches_dense_and_oracle(stag, ctx):
    """4^4 Haar, m = 0.1, 1e-10 in one workgroup: the dense solution and the
    oracle's Fig.1 iteration count."""
    cfg = synth.CONFIGS["c1_4x4x4x4"]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U = synth.config_links("c1_4x4x4x4")
    b = synth.config_rhs("c1_4x4x4x4")
    rc, st, x = solve(stag, ctx, L, U, b, [m], tol)
    log(st)
    assert rc == 0 and st[0]["status"] == 0
    assert true_res(U, L, [m], b, x)[0] <= tol
    A = dense.dense_A_even(U, L, m)
    ev = np.linalg.eigvalsh(A)
    xd = np.linalg.solve(A, b[0].ravel()).reshape(-1, 3)
    assert rel_norm(x[0], xd) <= (ev.max() / ev.min()) * tol
    _, ost = ostag.cg(lambda v: ostag.apply_A(U, v, L, m), b[0], tol)
    assert abs(st[0]["iters"] - ost["iters"]) <= 0.05 * ost["iters"] + 5


@pytest.mark.parametrize("inner", ["f32", "f16s"])
def test_mixed_matches_oracle_emulation(stag, ctx, inner):
    # two right-hand sides: 6^4 runs in one workgroup each only in batches
    L, m, tol = (6, 6, 6, 6), 0.03, 1e-8
    U = links(L, "haar", 81)
    b = np.concatenate([synth.gaussian_rhs(L, 1, 82), synth.gaussian_rhs(L, 1, 83)])
    rc, st, x = solve(stag, ctx, L, U, b, [m, m], tol, inner=inner)
    log(inner, st)
    assert rc == 0
    res = true_res(U, L, [m, m], b, x)[0]
    assert res <= tol
    assert abs(st[0]["true_rel_res"] - res) <= 0.05 * res + 1e-15
    _, est = ostag.mixed_cg(U, L, m, b[0], tol, prec=inner)
    slack = 0.05 if inner == "f32" else 0.25
    assert abs(st[0]["iters"] - est["iters"]) <= slack * est["iters"] + 10
    assert abs(st[0]["reliable_updates"] - est["updates"]) <= 2 + (0 if inner == "f32" else 4)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (6, 6, 6, 6)])
@pytest.mark.parametrize("inner", ["f64", "f32", "f16s"])
def test_one_workgroup_equals_kernel_per_stage(stag, ctx, L, inner):
    """Same systems through both solvers (3 RHS, different masses): both meet
    the true residual, with iteration counts and solutions that agree."""
    tol = 1e-9
    U = links(L, "haar", 91)
    masses = [0.1, 0.05, 0.2]
    b = synth.gaussian_rhs(L, 3, 92)
    rc1, st1, x1 = solve(stag, ctx, L, U, b, masses, tol, inner=inner, small=True)
    rc2, st2, x2 = solve(stag, ctx, L, U, b, masses, tol, inner=inner, small=False)
    log(L, inner, [s["iters"] for s in st1], [s["iters"] for s in st2])
    assert rc1 == 0 and rc2 == 0
    for r in range(3):
        assert max(true_res(U, L, masses, b, x1)) <= tol
        slack = 0.05 if inner != "f16s" else 0.25
        assert abs(st1[r]["iters"] - st2[r]["iters"]) <= slack * st2[r]["iters"] + 5
        assert rel_norm(x1[r], x2[r]) <= 1e-6


def test_restart_variant_and_r12(stag, ctx):
    """The Fig.2 variant and 12-parameter links in one workgroup."""
    L, m, tol = (6, 6, 6, 6), 0.03, 1e-8
    U = links(L, "haar", 81)
    b = np.concatenate([synth.gaussian_rhs(L, 1, 82), synth.gaussian_rhs(L, 1, 83)])
    rc, st, x = solve(stag, ctx, L, U, b, [m, m], tol, inner="f32", r12=True,
                      mixed_variant="restart")
    assert rc == 0 and max(true_res(U, L, [m, m], b, x)) <= tol
    _, est = ostag.refinement_cg(U, L, m, b[0], tol, prec="f32", eps_in=0.1)
    assert abs(st[0]["iters"] - est["iters"]) <= 0.05 * est["iters"] + 10


def test_zero_rhs_breakdown_free_and_cap(stag, ctx):
    """b = 0 gives x = 0 at once; a tiny iteration cap ends with ENOCONV."""
    L = (4, 4, 4, 4)
    U = links(L, "haar", 5)
    b = synth.gaussian_rhs(L, 2, 6)
    b[1] = 0
    rc, st, x = solve(stag, ctx, L, U, b, [0.1, 0.1], 1e-10)
    assert rc == 0 and st[1]["iters"] == 0 and not np.any(x[1])
    rc, st, _ = solve(stag, ctx, L, U, b[:1], [0.05], 1e-12, max_iter=7)
    assert rc == stag.STAG_ENOCONV and st[0]["iters"] == 7
    rc, st, _ = solve(stag, ctx, L, U, b[:1], [0.05], 1e-12, inner="f32", max_iter=7)
    assert rc == stag.STAG_ENOCONV and st[0]["iters"] == 7
