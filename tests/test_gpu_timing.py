"""Kernel timing and tuning run on the solver's own workspaces: they must
leave nothing behind that changes a later solve. A mixed solve before and
after stag_time_kernels (single and 8-RHS, fp32 and fp64 kernels, run in
the solve's order) and stag_tune gives the same iterations and bits, and an
eager solve with per-kernel events gives them too."""

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


def test_timing_and_tuning_leave_solves_unchanged(stag, monkeypatch):
    monkeypatch.delenv("STAG_TUNE_CACHE", raising=False)
    L, m, tol = (8, 8, 8, 16), 0.05, 1e-9
    U = synth.haar_links(L, 51)
    b = synth.gaussian_rhs(L, 1, 52)
    p = None
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64", "f32"), r12=True)
        p = stag.cg_params(tol=tol, inner="f32", small_lattice=False)
        fb = ctx.field(g, 0, "f64", 1).load(b)

        def solve():
            fx = ctx.field(g, 0, "f64", 1)
            rc, st = stag.stag_cg_solve(ctx, g, [m], fb, fx, p)
            assert rc == 0, st
            return st[0]["iters"], fx.store()

        it0, x0 = solve()
        for prec, n, reps in (("f32", 1, 20), ("f64", 1, 5), ("f32", 8, 5)):
            us = stag.stag_time_kernels(ctx, g, prec, n, reps)
            log("time_kernels", prec, n, [round(u, 2) for u in us])
            assert len(us) == 3 and all(math.isfinite(u) and u > 0 for u in us)
        it1, x1 = solve()
        assert it1 == it0 and np.array_equal(x1, x0)

        cfg, ms = stag.stag_tune(ctx, g, "f32", 1)
        log("tune", cfg, ms)
        assert ms > 0 and stag.stag_tune_get(ctx, "f32", 1, g.vh) == cfg
        it2, x2 = solve()
        assert it2 == it0 and np.array_equal(x2, x0)

        stag.stag_timing_enable(ctx, True)
        it3, x3 = solve()
        n1, ms1 = stag.stag_timing_read(ctx, stag.K_HOP1)
        nu, msu = stag.stag_timing_read(ctx, stag.K_UPDATE)
        stag.stag_timing_enable(ctx, False)
        assert it3 == it0 and np.array_equal(x3, x0)
        assert n1 >= it0 and nu >= it0 and ms1 > 0 and msu > 0

    Ax = oracle_apply_A(U, x0, L, m)
    assert math.sqrt(ostag.norm2(b[0] - Ax[0]) / ostag.norm2(b[0])) <= tol
