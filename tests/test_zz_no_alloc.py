"""stag_apply_A_noalloc, the variant of stag_apply_A for callers that cannot
allocate device memory: through the C ABI, its output equals stag_apply_A's
bit for bit (the same kernels; the intermediate sits in the library's device
scratch instead of a stream-ordered allocation), on two calls in a row, the
second with a smaller input, and against the oracle's A within the
precision's tolerance; inputs beyond the scratch are refused."""

import numpy as np
import pytest

import synth
from tests.gpu_common import links, log, oracle_apply_A, rel_max

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "f16s": 1e-3}


@pytest.fixture(scope="module")
def stag():
    import paper_1111_0125_amd as s
    return s


@pytest.mark.parametrize("r12", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16s"])
def test_noalloc_equals_apply_A_twice(stag, prec, r12):
    # first call: 16^3 x 8 with 3 right-hand sides (kernels of 2 and 1),
    # second: a smaller 8^3 x 4 lattice with 1 right-hand side
    cases = [((16, 16, 16, 8), 3, [0.1, 0.05, 0.3], 7), ((8, 8, 8, 4), 1, [0.2], 9)]
    with stag.Context(0) as ctx:
        for L, n, masses, seed in cases:
            log("noalloc", prec, "r12" if r12 else "full", L, n)
            U = links(L, "haar", seed)
            g = ctx.gauge(L, U, precisions=(prec,), r12=r12)
            v = synth.gaussian_rhs(L, n, seed + 1)
            fi = ctx.field(g, 0, prec, n).load(v)
            fa = ctx.field(g, 0, prec, n)
            fb = ctx.field(g, 0, prec, n)
            stag.stag_apply_A(ctx, g, masses, fi, fa)
            stag.stag_apply_A_noalloc(ctx, g, masses, fi, fb)
            a, b = fa.store(), fb.store()
            assert np.array_equal(a, b), (prec, L, float(np.abs(a - b).max()))
            ref = oracle_apply_A(U, v, L, np.array(masses))
            err = rel_max(b, ref)
            log("   oracle rel err", err)
            assert err <= TOL[prec]
            for f in (fi, fa, fb, g):
                f.destroy()


def test_noalloc_refuses_input_beyond_scratch(stag):
    """24^3 x 48 has 331776 sites per parity: four fp64 right-hand sides need
    a 63.7 MB intermediate, more than the 48 MiB scratch (EINVAL, nothing
    launched); three (47.8 MB) fit."""
    L = (24, 24, 24, 48)
    U = synth.unit_links(L)
    vh = 24 * 24 * 24 * 48 // 2
    assert 4 * vh * 48 > stag.NOALLOC_SCRATCH_BYTES >= 3 * vh * 48
    with stag.Context(0) as ctx:
        g = ctx.gauge(L, U, precisions=("f64",))
        v = synth.gaussian_rhs(L, 4, 5)
        fi = ctx.field(g, 0, "f64", 4).load(v)
        fo = ctx.field(g, 0, "f64", 4)
        with pytest.raises(stag.StagError) as ei:
            stag.stag_apply_A_noalloc(ctx, g, [0.1] * 4, fi, fo)
        assert ei.value.code == stag.STAG_EINVAL
        assert "scratch" in ctx.last_error()
        f3 = ctx.field(g, 0, "f64", 3).load(v[:3])
        o3 = ctx.field(g, 0, "f64", 3)
        o3r = ctx.field(g, 0, "f64", 3)
        stag.stag_apply_A_noalloc(ctx, g, [0.1] * 3, f3, o3)
        stag.stag_apply_A(ctx, g, [0.1] * 3, f3, o3r)
        assert np.array_equal(o3.store(), o3r.store())
