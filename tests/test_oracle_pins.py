"""Pins for the CPU oracle: each check ties the oracle to something other
than itself (brute force, closed forms, invariants, the paper's numbers)."""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import dense, stag

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# ---------------------------------------------------------------- generators

@pytest.mark.parametrize("kind", ["haar", "exp"])
def test_links_are_su3(kind):
    L = (4, 2, 2, 6)
    U = synth.haar_links(L, 1) if kind == "haar" else synth.exp_ih_links(L, 1, 0.5)
    uu = U @ np.conj(np.swapaxes(U, -1, -2))
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    det = np.linalg.det(U)
    assert np.abs(det - 1).max() < 1e-14


def test_haar_moment():
    # For Haar U(3) or SU(3), E|tr U|^2 = 1 (n >= 2 is not a special case).
    u = synth.haar_su3(synth.make_rng(99), (100000,))
    m2 = np.abs(np.trace(u, axis1=-2, axis2=-1)) ** 2
    se = m2.std() / math.sqrt(m2.size)
    assert abs(m2.mean() - 1.0) < 3 * se + 1e-3


def test_exp_links_close_to_identity_for_small_eps():
    U = synth.exp_ih_links((2, 2, 2, 2), 5, 1e-3)
    assert np.abs(U - np.eye(3)).max() < 1e-2


# ---------------------------------------------------------------- operator

@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 2, 4)])
def test_apply_A_matches_dense_bruteforce(L):
    U = synth.haar_links(L, 21)
    A = dense.dense_A_even(U, L, 0.3)
    v = synth.gaussian_rhs(L, 1, 22)[0]
    h = stag.apply_A(U, v, L, 0.3)
    assert rel(h, (A @ v.ravel()).reshape(-1, 3)) < 1e-13


@pytest.mark.parametrize("p_in", [0, 1])
def test_dslash_matches_dense_bruteforce(p_in):
    L = (2, 4, 2, 4)
    U = synth.haar_links(L, 23)
    D = dense.dense_D(U, L)
    e = dense.even_rows(L)
    allr = np.arange(D.shape[0])
    o = np.setdiff1d(allr, e)
    rows_in = e if p_in == 0 else o
    rows_out = o if p_in == 0 else e
    # the odd rows are in lex order too, which is checkerboard order
    v = synth.gaussian_rhs(L, 1, 24)[0]
    out = stag.dslash(U, v, L, p_in)
    ref = D[np.ix_(rows_out, rows_in)] @ v.ravel()
    assert rel(out, ref.reshape(-1, 3)) < 1e-13


def test_free_spectrum_4444():
    L, m = (4, 4, 4, 4), 0.1
    ev = np.linalg.eigvalsh(dense.dense_A_even(synth.unit_links(L), L, m))
    vals, counts = np.unique(np.round(ev, 9), return_counts=True)
    # m^2 + 4k for k = number of directions with sin^2 p = 1, multiplicity 24 C(4, k)
    assert np.allclose(vals, [0.01, 4.01, 8.01, 12.01, 16.01], atol=1e-12)
    assert list(counts) == [24, 96, 144, 96, 24]
    assert np.abs(ev - dense.free_spectrum(L, m)).max() < 1e-12


def test_twisted_gauge_rotated_spectrum():
    L, m = (4, 2, 4, 6), 0.2
    th = np.array([[0.3, 0.1], [0.5, -0.2], [0.7, 0.25], [-0.4, 0.9]])
    U = synth.gauge_transform_links(synth.twisted_links(L, th), synth.random_gauge(L, 31))
    ev = np.linalg.eigvalsh(dense.dense_A_even(U, L, m))
    assert np.abs(ev - dense.twisted_spectrum(L, m, th)).max() < 1e-12


def test_hermitian_positive_2222():
    L, m = (2, 2, 2, 2), 0.1
    A = dense.dense_A_even(synth.haar_links(L, 2), L, m)
    assert np.abs(A - A.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(A).min() >= m * m - 1e-12


def _haar_setup(L=(4, 6, 4, 8), seed=41):
    U = synth.haar_links(L, seed)
    v = synth.gaussian_rhs(L, 2, seed + 1)
    return L, U, v[0], v[1]


def test_hermiticity_and_positivity_identity():
    L, U, a, b = _haar_setup()
    m = 0.07
    Ab = stag.apply_A(U, b, L, m)
    Aa = stag.apply_A(U, a, L, m)
    lhs = stag.vdot(a, Ab)
    rhs = np.conj(stag.vdot(b, Aa))
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    # <chi, A chi> = m^2 |chi|^2 + |D_oe chi|^2
    t = stag.dslash(U, a, L, 0)
    ident = m * m * stag.norm2(a) + stag.norm2(t)
    assert abs(stag.vdot(a, Aa).real - ident) / ident < 1e-13
    assert abs(stag.vdot(a, Aa).imag) / ident < 1e-13


def test_dslash_anti_hermitian():
    L, U, a, _ = _haar_setup()
    phi_o = synth.gaussian_rhs(L, 1, 77)[0]
    lhs = stag.vdot(phi_o, stag.dslash(U, a, L, 0))
    rhs = -stag.vdot(stag.dslash(U, phi_o, L, 1), a)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def _even_g(g, L):
    return stag.from_full(np.zeros(g.shape[:4] + (3,)), L, 0), g.reshape(-1, 3, 3)[stag.parity(L).reshape(-1) == 0]


def test_gauge_covariance():
    L, U, a, _ = _haar_setup()
    m = 0.1
    g = synth.random_gauge(L, 43)
    Ug = synth.gauge_transform_links(U, g)
    _, ge = _even_g(g, L)
    ga = (ge @ a[..., None])[..., 0]
    lhs = stag.apply_A(Ug, ga, L, m)
    rhs = (ge @ stag.apply_A(U, a, L, m)[..., None])[..., 0]
    assert rel(lhs, rhs) < 1e-13


@pytest.mark.parametrize("shift", [(2, 0, 0, 0), (0, 2, 0, 0), (0, 0, 2, 0), (0, 0, 0, 2), (2, 2, 0, 4)])
def test_even_shift_covariance(shift):
    L, U, a, _ = _haar_setup()
    m = 0.1
    axes = (3, 2, 1, 0)

    def sh(f):
        for mu in range(4):
            f = np.roll(f, shift[mu], axis=axes[mu])
        return f

    Us = sh(U)
    a_full = stag.to_full(a, L, 0)
    as_ = stag.from_full(sh(a_full), L, 0)
    lhs = stag.apply_A(Us, as_, L, m)
    rhs = stag.from_full(sh(stag.to_full(stag.apply_A(U, a, L, m), L, 0)), L, 0)
    assert rel(lhs, rhs) < 1e-14


def test_fft_solve_matches_dense_and_operator():
    L, m = (4, 4, 2, 4), 0.3
    b = synth.gaussian_rhs(L, 1, 51)[0]
    A = dense.dense_A_even(synth.unit_links(L), L, m)
    x = dense.fft_solve(b, L, m)
    xd = np.linalg.solve(A, b.ravel()).reshape(-1, 3)
    assert rel(x, xd) < 1e-12
    L2 = (8, 8, 8, 8)
    th = np.array([[0.1, 0.2], [0.3, 0.4], [-0.5, 0.6], [0.7, -0.8]])
    g = synth.random_gauge(L2, 52)
    U = synth.gauge_transform_links(synth.twisted_links(L2, th), g)
    b2 = synth.gaussian_rhs(L2, 1, 53)[0]
    ge = g.reshape(-1, 3, 3)[stag.parity(L2).reshape(-1) == 0]
    gh_b = (np.conj(np.swapaxes(ge, -1, -2)) @ b2[..., None])[..., 0]
    x2 = (ge @ dense.fft_solve(gh_b, L2, m, th)[..., None])[..., 0]
    assert rel(stag.apply_A(U, x2, L2, m), b2) < 1e-12


# ---------------------------------------------------------------- CG (Fig.1)

def test_cg_free_field_terminates_in_five_iterations():
    # A has 5 distinct eigenvalues on the free 4^4 lattice, so exact CG
    # terminates after at most 5 steps.
    L, m = (4, 4, 4, 4), 0.1
    U = synth.unit_links(L)
    b = synth.gaussian_rhs(L, 1, 61)[0]
    x, st = stag.cg(lambda v: stag.apply_A(U, v, L, m), b, 1e-12)
    assert st["status"] == "ok" and st["iters"] <= 5
    assert rel(x, dense.fft_solve(b, L, m)) < 1e-11


def test_cg_haar_4444_matches_dense_solve():
    L, m, tol = (4, 4, 4, 4), 0.1, 1e-10
    U = synth.haar_links(L, 11)
    b = synth.gaussian_rhs(L, 1, 111)[0]
    x, st = stag.cg(lambda v: stag.apply_A(U, v, L, m), b, tol)
    A = dense.dense_A_even(U, L, m)
    assert st["status"] == "ok" and st["true_rel_res"] <= tol
    r = b.ravel() - A @ x.ravel()
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b.ravel())
    ev = np.linalg.eigvalsh(A)
    kappa = ev.max() / ev.min()
    xd = np.linalg.solve(A, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd) <= kappa * tol
    # Fig.1's cap of N iterations is too small in finite precision here
    assert st["iters"] > 3 * 128


def test_cg_zero_rhs():
    L = (2, 2, 2, 2)
    U = synth.haar_links(L, 1)
    x, st = stag.cg(lambda v: stag.apply_A(U, v, L, 0.1), np.zeros((8, 3), complex), 1e-8)
    assert st["iters"] == 0 and not np.any(x)


# ---------------------------------------------------------------- quantisers

def test_f16s_exact_values_roundtrip():
    rng = synth.make_rng(5)
    k = rng.integers(-1024, 1025, size=(50, 3, 2))
    k[:, 0, 0] = 1024  # the largest component sets the scale 2^-3 exactly
    v = (k[..., 0] + 1j * k[..., 1]) * (2.0 ** -13)
    payload, s = stag.f16s_encode(v)
    assert np.all(s == np.float32(2.0 ** -3))
    assert np.array_equal(stag.f16s_decode(payload, s), v.astype(np.complex64))


def test_f16s_rounding_and_bound():
    # with scale 4, (1 + 2^-11) * 2 encodes as 0.5 + 2^-12, half-way between
    # the fp16 neighbours 0.5 and 0.5 + 2^-11: round to nearest even gives 0.5;
    # 0.75 * 2^-11 above 0.5 is past the half-way point and rounds up.
    v = np.array([[4.0, (1 + 2 ** -11) * 2.0, 2.0 + 3 * 2 ** -11]], dtype=np.complex128)
    payload, s = stag.f16s_encode(v)
    assert s[0] == 4.0 and float(payload[0, 0, 0]) == 1.0
    assert float(payload[0, 1, 0]) == 0.5
    assert float(payload[0, 2, 0]) == 0.5 + 2 ** -11
    v2 = synth.gaussian_rhs((4, 4, 4, 4), 1, 6)[0]
    q = stag.q_f16s(v2)
    smax = np.maximum(np.abs(v2.real), np.abs(v2.imag)).max(axis=-1)
    assert np.all(np.abs(q - v2) <= (2.0 ** -11 + 2.0 ** -23) * 2 * smax[:, None])
    zero = stag.q_f16s(np.zeros((3, 3)))
    assert not np.any(zero)


def test_f32_low_operator_error():
    L, m = (4, 4, 4, 4), 0.1
    U = synth.haar_links(L, 71)
    v = synth.gaussian_rhs(L, 1, 72)[0]
    ref = stag.apply_A(U, v, L, m)
    e32 = rel(stag.LowOperator(U, L, m, "f32")(v), ref)
    e16 = rel(stag.LowOperator(U, L, m, "f16s")(v), ref)
    # unit round-offs: fp32 u = 2^-24, fp16 u = 2^-11 (relative to the site max)
    assert 1e-9 < e32 < 1e-6
    assert 1e-5 < e16 < 1e-3


def test_third_row_of_special_unitary_links():
    # for det U = 1 and U U^+ = 1 the third row is the conjugated cross
    # product of the first two (Sec.3.3); Haar links are phase-fixed to det 1
    U = synth.haar_links((4, 4, 4, 4), 75)
    assert np.abs(stag.su3_third_row(U) - U).max() < 1e-14
    # a unitary link with det e^{i phi} gets a third row off by e^{-i phi}
    W = U[0, 0, 0, 0, 0] * np.exp(0.2j)
    r = stag.su3_third_row(W)
    assert np.allclose(r[:2], W[:2], rtol=0, atol=0)
    assert np.allclose(r[2], W[2] * np.exp(-0.6j), atol=1e-14)


@pytest.mark.parametrize("prec,lo,hi", [("f32", 1e-9, 1e-6), ("f16s", 1e-5, 1e-3)])
def test_twelve_parameter_low_operator_error(prec, lo, hi):
    # rebuilding the third row from stored rows adds an error of the order of
    # the storage rounding and no more: within the full-storage bounds and at
    # most twice the full-storage error on the same links and vector
    L, m = (6, 4, 4, 8), 0.1
    U = synth.haar_links(L, 73)
    v = synth.gaussian_rhs(L, 1, 74)[0]
    ref = stag.apply_A(U, v, L, m)
    full = rel(stag.LowOperator(U, L, m, prec)(v), ref)
    r12 = rel(stag.LowOperator(U, L, m, prec, r12=True)(v), ref)
    assert lo < r12 < hi
    assert r12 < 2 * full
    with pytest.raises(ValueError):
        stag.LowOperator(U, L, m, prec, Ulong=U, r12=True)


# ---------------------------------------------------------------- mixed CG (Sec.3)

@pytest.fixture(scope="module")
def mixed_case():
    # m = 0.03 gives ~1600 iterations, enough for the per-update fp64 work
    # to be a small share as in the paper's production solves
    L, m, tol = (6, 6, 6, 6), 0.03, 1e-8
    U = synth.haar_links(L, 81)
    b = synth.gaussian_rhs(L, 1, 82)[0]
    x64, st64 = stag.cg(lambda v: stag.apply_A(U, v, L, m), b, tol)
    return L, m, tol, U, b, st64


def test_mixed_f32_preserves_iterations(mixed_case):
    L, m, tol, U, b, st64 = mixed_case
    claims = json.load(open(os.path.join(GOLDEN, "paper_mixed_claims.json")))
    x, st = stag.mixed_cg(U, L, m, b, tol, prec="f32")
    assert st["status"] == "ok"
    res = math.sqrt(stag.norm2(b - stag.apply_A(U, x, L, m)) / stag.norm2(b))
    assert res <= tol
    assert abs(st["iters"] - st64["iters"]) <= claims["iteration_count_rel_tol"] * st64["iters"]
    share = st["iters"] / (st["iters"] + st["updates"] + 1)
    assert share >= claims["single_precision_share_min"]
    # one update per decade of residual reduction at delta = 0.1
    assert 6 <= st["updates"] <= 12


def test_mixed_f16s_true_residual(mixed_case):
    L, m, tol, U, b, st64 = mixed_case
    x, st = stag.mixed_cg(U, L, m, b, tol, prec="f16s")
    assert st["status"] == "ok"
    res = math.sqrt(stag.norm2(b - stag.apply_A(U, x, L, m)) / stag.norm2(b))
    assert res <= tol


def test_refinement_fig2_converges(mixed_case):
    L, m, tol, U, b, st64 = mixed_case
    x, st = stag.refinement_cg(U, L, m, b, tol, prec="f32")
    assert st["status"] == "ok" and st["true_rel_res"] <= tol
    # without the carried direction each restart loses the Krylov space
    assert st["iters"] >= st64["iters"]


# ---------------------------------------------------------------- paper numbers

def test_update_ablations_agree_when_well_conditioned():
    """Both one-sided update variants of Sec.3.2 are still correct solvers on a
    well-conditioned system far from fp32's limit: all three agree with the
    dense solve and take the same iterations."""
    L, m, tol = (4, 4, 4, 4), 1.0, 1e-5
    U = synth.haar_links(L, 11)
    b = synth.gaussian_rhs(L, 1, 111)[0]
    A = dense.dense_A_even(U, L, m)
    xd = np.linalg.solve(A, b.ravel()).reshape(-1, 3)
    ev = np.linalg.eigvalsh(A)
    iters = set()
    for upd in ("both", "reliable", "fold_only"):
        x, st = stag.mixed_cg(U, L, m, b, tol, prec="f32", update=upd)
        assert st["status"] == "ok", (upd, st)
        res = math.sqrt(stag.norm2(b - stag.apply_A(U, x, L, m)) / stag.norm2(b))
        assert res <= tol
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= (ev.max() / ev.min()) * tol
        iters.add(st["iters"])
    assert len(iters) == 1


def test_both_updates_are_needed():
    """Sec.3.2 applies the reliable and the group-wise update together: near a
    tolerance fp32 cannot hold, replacing the residual alone (the reliable
    update without folding y into x) keeps the solution in fp32 and stalls far
    above it, and folding y into x alone (without the residual recompute)
    lets the iterated residual drift from the true one, which then misses it."""
    L, m, tol = (4, 4, 4, 4), 0.1, 1e-10
    U = synth.haar_links(L, 11)
    b = synth.gaussian_rhs(L, 1, 111)[0]
    _, both = stag.mixed_cg(U, L, m, b, tol, prec="f32")
    assert both["status"] == "ok" and both["true_rel_res"] <= tol
    x, rel = stag.mixed_cg(U, L, m, b, tol, prec="f32", update="reliable")
    assert rel["status"] == "noconv" and rel["true_rel_res"] > 1e3 * tol
    # the reported residual is that of the returned x = x + y
    res = math.sqrt(stag.norm2(b - stag.apply_A(U, x, L, m)) / stag.norm2(b))
    assert abs(res - rel["true_rel_res"]) <= 1e-12
    x, gw = stag.mixed_cg(U, L, m, b, tol, prec="f32", update="fold_only")
    assert gw["status"] == "inaccurate" and gw["true_rel_res"] > 10 * tol
    assert abs(gw["iters"] - both["iters"]) <= 0.05 * both["iters"]


def test_slow_refinement_cycle_ends_the_fp16_pass():
    """With fp16 storage on a system it cannot refine well (8^4 Haar,
    m = 0.01: kappa u16 >> 1) the first refinement cycle reduces the iterated
    residual tenfold but the true residual by less than half, so slow_ratio
    ends the pass there (without it the same iteration runs on past the cap,
    where plain fp16 refinement needs over 13 000 iterations); on a system fp16
    does refine, slow_ratio changes nothing."""
    L, m, tol = (8, 8, 8, 8), 0.01, 1e-10
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 1, 1001)[0]
    _, slow = stag.mixed_cg(U, L, m, b, tol, prec="f16s", max_stall=3, slow_ratio=0.5)
    assert slow["status"] == "stall" and slow["updates"] == 1 and slow["restarts"] == 0
    assert 0.5 < slow["true_rel_res"] < 1.0
    _, capped = stag.mixed_cg(U, L, m, b, tol, prec="f16s", max_stall=3,
                              max_iter=slow["iters"] + 50)
    assert capped["status"] == "noconv" and capped["updates"] >= 1
    L, m, tol = (4, 4, 4, 4), 0.5, 1e-8
    U = synth.haar_links(L, 11)
    b = synth.gaussian_rhs(L, 1, 111)[0]
    x1, a = stag.mixed_cg(U, L, m, b, tol, prec="f16s", slow_ratio=0.5)
    x2, c = stag.mixed_cg(U, L, m, b, tol, prec="f16s")
    assert a == c and a["status"] == "ok" and np.array_equal(x1, x2)


def test_cg_budget_ends_an_fp16_pass_that_lags_cg():
    """The iteration budget of the CG convergence bound (6^4 Haar links,
    1e-8). fp32 refinement keeps within the bound itself (the bound holds
    for CG, and the budget's formula would exceed it with a factor or a term
    dropped). fp16 storage at m = 0.05 keeps within twice it, so the budget
    changes nothing. At m = 0.02 every fp16 cycle still contracts the true
    residual tenfold, but at 3x the iterations CG needs (7 131 iterations in
    all against fp32's 2 419), so the budget ends the pass."""
    L = (6, 6, 6, 6)
    U = synth.haar_links(L, 15)
    b = synth.gaussian_rhs(L, 1, 1001)[0]
    _, f32 = stag.mixed_cg(U, L, 0.02, b, 1e-8, prec="f32", r12=True, cg_budget=1.2)
    assert f32["status"] == "ok"
    _, lag = stag.mixed_cg(U, L, 0.02, b, 1e-8, prec="f16s", r12=True, cg_budget=2.0)
    assert lag["status"] == "stall" and lag["restarts"] == 0
    assert 2 <= lag["updates"] <= 6 and lag["iters"] < 0.6 * 7131
    assert lag["true_rel_res"] < 1e-2
    x1, a = stag.mixed_cg(U, L, 0.05, b, 1e-8, prec="f16s", r12=True, cg_budget=2.0)
    x2, c = stag.mixed_cg(U, L, 0.05, b, 1e-8, prec="f16s", r12=True)
    assert a == c and a["status"] == "ok" and np.array_equal(x1, x2)


def test_paper_cost_model_golden():
    g = json.load(open(os.path.join(GOLDEN, "paper_cost_model.json")))
    reals = 8 * 18 + 8 * 6 + 6
    assert reals * 8 == g["bytes_per_site_D_fp64"]
    from paper_1111_0125_amd import costs
    assert costs.paper_d_bytes_per_site("f64") == g["bytes_per_site_D_fp64"]
    assert 8 * 9 * 8 == g["flops_per_site_D"]
    Lx, Ly, Lz, Lt = g["lattice"]
    ve = Lx * Ly * Lz * Lt // 2
    assert math.floor(ve * g["flops_per_site_D"] / 1e8) / 10 == g["gflop_per_D_even"]
    assert math.floor(ve * g["bytes_per_site_D_fp64"] / 1e8) / 10 == g["gbyte_per_D_even"]


# ---------------------------------------------------------------- C oracle

@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 4, 8), (8, 8, 8, 8)])
def test_c_oracle_matches_numpy(L):
    from oracle import c as oc
    U = synth.haar_links(L, 91)
    v = synth.gaussian_rhs(L, 1, 92)[0]
    assert rel(oc.apply_A(U, v, L, 0.05), stag.apply_A(U, v, L, 0.05)) < 1e-13
    for p in (0, 1):
        assert rel(oc.dslash(U, v, L, p), stag.dslash(U, v, L, p)) < 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 2, 4, 2), (4, 6, 2, 8)])
def test_c_oracle_improved_matches_numpy(L):
    from oracle import c as oc
    fat = synth.gaussian_links(L, 301)
    lng = synth.gaussian_links(L, 302)
    v = synth.gaussian_rhs(L, 1, 303)[0]
    assert rel(oc.apply_A(fat, v, L, 0.05, Ulong=lng),
               stag.apply_A(fat, v, L, 0.05, Ulong=lng)) < 1e-13
    for p in (0, 1):
        assert rel(oc.dslash(fat, v, L, p, Ulong=lng), stag.dslash(fat, v, L, p, Ulong=lng)) < 1e-13


def test_c_oracle_cg():
    from oracle import c as oc
    L, m, tol = (4, 4, 4, 4), 0.1, 1e-10
    U = synth.haar_links(L, 11)
    b = synth.gaussian_rhs(L, 1, 111)[0]
    x, st = oc.cg(U, b, L, m, tol)
    assert st["status"] == "ok" and st["true_rel_res"] <= tol
    xd = np.linalg.solve(dense.dense_A_even(U, L, m), b.ravel()).reshape(-1, 3)
    assert rel(x, xd) < 1e-6


# ---------------------------------------------------------------- improved operator

# The improved (fat-link + three-hop) operator extends Eq.5 by the terms
# eta N(x) chi(x+3mu) - eta N(x-3mu)^+ chi(x-3mu) with caller-supplied long
# links N. Extents 4 alias x+3mu with x-mu, extent 6 aliases x+3mu with
# x-3mu and extent 2 folds all four onto one neighbour.

@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 2, 4, 2)])
@pytest.mark.parametrize("p_in", [0, 1])
def test_improved_dslash_matches_dense_bruteforce(L, p_in):
    fat = synth.gaussian_links(L, 201)
    lng = synth.gaussian_links(L, 202)
    D = dense.dense_D(fat, L, lng)
    e = dense.even_rows(L)
    o = np.setdiff1d(np.arange(D.shape[0]), e)
    rows_in, rows_out = (e, o) if p_in == 0 else (o, e)
    v = synth.gaussian_rhs(L, 1, 203)[0]
    out = stag.dslash(fat, v, L, p_in, Ulong=lng)
    ref = D[np.ix_(rows_out, rows_in)] @ v.ravel()
    assert rel(out, ref.reshape(-1, 3)) < 1e-13
    # the three-hop terms really contribute
    assert rel(stag.dslash(fat, v, L, p_in), ref.reshape(-1, 3)) > 1e-2


def test_improved_dense_is_anti_hermitian_and_A_positive():
    L, m = (4, 2, 6, 2), 0.2
    fat = synth.gaussian_links(L, 211)
    lng = synth.gaussian_links(L, 212)
    D = dense.dense_D(fat, L, lng)
    assert np.abs(D + D.conj().T).max() < 1e-14
    A = dense.dense_A_even(fat, L, m, lng)
    assert np.abs(A - A.conj().T).max() < 1e-13
    assert np.linalg.eigvalsh(A).min() >= m * m - 1e-12


def test_improved_free_spectrum_twisted_and_rotated():
    # fat = c1 U, long = c3 U U U for constant diagonal U, gauge rotated:
    # eigenvalues m^2 + sum_mu 4 (c1 sin q + c3 sin 3q)^2
    L, m = (4, 6, 4, 4), 0.15
    th = np.array([[0.3, 0.1], [0.5, -0.2], [0.7, 0.25], [-0.4, 0.9]])
    U = synth.gauge_transform_links(synth.twisted_links(L, th), synth.random_gauge(L, 221))
    fat, lng = synth.naik_links(U)
    ev = np.linalg.eigvalsh(dense.dense_A_even(fat, L, m, lng))
    ref = dense.twisted_spectrum(L, m, th, naik=(synth.NAIK_C1, synth.NAIK_C3))
    assert np.abs(ev - ref).max() < 1e-12
    # and not the one-hop spectrum with the fat links alone
    assert np.abs(ev - dense.twisted_spectrum(L, m, th)).max() > 1e-2


def test_naik_coefficients_cancel_leading_error():
    # the improved symbol 2 (c1 sin p + c3 sin 3p) = 2p + O(p^5)
    p = np.array([1e-2, 2e-2])
    sym = 2 * (synth.NAIK_C1 * np.sin(p) + synth.NAIK_C3 * np.sin(3 * p))
    err = np.abs(sym - 2 * p)
    assert np.all(err < 2 * p ** 5)
    assert abs(math.log2(err[1] / err[0]) - 5) < 0.05


def test_improved_gauge_covariance():
    L, m = (4, 6, 4, 8), 0.1
    fat = synth.gaussian_links(L, 231)
    lng = synth.gaussian_links(L, 232)
    a = synth.gaussian_rhs(L, 1, 233)[0]
    g = synth.random_gauge(L, 234)
    fg = synth.gauge_transform_links(fat, g)
    lg = synth.gauge_transform_links(lng, g, dist=3)
    ge = g.reshape(-1, 3, 3)[stag.parity(L).reshape(-1) == 0]
    lhs = stag.apply_A(fg, (ge @ a[..., None])[..., 0], L, m, Ulong=lg)
    rhs = (ge @ stag.apply_A(fat, a, L, m, Ulong=lng)[..., None])[..., 0]
    assert rel(lhs, rhs) < 1e-13


def test_improved_cg_matches_fft_solve():
    L, m, tol = (8, 8, 8, 8), 0.05, 1e-12
    th = np.array([[0.1, 0.2], [0.3, 0.4], [-0.5, 0.6], [0.7, -0.8]])
    g = synth.random_gauge(L, 241)
    fat, lng = synth.naik_links(synth.gauge_transform_links(synth.twisted_links(L, th), g))
    b = synth.gaussian_rhs(L, 1, 242)[0]
    x, st = stag.cg(lambda v: stag.apply_A(fat, v, L, m, Ulong=lng), b, tol)
    assert st["status"] == "ok"
    ge = g.reshape(-1, 3, 3)[stag.parity(L).reshape(-1) == 0]
    gh_b = (np.conj(np.swapaxes(ge, -1, -2)) @ b[..., None])[..., 0]
    xe = (ge @ dense.fft_solve(gh_b, L, m, th, naik=(synth.NAIK_C1, synth.NAIK_C3))[..., None])[..., 0]
    assert rel(x, xe) < 1e-9


def test_improved_low_operator_error():
    L, m = (4, 4, 4, 6), 0.1
    fat, lng = synth.naik_links(synth.haar_links(L, 251), fat_noise=0.05, seed=252)
    v = synth.gaussian_rhs(L, 1, 253)[0]
    ref = stag.apply_A(fat, v, L, m, Ulong=lng)
    e32 = rel(stag.LowOperator(fat, L, m, "f32", lng)(v), ref)
    e16 = rel(stag.LowOperator(fat, L, m, "f16s", lng)(v), ref)
    assert 1e-9 < e32 < 1e-6
    assert 1e-5 < e16 < 1e-3
    # one fp16 scale per site covers its fat and its long links
    def amax(W):  # over the links stored at each site, after rounding to fp32
        W = W.astype(np.complex64)
        return np.maximum(np.abs(W.real), np.abs(W.imag)).max(axis=(-1, -2, -3))
    s = stag.f16s_link_scale(fat, L, lng)
    assert np.all(s >= amax(lng)) and np.all(s >= amax(fat))


def test_shared_fp16_scale_keeps_long_links_significands():
    """The long links are about 27 times smaller than the fat links sharing
    their site scale, but fp16 is a floating format: N / s sits far above the
    fp16 normal range's lower end (6.1e-5), so it keeps its 11-bit significand
    and a scale of its own would lower its rounding error by far less than a
    factor 2 (not the 2^5 a fixed-point format would lose)."""
    L = (4, 4, 4, 6)
    fat, lng = synth.naik_links(synth.haar_links(L, 251), fat_noise=0.05, seed=252)
    shared = stag.f16s_link_scale(fat, L, lng)
    own = stag.f16s_link_scale(lng, L)  # long links alone (their own maximum)
    ratio = (own / shared).astype(np.float64)
    assert 0.02 < ratio.min() and ratio.max() < 0.06
    nmu = lng[..., 0, :, :]
    q = lambda s_: stag._q_link_f16(nmu.astype(np.complex64), s_)
    small = np.abs(nmu) > 1e-3 * np.abs(nmu).max()
    rel_shared = (np.abs(q(shared) - nmu) / np.abs(nmu))[small].max()
    rel_own = (np.abs(q(own) - nmu) / np.abs(nmu))[small].max()
    assert rel_shared < 2.0 ** -10 and rel_own < 2.0 ** -10
    assert rel_shared < 2.0 * rel_own


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_improved_mixed_cg_true_residual(prec):
    L, m, tol = (6, 6, 6, 6), 0.05, 1e-10
    fat, lng = synth.naik_links(synth.haar_links(L, 261), fat_noise=0.05, seed=262)
    b = synth.gaussian_rhs(L, 1, 263)[0]
    _, st64 = stag.cg(lambda v: stag.apply_A(fat, v, L, m, Ulong=lng), b, tol)
    x, st = stag.mixed_cg(fat, L, m, b, tol, prec=prec, Ulong=lng)
    assert st["status"] == "ok" and st["true_rel_res"] <= tol
    r = b - stag.apply_A(fat, x, L, m, Ulong=lng)
    assert math.sqrt(stag.norm2(r) / stag.norm2(b)) <= tol
    if prec == "f32":
        assert st["iters"] <= 1.1 * st64["iters"]


# ---------------------------------------------------------------- pins bite

def _mut_no_dagger(u, v):
    return (u @ v[..., :, None])[..., 0]


def _mut_transpose_only(u, v):
    return (np.swapaxes(u, -1, -2) @ v[..., :, None])[..., 0]


def _mut_eta_ones(L):
    Lx, Ly, Lz, Lt = L
    return np.ones((4, Lt, Lz, Ly, Lx))


def _mut_eta_own_coord(L):
    x, y, z, t = stag.coords(L)
    Lx, Ly, Lz, Lt = L
    shp = (Lt, Lz, Ly, Lx)
    return np.stack([np.broadcast_to((-1.0) ** c, shp) for c in (x, y, z, t)])


@pytest.mark.parametrize("mutation", [
    ("_mhv", _mut_no_dagger),
    ("_mhv", _mut_transpose_only),
    ("eta", _mut_eta_ones),
    ("eta", _mut_eta_own_coord),
    ("MU_AXIS", (2, 3, 1, 0)),
    ("MU_AXIS", (0, 1, 2, 3)),
])
def test_pins_catch_planted_mistakes(monkeypatch, mutation):
    """Each plausible mistake planted in the oracle makes a pin fail."""
    name, value = mutation
    monkeypatch.setattr(stag, name, value)
    failures = 0
    # brute force from Eq.4 (independent of the patched helpers)
    L = (2, 4, 2, 4)
    U = synth.haar_links(L, 21)
    v = synth.gaussian_rhs(L, 1, 22)[0]
    monkeypatch.undo()
    A = dense.dense_A_even(U, L, 0.3)
    monkeypatch.setattr(stag, name, value)
    if rel(stag.apply_A(U, v, L, 0.3), (A @ v.ravel()).reshape(-1, 3)) > 1e-13:
        failures += 1
    # free-field closed form on an anisotropic lattice: x = A^{-1} b by FFT
    L2 = (4, 2, 6, 4)
    b = synth.gaussian_rhs(L2, 1, 5)[0]
    monkeypatch.undo()
    x = dense.fft_solve(b, L2, 0.3)
    monkeypatch.setattr(stag, name, value)
    if rel(stag.apply_A(synth.unit_links(L2), x, L2, 0.3), b) > 1e-12:
        failures += 1
    assert failures >= 1
