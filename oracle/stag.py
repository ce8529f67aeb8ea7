"""numpy fp64 oracle: staggered Dirac operator, normal operator and CG solvers.

TEST INFRASTRUCTURE (see the package docstring): used by tests, the smoke
check and the benchmark's CPU-baseline leg only.

Conventions (the paper does not state them; these are the readings used):

* lattice L = (Lx, Ly, Lz, Lt), all extents even, periodic in all four
  directions; arrays are indexed [t, z, y, x];
* parity of a site = (x + y + z + t) mod 2; "even sites" have parity 0
  (Sec.2, the operator is applied over the even sites);
* the staggered phase multiplied into the link U_mu (Sec.2, text after
  Eq.5) is eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) with mu = 0..3 = x, y, z, t;
* even-site vectors are stored in lexicographic order of the even sites,
  which is the checkerboard index lex // 2;
* D has no factor 1/2 (Eq.4-5 as printed), so for unit links the even-even
  block of A = -D^2 + m^2 has eigenvalues m^2 + 4 sum_mu sin^2 p_mu.
"""

from __future__ import annotations

import math

import numpy as np

MU_AXIS = (3, 2, 1, 0)  # array axis of direction mu in [t, z, y, x] arrays


# --------------------------------------------------------------------------
# Lattice bookkeeping
# --------------------------------------------------------------------------

def extents(L):
    L = tuple(int(v) for v in L)
    if len(L) != 4 or any(v < 2 or v % 2 for v in L):
        raise ValueError(f"bad lattice extents {L}")
    return L


def coords(L):
    """Broadcastable coordinate arrays x, y, z, t over [t, z, y, x]."""
    Lx, Ly, Lz, Lt = extents(L)
    x = np.arange(Lx).reshape(1, 1, 1, Lx)
    y = np.arange(Ly).reshape(1, 1, Ly, 1)
    z = np.arange(Lz).reshape(1, Lz, 1, 1)
    t = np.arange(Lt).reshape(Lt, 1, 1, 1)
    return x, y, z, t


def parity(L):
    x, y, z, t = coords(L)
    Lx, Ly, Lz, Lt = L
    return np.broadcast_to((x + y + z + t) % 2, (Lt, Lz, Ly, Lx))


def eta(L):
    """Staggered phases eta_mu(x), shape (4, Lt, Lz, Ly, Lx), values +-1."""
    x, y, z, t = coords(L)
    Lx, Ly, Lz, Lt = L
    shp = (Lt, Lz, Ly, Lx)
    e = np.empty((4,) + shp)
    e[0] = 1.0
    e[1] = np.broadcast_to((-1.0) ** x, shp)
    e[2] = np.broadcast_to((-1.0) ** (x + y), shp)
    e[3] = np.broadcast_to((-1.0) ** (x + y + z), shp)
    return e


def num_half(L):
    Lx, Ly, Lz, Lt = extents(L)
    return Lx * Ly * Lz * Lt // 2


def to_full(v, L, p):
    """Embed a parity-p vector (Vh, 3) into a full-lattice field (zeros elsewhere)."""
    Lx, Ly, Lz, Lt = extents(L)
    full = np.zeros((Lx * Ly * Lz * Lt, 3), dtype=np.result_type(v.dtype, np.complex64))
    mask = parity(L).reshape(-1) == p
    full[mask] = v
    return full.reshape(Lt, Lz, Ly, Lx, 3)


def from_full(full, L, p):
    """The parity-p sites of a full-lattice field, in checkerboard order."""
    mask = parity(L).reshape(-1) == p
    return full.reshape(-1, 3)[mask]


# --------------------------------------------------------------------------
# Dirac operator, Eq.4-5, and the normal operator, Eq.2-3
# --------------------------------------------------------------------------

def _mv(u, v):
    """Colour matrix times colour vector at every site."""
    return (u @ v[..., :, None])[..., 0]


def _mhv(u, v):
    """Colour matrix dagger times colour vector at every site."""
    return (np.conj(np.swapaxes(u, -1, -2)) @ v[..., :, None])[..., 0]


def dslash_full(U, chi, L, dtype=np.complex128, Ulong=None):
    """(D chi)(x) = sum_mu eta_mu(x) U_mu(x) chi(x+mu) - eta_mu(x-mu) U_mu(x-mu)^+ chi(x-mu).

    Eq.5 with the phases of Sec.2 multiplied into the links; chi is a
    full-lattice field [t, z, y, x, c]. Both hops are accumulated, so on an
    extent-2 direction (where x+mu and x-mu coincide) both terms count.
    ``dtype`` selects the arithmetic (complex64 emulates fp32 arithmetic).

    With ``Ulong`` (the improved operator: U then holds the fat links) the
    three-hop terms eta_mu(x) N_mu(x) chi(x+3mu) - eta_mu(x-3mu) N_mu(x-3mu)^+
    chi(x-3mu) are added, N being the caller's long links (products of three
    links along mu with the Naik coefficient folded in). The phase does not
    depend on x_mu, so eta_mu(x-3mu) = eta_mu(x).
    """
    L = extents(L)
    e = eta(L).astype(np.float32 if dtype == np.complex64 else np.float64)
    chi = chi.astype(dtype, copy=False)
    out = np.zeros_like(chi)
    for mu in range(4):
        ax = MU_AXIS[mu]
        uf = (e[mu][..., None, None] * U[..., mu, :, :]).astype(dtype, copy=False)
        out += _mv(uf, np.roll(chi, -1, axis=ax))
        out -= np.roll(_mhv(uf, chi), 1, axis=ax)
        if Ulong is not None:
            nf = (e[mu][..., None, None] * Ulong[..., mu, :, :]).astype(dtype, copy=False)
            out += _mv(nf, np.roll(chi, -3, axis=ax))
            out -= np.roll(_mhv(nf, chi), 3, axis=ax)
    return out


def dslash(U, v, L, p_in, Ulong=None):
    """Parity-to-parity Dirac operator: D_oe for p_in = 0, D_eo for p_in = 1.

    v has shape (Vh, 3) on parity p_in; the result lives on parity 1 - p_in
    (a three-hop also changes parity). Ulong: the improved operator.
    """
    return from_full(dslash_full(U, to_full(v, L, p_in), L, Ulong=Ulong), L, 1 - p_in)


def apply_A(U, chi_e, L, m, Ulong=None):
    """h = A chi with A = -D^2 + m^2 (Eq.2-3), chi and h on even sites.

    D maps each parity to the other, so on even sites -D^2 = -D_eo D_oe.
    Ulong: the improved operator (U then holds the fat links).
    """
    full = to_full(chi_e, L, 0)
    dd = dslash_full(U, dslash_full(U, full, L, Ulong=Ulong), L, Ulong=Ulong)
    return m * m * chi_e - from_full(dd, L, 0)


# --------------------------------------------------------------------------
# Fig.1 conjugate gradient, fp64
# --------------------------------------------------------------------------

def vdot(a, b):
    """<a, b> = sum conj(a) b in fp64."""
    return np.vdot(a.astype(np.complex128).ravel(), b.astype(np.complex128).ravel())


def norm2(a):
    return float(vdot(a, a).real)


def default_max_iter(n_unknowns):
    # Fig.1 caps the loop at the dimension N; finite precision needs more.
    return int(min(10 * n_unknowns, 1_000_000))


def cg(apply, b, tol, max_iter=None, x0=None):
    """Plain CG of Fig.1 in fp64 for one right-hand side.

    The stopping test is relative to |b| (Fig.1 uses |r_0|, identical for
    x0 = 0). When the iterated residual meets it, the true residual b - A x
    is recomputed; if that misses the tolerance the iteration restarts from
    it (r = b - A x, d = r), otherwise the solve ends.
    Returns (x, stats dict).
    """
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    max_iter = default_max_iter(n) if not max_iter or max_iter <= 0 else max_iter
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bb = norm2(b)
    stats = dict(iters=0, restarts=0, status="ok")
    if bb == 0.0:
        stats.update(true_rel_res=0.0, iter_rel_res=0.0)
        return np.zeros_like(b), stats
    stop = tol * tol * bb
    r = b - apply(x)
    d = r.copy()
    delta_new = norm2(r)
    i = 0
    while True:
        while i < max_iter and delta_new > stop:
            q = apply(d)
            dq = vdot(d, q).real
            if not (dq > 0.0 and math.isfinite(dq)):
                stats["status"] = "breakdown"
                break
            alpha = delta_new / dq
            x = x + alpha * d
            r = r - alpha * q
            delta_old = delta_new
            delta_new = norm2(r)
            beta = delta_new / delta_old
            d = r + beta * d
            i += 1
        true_r = b - apply(x)
        true_rr = norm2(true_r)
        if stats["status"] != "ok" or true_rr <= stop or i >= max_iter:
            break
        r = true_r
        d = r.copy()
        delta_new = true_rr
        stats["restarts"] += 1
    stats["iters"] = i
    stats["true_rel_res"] = math.sqrt(true_rr / bb)
    stats["iter_rel_res"] = math.sqrt(delta_new / bb)
    if stats["status"] == "ok" and true_rr > stop:
        stats["status"] = "noconv"
    return x, stats


# --------------------------------------------------------------------------
# Storage quantisers for the low-precision inner solver
# --------------------------------------------------------------------------

def q_f32(v):
    """Round to fp32 storage (round to nearest even)."""
    return np.asarray(v).astype(np.complex64)


def f16s_encode(v):
    """FP16 storage with one fp32 scale per site.

    v has shape (..., 3) (one colour vector per site). The value is first
    rounded to fp32; the site scale s is the largest |Re| or |Im| of the six
    reals; the payload is half(re/s), half(im/s) with the division done in
    fp32 and rounding to nearest even. s = 0 encodes zeros.
    Returns (payload float16 array (..., 3, 2), scale float32 array (...)).
    """
    v32 = np.asarray(v).astype(np.complex64)
    re = v32.real.astype(np.float32)
    im = v32.imag.astype(np.float32)
    s = np.maximum(np.abs(re).max(axis=-1), np.abs(im).max(axis=-1)).astype(np.float32)
    safe = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    pr = (re / safe[..., None]).astype(np.float32).astype(np.float16)
    pi = (im / safe[..., None]).astype(np.float32).astype(np.float16)
    zero = s == 0
    pr[zero] = 0
    pi[zero] = 0
    return np.stack([pr, pi], axis=-1), s


def f16s_decode(payload, s):
    """fp32 value = float(payload) * s, computed in fp32."""
    p32 = payload.astype(np.float32)
    re = (p32[..., 0] * s[..., None]).astype(np.float32)
    im = (p32[..., 1] * s[..., None]).astype(np.float32)
    return (re + 1j * im).astype(np.complex64)


def q_f16s(v):
    payload, s = f16s_encode(v)
    return f16s_decode(payload, s)


def quantiser(prec):
    if prec == "f32":
        return q_f32
    if prec == "f16s":
        return q_f16s
    raise ValueError(prec)


def f16s_link_scale(U, L, Ulong=None):
    """Per-site scale for fp16 links.

    A site x of either parity reads, in the hop stage that produces x, the
    four links U_mu(x) and the four links U_mu(x - mu); its scale is the
    largest |Re| or |Im| over those 144 reals, rounded to fp32. The improved
    operator also reads N_mu(x) and N_mu(x - 3mu), and the scale covers
    those 288 reals.
    """
    def amax(W):
        W32 = W.astype(np.complex64)
        return np.maximum(np.abs(W32.real), np.abs(W32.imag)).max(axis=(-1, -2))  # [t,z,y,x,mu]

    a = amax(U)
    s = a.max(axis=-1)
    for mu in range(4):
        s = np.maximum(s, np.roll(a[..., mu], 1, axis=MU_AXIS[mu]))
    if Ulong is not None:
        n = amax(Ulong)
        s = np.maximum(s, n.max(axis=-1))
        for mu in range(4):
            s = np.maximum(s, np.roll(n[..., mu], 3, axis=MU_AXIS[mu]))
    return s.astype(np.float32)


def _q_link_f16(u32, s):
    safe = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)[..., None, None]
    re = (u32.real.astype(np.float32) / safe).astype(np.float32).astype(np.float16)
    im = (u32.imag.astype(np.float32) / safe).astype(np.float32).astype(np.float16)
    return ((re.astype(np.float32) * safe).astype(np.float32)
            + 1j * (im.astype(np.float32) * safe).astype(np.float32)).astype(np.complex64)


def su3_third_row(W):
    """The link with its third row replaced by the conjugated cross product
    of its first two, computed in W's precision (Sec.3.3, link compression:
    for a special unitary 3x3 matrix the third row follows from the other
    two, so only twelve real parameters need storing)."""
    a, b = W[..., 0, :], W[..., 1, :]
    c = np.conj(np.cross(a, b)).astype(W.dtype)
    return np.concatenate([W[..., :2, :], c[..., None, :]], axis=-2)


def _dag(W):
    return np.conj(np.swapaxes(W, -1, -2))


class LowOperator:
    """A in the inner solver's precision: fp32 arithmetic on stored operands.

    ``prec`` = "f32": links and spinors stored as fp32.
    ``prec`` = "f16s": links stored as fp16 with the per-site scale of
    ``f16s_link_scale``; the intermediate odd-site vector and the result are
    stored with ``q_f16s``. Arithmetic is fp32 in both cases.
    ``r12``: twelve-parameter links (SU(3) only): each hop stores the first
    two rows of the matrix it multiplies by, W_mu(x) forward and
    W_mu(x - mu)^+ backward, in the storage precision, and the third row is
    rebuilt from the stored rows in fp32 (``su3_third_row``).
    ``Ulong``: the improved operator (three-hop terms, U = fat links).
    """

    def __init__(self, U, L, m, prec, Ulong=None, r12=False):
        if r12 and Ulong is not None:
            raise ValueError("twelve-parameter links need SU(3) links")
        self.L = extents(L)
        self.m2 = np.float32(m * m)
        self.prec = prec
        self.q = quantiser(prec)
        e = eta(self.L).astype(np.float32)
        self.hops = []  # (distance, direction axis, forward link, backward link at x)
        if prec == "f16s":
            s = f16s_link_scale(U, self.L, Ulong)
        fields = [(1, U)] if Ulong is None else [(1, U), (3, Ulong)]
        for dist, W in fields:
            W32 = W.astype(np.complex64)
            for mu in range(4):
                ax = MU_AXIS[mu]
                u = W32[..., mu, :, :]
                ub = np.roll(u, dist, axis=ax)        # W_mu(x - dist mu) stored at x
                if prec == "f16s":
                    u = _q_link_f16(u, s)
                    ub = _q_link_f16(ub, s)
                if r12:
                    u = su3_third_row(u)
                    ub = _dag(su3_third_row(_dag(ub)))
                fwd = (e[mu][..., None, None] * u).astype(np.complex64)
                bwd = (np.roll(e[mu], dist, axis=ax)[..., None, None] * ub).astype(np.complex64)
                self.hops.append((dist, ax, fwd, bwd))

    def dslash_full(self, chi):
        out = np.zeros_like(chi, dtype=np.complex64)
        for dist, ax, fwd, bwd in self.hops:
            out += _mv(fwd, np.roll(chi, -dist, axis=ax))
            out -= _mhv(bwd, np.roll(chi, dist, axis=ax))
        return out

    def __call__(self, d):
        """Stored result of A d for a stored even-site vector d."""
        full = to_full(self.q(d), self.L, 0).astype(np.complex64)
        t = self.q(from_full(self.dslash_full(full), self.L, 1))
        h = self.dslash_full(to_full(t, self.L, 1).astype(np.complex64))
        out = (self.m2 * self.q(d) - from_full(h, self.L, 0)).astype(np.complex64)
        return self.q(out)


# --------------------------------------------------------------------------
# Fig.2 iterative refinement (outer fp64, fresh low-precision inner CG)
# --------------------------------------------------------------------------

def refinement_cg(U, L, m, b, tol, prec="f32", eps_in=0.1, max_iter=None, Ulong=None, r12=False):
    """Mixed CG by iterative refinement, Fig.2: the inner solve starts from
    y = 0, r = r_k, d = r_k every outer step (no information carried over).
    Ulong: the improved operator (U = fat links); r12: twelve-parameter
    low-precision links (``LowOperator``)."""
    A64 = lambda v: apply_A(U, v, L, m, Ulong)
    Alow = LowOperator(U, L, m, prec, Ulong, r12)
    q = quantiser(prec)
    b = np.asarray(b, dtype=np.complex128)
    max_iter = default_max_iter(b.size) if not max_iter or max_iter <= 0 else max_iter
    x = np.zeros_like(b)
    r = b.copy()
    bb = norm2(b)
    stats = dict(iters=0, outer=0, status="ok")
    rr = norm2(r)
    while rr > tol * tol * bb and stats["iters"] < max_iter:
        y = np.zeros(b.shape, dtype=np.complex64)
        rs = q(r)
        d = rs.copy()
        rrs = norm2(rs)
        rrs0 = rrs
        while rrs > eps_in * eps_in * rrs0 and stats["iters"] < max_iter:
            Ad = Alow(d)
            alpha = rrs / vdot(d, Ad).real
            a32 = np.float32(alpha)
            y = (y + a32 * d).astype(np.complex64)
            rs = q((rs - a32 * Ad).astype(np.complex64))
            rrs_old = rrs
            rrs = norm2(rs)
            d = q((rs + np.float32(rrs / rrs_old) * d).astype(np.complex64))
            stats["iters"] += 1
        x = x + y.astype(np.complex128)
        r = b - A64(x)
        rr = norm2(r)
        stats["outer"] += 1
    stats["true_rel_res"] = math.sqrt(rr / bb) if bb > 0 else 0.0
    if rr > tol * tol * bb:
        stats["status"] = "noconv"
    return x, stats


# --------------------------------------------------------------------------
# Sec.3.2 corrected mixed-precision CG
# --------------------------------------------------------------------------

def mixed_cg(U, L, m, b, tol, prec="f32", delta=0.1, stall_iters=None,
             max_iter=None, max_stall=20, carry_direction=True, update="both", Ulong=None,
             slow_ratio=None, r12=False, cg_budget=None):
    """Corrected mixed-precision CG of Sec.3.2, emulated on the CPU.

    Inner iterations run on stored low-precision vectors (fp32 arithmetic,
    alpha and beta rounded to fp32 when applied); all inner products are
    accumulated in fp64 (Sec.3.2, last paragraph). The partial solution y is
    fp32 (never fp16). The update trigger starts both a reliable update and
    a group-wise update at once (Sec.3.2 uses the two together):

    * |r_s| < delta * max|r_s| since the last update, or |r_s| within the
      requested tolerance: x += y in fp64, y = 0, r = b - A x in fp64, the
      low-precision residual is replaced by the rounded true residual, and
      the direction is carried over as d = r + beta d (Eq.6) with
      beta = |r_true|^2 / |r_s,prev|^2;
    * no new residual minimum for ``stall_iters`` iterations (a safeguard the
      paper does not need with fp32 storage; by default 100 with fp16+scale
      storage and off with fp32): the same update, but the direction
      restarts from d = r. ``max_stall`` consecutive stall updates without
      halving the true residual norm end the solve ("stall").

    Convergence is declared only on the fp64 true residual.
    ``carry_direction=False`` restarts d = r at every update (ablation).
    ``update`` selects ablations that split the update into its two
    ingredients (Sec.3.2's group-wise paragraph, read literally, already
    contains the fp64 residual recompute and so equals "both"):
    "reliable" only replaces the low-precision residual by r = b - A (x + y)
    computed in fp64 at a trigger and never folds y into x (the solution
    stays in fp32); "fold_only" only folds y into x in fp64 (y = 0) and
    never recomputes r, the direction continuing with the iterated beta;
    when its iterated residual meets the tolerance the true residual is
    computed once and decides ("inaccurate" if it misses).
    ``Ulong``: the improved operator (U = fat links), in both precisions.
    ``r12``: twelve-parameter links in the low precision (``LowOperator``).
    ``slow_ratio``: end with status "stall" at the first (non-stall) update
    whose true residual norm fell by less than this factor since the previous
    update: iterative refinement contracts the true residual by about the inner
    reduction ``delta`` per cycle when the inner precision can resolve the
    system, so a cycle that does not even halve it means the low precision
    cannot refine it (the setting a solver that can hand over to a higher
    inner precision uses).
    ``cg_budget``: also end with status "stall" at the first regular update
    after more iterations than ``cg_budget`` times what the CG convergence
    bound allows for the true-residual reduction reached so far: with
    sqrt(kappa) estimated as sk = sqrt(lam / m^2) and R = |r_true| / |b|, the
    allowance is sk/2 (ln(2/R) + ln(sk)) (the A-norm error bound
    2 ((sk-1)/(sk+1))^k, with the residual up to sk times further off). m^2
    bounds the smallest eigenvalue from below; lam is the largest Lanczos
    diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1} of the first cycle (a
    Rayleigh quotient of the residual, so at most the largest eigenvalue; in
    later cycles of a low-precision recurrence it loses that meaning and
    grows far past the operator's norm, so it is taken from the first cycle
    only). The inner precision then converges much slower than CG can on
    this system, even if every cycle still contracts the true residual.
    Returns (x, stats).
    """
    if update not in ("both", "reliable", "fold_only"):
        raise ValueError(update)
    if stall_iters is None:
        stall_iters = 100 if prec == "f16s" else math.inf
    A64 = lambda v: apply_A(U, v, L, m, Ulong)
    Alow = LowOperator(U, L, m, prec, Ulong, r12)
    q = quantiser(prec)
    b = np.asarray(b, dtype=np.complex128)
    max_iter = default_max_iter(b.size) if not max_iter or max_iter <= 0 else max_iter
    bb = norm2(b)
    stats = dict(iters=0, updates=0, restarts=0, status="ok")
    x = np.zeros_like(b)
    if bb == 0.0:
        stats.update(true_rel_res=0.0)
        return x, stats
    stop = tol * tol * bb
    r64 = b - A64(x)
    rr = norm2(r64)
    if rr <= stop:
        stats["true_rel_res"] = math.sqrt(rr / bb)
        return x, stats
    y = np.zeros(b.shape, dtype=np.complex64)
    rs = q(r64)
    d = rs.copy()
    rmax = rmin = math.sqrt(rr)
    since = 0
    stall_count = 0
    best_true = rr
    true_rr = rr
    true_rr0 = rr
    lam = 0.0           # largest Lanczos diagonal seen (cg_budget)
    alpha = 0.0
    beta_d = 0.0        # the beta that formed the current direction (0: d = r)
    while stats["iters"] < max_iter:
        Ad = Alow(d)
        pAp = vdot(d, Ad).real
        if not (pAp > 0.0 and math.isfinite(pAp)):
            stats["status"] = "breakdown"
            break
        if cg_budget and stats["updates"] == 0:
            lam = max(lam, pAp / rr + (beta_d / alpha if beta_d > 0.0 and alpha > 0.0 else 0.0))
        alpha = rr / pAp
        a32 = np.float32(alpha)
        y = (y + a32 * d).astype(np.complex64)
        rs = q((rs - a32 * Ad).astype(np.complex64))
        rr_old = rr
        rr = norm2(rs)
        stats["iters"] += 1
        rn = math.sqrt(rr)
        rmax = max(rmax, rn)
        if rn < rmin:
            rmin = rn
            since = 0
        else:
            since += 1
        upd = rn < delta * rmax or rr <= stop
        stall = (not upd) and since >= stall_iters
        if (upd or stall) and update == "fold_only":
            # fold the correction into x; the iterated residual carries on
            x = x + y.astype(np.complex128)
            y[:] = 0
            stats["updates"] += 1
            if rr <= stop:
                true_rr = norm2(b - A64(x))
                if true_rr > stop:
                    stats["status"] = "inaccurate"
                break
            rmax = rmin = rn
            since = 0
            if stall:
                stats["restarts"] += 1
                d = rs.copy()
                beta_d = 0.0
                continue
        elif upd or stall:
            if update == "both":
                x = x + y.astype(np.complex128)
                y[:] = 0
                r64 = b - A64(x)
            else:  # reliable only: y stays, r from x + y
                r64 = b - A64(x + y.astype(np.complex128))
            rr = norm2(r64)
            prev_true, true_rr = true_rr, rr
            stats["updates"] += 1
            if rr <= stop:
                break
            if slow_ratio and not stall and rr > slow_ratio * slow_ratio * prev_true:
                stats["status"] = "stall"
                break
            if cg_budget and not stall and lam > 0.0 and rr < true_rr0:
                sk = math.sqrt(lam / (m * m))
                allow = 0.5 * sk * (math.log(2.0 / math.sqrt(rr / true_rr0)) + math.log(sk))
                if stats["iters"] > cg_budget * allow:
                    stats["status"] = "stall"
                    break
            rs = q(r64)
            rmax = rmin = math.sqrt(rr)
            since = 0
            if stall:
                stats["restarts"] += 1
                if rr < 0.25 * best_true:
                    stall_count = 0
                else:
                    stall_count += 1
                    if stall_count >= max_stall:
                        stats["status"] = "stall"
                        break
                best_true = min(best_true, rr)
                d = rs.copy()
                beta_d = 0.0
                continue
            best_true = min(best_true, rr)
            if not carry_direction:
                d = rs.copy()
                beta_d = 0.0
                continue
        beta = rr / rr_old
        beta_d = beta
        d = q((rs + np.float32(beta) * d).astype(np.complex64))
    if update == "reliable":
        # the solution is x + y; x is never updated by this variant
        x = x + y.astype(np.complex128)
        true_rr = norm2(b - A64(x))
        if stats["status"] == "ok" and true_rr > stop:
            stats["status"] = "noconv"
    elif stats["status"] == "ok" and true_rr > stop:
        # ran out of iterations: fold in the pending correction
        x = x + y.astype(np.complex128)
        true_rr = norm2(b - A64(x))
        if true_rr > stop:
            stats["status"] = "noconv"
    stats["true_rel_res"] = math.sqrt(true_rr / bb)
    return x, stats
