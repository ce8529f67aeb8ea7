"""Brute-force and closed-form references that pin the oracle.

TEST INFRASTRUCTURE (see the package docstring).

* ``dense_D``: the Dirac matrix assembled entry by entry from the matrix
  form of Eq.4, D_{x,y} = U_mu(x) delta_{y,x+mu} - U_mu(x-mu)^+ delta_{y,x-mu}
  (phases of Sec.2 folded in), with a pure-Python loop over sites. It shares
  no code with the vectorised operator in ``oracle.stag``.
* ``dense_A_even``: m^2 - D^2 (Eq.3) restricted to the even sites.
* ``free_spectrum`` / ``twisted_spectrum``: eigenvalues of A for unit links
  and for constant diagonal links, from Fourier analysis: with the staggered
  phases the cross terms of D^2 cancel and -D^2 acts as
  sum_mu 4 sin^2(p_mu + theta_mu) on a colour component with twist theta.
  With ``naik=(c1, c3)`` the links are c1 times those and the long links
  c3 times their cube (the improved operator); a three-hop also anticommutes
  with the other directions' phases, and -D^2 acts as
  sum_mu 4 (c1 sin q_mu + c3 sin 3 q_mu)^2 with q = p + theta.
* ``fft_solve``: the exact solution of A x = b for such fields.
"""

from __future__ import annotations

import itertools

import numpy as np


def _lex(c, L):
    x, y, z, t = c
    Lx, Ly, Lz, Lt = L
    return x + Lx * (y + Ly * (z + Lz * t))


def _eta(mu, c):
    return -1.0 if sum(c[:mu]) % 2 else 1.0


def dense_D(U, L, Ulong=None):
    """Full 3V x 3V Dirac matrix (rows/cols ordered lex * 3 + colour).

    With Ulong (improved operator, U = fat links) the three-hop entries
    eta N(x) at x+3mu and -eta N(x-3mu)^+ at x-3mu are added as well."""
    L = tuple(int(v) for v in L)
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    hops = [(1, U)] if Ulong is None else [(1, U), (3, Ulong)]
    for c in itertools.product(range(Lx), range(Ly), range(Lz), range(Lt)):
        x = _lex(c, L)
        for mu in range(4):
            for dist, W in hops:
                fwd = list(c)
                fwd[mu] = (fwd[mu] + dist) % L[mu]
                bwd = list(c)
                bwd[mu] = (bwd[mu] - dist) % L[mu]
                w_here = W[c[3], c[2], c[1], c[0], mu]
                w_back = W[bwd[3], bwd[2], bwd[1], bwd[0], mu]
                y_f = _lex(fwd, L)
                y_b = _lex(bwd, L)
                D[3 * x:3 * x + 3, 3 * y_f:3 * y_f + 3] += _eta(mu, c) * w_here
                D[3 * x:3 * x + 3, 3 * y_b:3 * y_b + 3] -= _eta(mu, bwd) * np.conj(w_back.T)
    return D


def even_rows(L):
    """Indices (lex * 3 + colour) of the even sites in checkerboard order."""
    L = tuple(int(v) for v in L)
    Lx, Ly, Lz, Lt = L
    idx = []
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    if (x + y + z + t) % 2 == 0:
                        lex = _lex((x, y, z, t), L)
                        idx.extend([3 * lex, 3 * lex + 1, 3 * lex + 2])
    return np.array(idx)


def dense_A_even(U, L, m, Ulong=None):
    D = dense_D(U, L, Ulong)
    A = m * m * np.eye(D.shape[0]) - D @ D
    e = even_rows(L)
    return A[np.ix_(e, e)]


def _momenta(L):
    """sin^2 tables per direction for p_mu = 2 pi n / L_mu, on [t, z, y, x]."""
    Lx, Ly, Lz, Lt = L
    return [2 * np.pi * np.arange(n) / n for n in (Lx, Ly, Lz, Lt)]


def _hop_symbol(q, naik):
    """|D| symbol of one direction: 2 sin q, or 2 (c1 sin q + c3 sin 3q)."""
    if naik is None:
        return 2.0 * np.sin(q)
    c1, c3 = naik
    return 2.0 * (c1 * np.sin(q) + c3 * np.sin(3.0 * q))


def free_spectrum(L, m, naik=None):
    """Sorted eigenvalues of A on the even sites for unit links (3 colours).

    Momenta p and p + (pi, pi, pi, pi) share one even-site eigenvector pair,
    so each value of the full-lattice set is counted once per such pair.
    """
    return twisted_spectrum(L, m, np.zeros((4, 2)), naik)


def twisted_spectrum(L, m, theta, naik=None):
    """Sorted eigenvalues of A for constant links diag(e^{i a}, e^{i b}, e^{-i(a+b)})
    (times c1, with long links c3 diag(e^{3i a}, ...), for naik = (c1, c3))."""
    theta = np.asarray(theta, dtype=np.float64).reshape(4, 2)
    ps = _momenta(L)
    vals = []
    for c in range(3):
        th = [(theta[mu, 0], theta[mu, 1], -theta[mu, 0] - theta[mu, 1])[c] for mu in range(4)]
        grid = np.zeros([len(p) for p in ps])
        for mu in range(4):
            shape = [1, 1, 1, 1]
            shape[mu] = len(ps[mu])
            grid = grid + _hop_symbol(ps[mu] + th[mu], naik).reshape(shape) ** 2
        vals.append(m * m + grid.ravel())
    v = np.sort(np.concatenate(vals))
    # every eigenvalue of the full lattice operator appears twice (once per
    # parity sector); the even-site block holds one copy of each pair
    return v[::2]


def fft_solve(b_even, L, m, theta=None, naik=None):
    """Exact solution of A x = b for constant diagonal links (unit links when
    theta is None; the improved operator's fields of ``twisted_spectrum``
    with naik), by Fourier transform of the full lattice with b placed on
    the even sites and zeros on the odd ones. Returns the even-site x."""
    from .stag import to_full, from_full
    L = tuple(int(v) for v in L)
    theta = np.zeros((4, 2)) if theta is None else np.asarray(theta, dtype=np.float64).reshape(4, 2)
    full = to_full(np.asarray(b_even, dtype=np.complex128), L, 0)  # [t, z, y, x, c]
    Lx, Ly, Lz, Lt = L
    out = np.empty_like(full)
    n = [np.fft.fftfreq(k) * 2 * np.pi for k in (Lt, Lz, Ly, Lx)]  # p on array axes
    dir_of_axis = (3, 2, 1, 0)
    for c in range(3):
        lam = np.full((Lt, Lz, Ly, Lx), m * m)
        for ax in range(4):
            mu = dir_of_axis[ax]
            th = (theta[mu, 0], theta[mu, 1], -theta[mu, 0] - theta[mu, 1])[c]
            shape = [1, 1, 1, 1]
            shape[ax] = len(n[ax])
            lam = lam + _hop_symbol(n[ax] + th, naik).reshape(shape) ** 2
        out[..., c] = np.fft.ifftn(np.fft.fftn(full[..., c]) / lam)
    return from_full(out, L, 0)
