"""Seeded synthetic inputs for the staggered CG solve.

This module only draws random numbers and assembles input fields in the
canonical host layouts below. It contains none of the solver's arithmetic
(no Dirac operator, no CG), so both the CPU oracle and the HIP path can take
their inputs from here without sharing any of the method.

Canonical host layouts (all complex128, C order):

* lattice extents ``L = (Lx, Ly, Lz, Lt)``, every extent even and >= 2;
* gauge links ``U[t, z, y, x, mu, a, b]`` with ``mu = 0..3`` for the x, y, z
  and t directions; the staggered phases are *not* included;
* even-parity spinors ``chi[rhs, s, c]`` with ``s = lex // 2`` over the even
  sites in lexicographic order ``lex = x + Lx*(y + Ly*(z + Lz*t))`` and colour
  ``c = 0..2``;
* site-local SU(3) matrices ``g[t, z, y, x, a, b]``.

Every generator takes an explicit integer seed and uses
``numpy.random.Generator(PCG64(seed))``; draws are made in the canonical
order of the output array.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "make_rng",
    "check_extents",
    "complex_gaussian",
    "haar_su3",
    "exp_ih_su3",
    "haar_links",
    "exp_ih_links",
    "unit_links",
    "twisted_links",
    "random_gauge",
    "gauge_transform_links",
    "gaussian_links",
    "naik_links",
    "NAIK_C1",
    "NAIK_C3",
    "gaussian_rhs",
    "request_stream",
    "CONFIGS",
]


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def check_extents(L) -> tuple:
    L = tuple(int(v) for v in L)
    if len(L) != 4 or any(v < 2 or v % 2 for v in L):
        raise ValueError(f"lattice extents must be 4 even integers >= 2, got {L}")
    return L


def _link_shape(L):
    Lx, Ly, Lz, Lt = check_extents(L)
    return (Lt, Lz, Ly, Lx, 4)


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """(N(0,1) + i N(0,1)) / sqrt(2) per entry: unit variance complex normal."""
    g = rng.standard_normal(tuple(shape) + (2,))
    return (g[..., 0] + 1j * g[..., 1]) * np.sqrt(0.5)


def _det3(m: np.ndarray) -> np.ndarray:
    return (m[..., 0, 0] * (m[..., 1, 1] * m[..., 2, 2] - m[..., 1, 2] * m[..., 2, 1])
            - m[..., 0, 1] * (m[..., 1, 0] * m[..., 2, 2] - m[..., 1, 2] * m[..., 2, 0])
            + m[..., 0, 2] * (m[..., 1, 0] * m[..., 2, 1] - m[..., 1, 1] * m[..., 2, 0]))


def _fix_det(q: np.ndarray) -> np.ndarray:
    """Scale a unitary matrix by the principal cube root of 1/det, giving det 1."""
    phase = np.angle(_det3(q))
    return q * np.exp(-1j * phase / 3.0)[..., None, None]


def haar_su3(rng: np.random.Generator, shape) -> np.ndarray:
    """Haar-distributed SU(3) matrices.

    A complex Gaussian matrix is orthonormalised column by column (Gram-Schmidt
    with re-orthogonalisation; this equals
    the Q factor of a QR decomposition whose R has a positive real diagonal,
    which is what makes Q Haar-distributed on U(3)); the result is then
    multiplied by exp(-i arg(det)/3) so that det = 1.
    """
    z = complex_gaussian(rng, tuple(shape) + (3, 3))
    cols = [z[..., :, j] for j in range(3)]
    q = []
    for j in range(3):
        v = cols[j].copy()
        for _ in range(2):  # a second pass restores orthogonality to rounding
            for k in range(j):
                v -= np.sum(np.conj(q[k]) * v, axis=-1, keepdims=True) * q[k]
        v /= np.sqrt(np.sum(np.abs(v) ** 2, axis=-1, keepdims=True))
        q.append(v)
    u = np.stack(q, axis=-1)
    return _fix_det(u)


def exp_ih_su3(rng: np.random.Generator, shape, eps: float) -> np.ndarray:
    """exp(i*eps*H) with H a traceless Hermitian Gaussian matrix.

    H = (G + G^dagger)/2 - tr(.)/3 with G complex Gaussian; the exponential is
    taken through the eigen-decomposition H = V diag(w) V^dagger. eps sets how
    far the links sit from the identity (the disorder of the field).
    """
    g = complex_gaussian(rng, tuple(shape) + (3, 3))
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    u = (v * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))
    return u


def haar_links(L, seed: int) -> np.ndarray:
    return haar_su3(make_rng(seed), _link_shape(L))


def exp_ih_links(L, seed: int, eps: float) -> np.ndarray:
    return exp_ih_su3(make_rng(seed), _link_shape(L), eps)


def unit_links(L) -> np.ndarray:
    shp = _link_shape(L)
    u = np.zeros(shp + (3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def twisted_links(L, theta) -> np.ndarray:
    """Constant diagonal SU(3) links.

    theta has shape (4, 2): U_mu = diag(e^{i th0}, e^{i th1}, e^{-i(th0+th1)})
    on every site.
    """
    theta = np.asarray(theta, dtype=np.float64).reshape(4, 2)
    shp = _link_shape(L)
    u = np.zeros(shp + (3, 3), dtype=np.complex128)
    for mu in range(4):
        a, b = theta[mu]
        u[..., mu, 0, 0] = np.exp(1j * a)
        u[..., mu, 1, 1] = np.exp(1j * b)
        u[..., mu, 2, 2] = np.exp(-1j * (a + b))
    return u


def random_gauge(L, seed: int) -> np.ndarray:
    """Site-local Haar SU(3) matrices g[t, z, y, x, a, b]."""
    Lx, Ly, Lz, Lt = check_extents(L)
    return haar_su3(make_rng(seed), (Lt, Lz, Ly, Lx))


_MU_AXIS = (3, 2, 1, 0)  # array axis of the x, y, z, t direction in [t, z, y, x]


def gauge_transform_links(U: np.ndarray, g: np.ndarray, dist: int = 1) -> np.ndarray:
    """U^g_mu(x) = g(x) U_mu(x) g(x + dist mu)^dagger (periodic lattice).

    dist = 3 transforms long links, which connect x to x + 3 mu."""
    out = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -int(dist), axis=_MU_AXIS[mu])
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(g_fwd, -1, -2))
    return out


def gaussian_links(L, seed: int) -> np.ndarray:
    """Links with independent unit-variance complex normal entries (not unitary)."""
    return complex_gaussian(make_rng(seed), _link_shape(L) + (3, 3))


# Coefficients of the one- and three-hop terms that cancel the leading
# discretisation error of the symmetric difference (no factor 1/2 in front):
# c1 (f(x+1) - f(x-1)) + c3 (f(x+3) - f(x-3)) = 2 f'(x) + O(f^(5)).
NAIK_C1 = 9.0 / 8.0
NAIK_C3 = -1.0 / 24.0


def naik_links(U: np.ndarray, c1: float = NAIK_C1, c3: float = NAIK_C3,
               fat_noise: float = 0.0, seed: int = 0):
    """Input fields of the improved staggered operator built from links U.

    Returns (fat, long): fat_mu(x) = c1 U_mu(x) (+ fat_noise times complex
    normal entries, so that fat links are not unitary, like smeared links),
    long_mu(x) = c3 U_mu(x) U_mu(x + mu) U_mu(x + 2 mu).
    """
    fat = c1 * U
    if fat_noise:
        fat = fat + fat_noise * complex_gaussian(make_rng(seed), U.shape)
    long = np.empty_like(U)
    for mu in range(4):
        ax = _MU_AXIS[mu]
        u = U[..., mu, :, :]
        long[..., mu, :, :] = c3 * (u @ np.roll(u, -1, axis=ax) @ np.roll(u, -2, axis=ax))
    return fat, long


def gaussian_rhs(L, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian even-parity right-hand sides, shape (nrhs, Ve, 3)."""
    Lx, Ly, Lz, Lt = check_extents(L)
    ve = Lx * Ly * Lz * Lt // 2
    return complex_gaussian(make_rng(seed), (int(nrhs), ve, 3))


def request_stream(seed: int, n: int, rate: float, sizes, masses, tols,
                   max_nrhs: int = 8):
    """Poisson arrivals of solve requests.

    Returns a list of dicts with arrival time (s), lattice index into
    ``sizes``, mass, tolerance, number of right-hand sides and the RHS seed.
    """
    rng = make_rng(seed)
    t = 0.0
    out = []
    for i in range(int(n)):
        t += rng.exponential(1.0 / rate)
        out.append({
            "id": i,
            "t": t,
            "lattice": int(rng.integers(len(sizes))),
            "mass": float(masses[int(rng.integers(len(masses)))]),
            "tol": float(tols[int(rng.integers(len(tols)))]),
            "nrhs": int(rng.integers(1, max_nrhs + 1)),
            "rhs_seed": 1000 + i,
        })
    return out


# The workloads the solver is exercised on: lattice extents, link recipe,
# mass, number of right-hand sides, tolerance and the two seeds.
CONFIGS = {
    "c1_4x4x4x4": dict(L=(4, 4, 4, 4), links="haar", eps=None, gauge_seed=11,
                       rhs_seed=111, mass=0.1, nrhs=1, tol=1e-10),
    "c2_16x16x16x32": dict(L=(16, 16, 16, 32), links="exp", eps=0.3, gauge_seed=12,
                           rhs_seed=112, mass=0.01, nrhs=1, tol=1e-8),
    "c3_32x32x32x64": dict(L=(32, 32, 32, 64), links="haar", eps=None, gauge_seed=13,
                           rhs_seed=113, mass=0.005, nrhs=1, tol=1e-10),
    "c4_24x24x24x48": dict(L=(24, 24, 24, 48), links="exp", eps=0.5, gauge_seed=14,
                           rhs_seed=114, mass=0.01, nrhs=12, tol=1e-8),
}


def config_links(name: str) -> np.ndarray:
    c = CONFIGS[name]
    if c["links"] == "haar":
        return haar_links(c["L"], c["gauge_seed"])
    return exp_ih_links(c["L"], c["gauge_seed"], c["eps"])


def config_rhs(name: str) -> np.ndarray:
    c = CONFIGS[name]
    return gaussian_rhs(c["L"], c["nrhs"], c["rhs_seed"])


__all__ += ["config_links", "config_rhs"]
