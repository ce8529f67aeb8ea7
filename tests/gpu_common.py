"""Shared helpers of the GPU parity tests (imported only by tests)."""

import functools
import sys

import numpy as np

import synth


def log(*a):
    print(*a, flush=True, file=sys.stderr)


def rel_max(a, b):
    """max |a - b| / max |b| over all entries."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_norm(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@functools.lru_cache(maxsize=8)
def links(L, kind="haar", seed=1, eps=0.3):
    if kind == "haar":
        return synth.haar_links(L, seed)
    if kind == "exp":
        return synth.exp_ih_links(L, seed, eps)
    if kind == "unit":
        return synth.unit_links(L)
    raise ValueError(kind)


def oracle_apply_A(U, v, L, m):
    """fp64 oracle A on (nrhs, Vh, 3); the C oracle for speed on big lattices."""
    from oracle import c as oc
    return np.stack([oc.apply_A(U, v[r], L, m if np.isscalar(m) else m[r]) for r in range(v.shape[0])])


def oracle_dslash(U, v, L, p_in):
    from oracle import c as oc
    return np.stack([oc.dslash(U, v[r], L, p_in) for r in range(v.shape[0])])
