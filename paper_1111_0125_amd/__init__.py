"""Python binding of libstag: CG solves of b = A x with the even-odd staggered
normal operator A = m^2 - D_eo D_oe on an AMD Instinct MI355X.

Argument marshalling only: every step of the operator and the solver runs in
the HIP kernels of ``libstag.so`` (built in-tree by
``python paper_1111_0125_amd/build.py``). Importing this package without the
built library raises ImportError; there is no CPU fallback.

Arrays are passed either as host numpy arrays or as device tensors (any
object with ``data_ptr()`` and ``is_cuda``, e.g. torch), in the canonical
complex128 layouts of ``include/stag.h``:

* links ``U[t, z, y, x, mu, a, b]`` (no staggered phases),
* vectors ``v[rhs, s, c]`` over the sites of one parity, ``s = lex // 2``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstag.so")

STAG_OK = 0
STAG_PENDING = 1
STAG_EINVAL = -1
STAG_ENOMEM = -2
STAG_EDEVICE = -3
STAG_ENOCONV = -4
STAG_EBREAKDOWN = -5
STAG_ESTALL = -6
STAG_EBUSY = -7
NOALLOC_SCRATCH_BYTES = 48 << 20  # STAG_NOALLOC_SCRATCH_BYTES
STAG_ENOTFOUND = -8

F64, F32, F16S = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "f16s": F16S}
MIXED_CARRY, MIXED_RESTART, MIXED_RELIABLE, MIXED_FOLD_ONLY = 0, 1, 2, 3
GAUGE_R12 = 1 << 4
TUNE_IMPROVED = 1 << 8
MAX_RHS = 16

STATUS_NAME = {
    STAG_OK: "ok", STAG_PENDING: "pending", STAG_EINVAL: "einval", STAG_ENOMEM: "enomem",
    STAG_EDEVICE: "edevice", STAG_ENOCONV: "enoconv", STAG_EBREAKDOWN: "ebreakdown",
    STAG_ESTALL: "estall", STAG_EBUSY: "ebusy", STAG_ENOTFOUND: "enotfound",
}


class StagError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAME.get(code, code)}: {msg}")
        self.code = code


class TuneCfg(ctypes.Structure):
    _fields_ = [("S1", ctypes.c_int), ("S2", ctypes.c_int), ("nt", ctypes.c_int),
                ("swizzle", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


K_HOP1, K_HOP2, K_HOP1_64, K_HOP2_64, K_UPDATE, K_XPAY, K_OTHER = range(7)


class CgParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("inner_prec", ctypes.c_int),
        ("delta", ctypes.c_double),
        ("stall_iters", ctypes.c_int),
        ("max_stall", ctypes.c_int),
        ("graph_k", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("use_x0", ctypes.c_int),
        ("escalate", ctypes.c_int),
        ("mixed_variant", ctypes.c_int),
        ("small_lattice", ctypes.c_int),
    ]


class CgStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("reliable_updates", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("status", ctypes.c_int),
        ("true_rel_res", ctypes.c_double),
        ("iter_rel_res", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("inner_final", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: run `python paper_1111_0125_amd/build.py` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "stag_version": ([], ip),
        "stag_create": ([ip, ctypes.c_size_t, pp], ip),
        "stag_destroy": ([vp], ip),
        "stag_last_error": ([vp], ctypes.c_char_p),
        "stag_memory_used": ([vp, ctypes.POINTER(ctypes.c_size_t)], ip),
        "stag_gauge_create": ([vp, ctypes.POINTER(ctypes.c_int), vp, ip, ip, pp], ip),
        "stag_gauge_create_improved": ([vp, ctypes.POINTER(ctypes.c_int), vp, vp, ip, ip, pp], ip),
        "stag_gauge_destroy": ([vp], ip),
        "stag_gauge_sites": ([vp, ctypes.POINTER(ctypes.c_int64)], ip),
        "stag_field_create": ([vp, vp, ip, ip, ip, pp], ip),
        "stag_field_import": ([vp, vp, ip, vp], ip),
        "stag_field_export": ([vp, vp, ip, vp], ip),
        "stag_field_destroy": ([vp], ip),
        "stag_dslash": ([vp, vp, vp, vp, vp], ip),
        "stag_apply_A": ([vp, vp, ctypes.POINTER(dp), vp, vp, vp], ip),
        "stag_apply_A_noalloc": ([vp, vp, ctypes.POINTER(dp), vp, vp, vp], ip),
        "stag_cg_params_default": ([ctypes.POINTER(CgParams)], None),
        "stag_cg_solve": ([vp, vp, ctypes.POINTER(dp), vp, vp, ctypes.POINTER(CgParams),
                           ctypes.POINTER(CgStats), vp], ip),
        "stag_tune_get": ([vp, ip, ip, ctypes.c_int64, ctypes.POINTER(TuneCfg)], ip),
        "stag_tune_set": ([vp, ip, ip, ctypes.c_int64, ctypes.POINTER(TuneCfg)], ip),
        "stag_tune": ([vp, vp, ip, ip, ctypes.POINTER(TuneCfg), ctypes.POINTER(dp)], ip),
        "stag_tune_counts": ([vp, ctypes.POINTER(ip), ctypes.POINTER(ip)], ip),
        "stag_solver_submit": ([vp, vp, dp, ip, vp, dp, ip, ctypes.POINTER(ctypes.c_int64)], ip),
        "stag_solver_poll": ([vp, ctypes.c_int64, vp, ctypes.POINTER(CgStats),
                              ctypes.POINTER(dp)], ip),
        "stag_solver_config": ([vp, ip, ip, ip], ip),
        "stag_timing_enable": ([vp, ip], ip),
        "stag_time_kernels": ([vp, vp, ip, ip, ip, ctypes.POINTER(dp)], ip),
        "stag_timing_read": ([vp, ip, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(dp)], ip),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _ptr(a):
    """(pointer, on_device) of a host numpy array or a device tensor."""
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr()), 1 if getattr(a, "is_cuda", False) else 0
    arr = np.ascontiguousarray(a)
    return ctypes.c_void_p(arr.ctypes.data), 0


def _check_c128(a, shape, what):
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.complex128 or not a.is_contiguous():
            raise ValueError(f"{what}: need a contiguous complex128 tensor")
        if tuple(a.shape) != tuple(shape):
            raise ValueError(f"{what}: shape {tuple(a.shape)} != {tuple(shape)}")
        return a
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != tuple(shape):
        raise ValueError(f"{what}: shape {a.shape} != {tuple(shape)}")
    return a


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        s = s.cuda_stream
    return ctypes.c_void_p(int(s)) if s else None


class Context:
    """A libstag context bound to one GPU (stag_create / stag_destroy)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        rc = lib.stag_create(int(device), int(hbm_budget), ctypes.byref(h))
        if rc != STAG_OK:
            raise StagError(rc, lib.stag_last_error(None).decode())
        self.h = h
        self._objs = []

    def check(self, rc):
        if rc not in (STAG_OK, STAG_PENDING):
            raise StagError(rc, self.last_error())
        return rc

    def last_error(self) -> str:
        return lib.stag_last_error(self.h).decode()

    def memory_used(self) -> int:
        v = ctypes.c_size_t()
        self.check(lib.stag_memory_used(self.h, ctypes.byref(v)))
        return v.value

    def close(self):
        if self.h:
            lib.stag_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gauge(self, L, U, precisions=("f64", "f32"), r12=False, long=None) -> "Gauge":
        return Gauge(self, L, U, precisions, r12, long)

    def field(self, gauge, parity=0, prec="f64", nrhs=1) -> "Field":
        return Field(self, gauge, parity, prec, nrhs)


class Gauge:
    """A resident gauge field (stag_gauge_create); r12: 12-parameter copies
    (SU(3) links only). With ``long`` (stag_gauge_create_improved) the
    improved operator: U holds the fat links, ``long`` the long links, both
    host arrays or both device tensors."""

    def __init__(self, ctx: Context, L, U, precisions=("f64", "f32"), r12=False, long=None):
        L = tuple(int(v) for v in L)
        Lx, Ly, Lz, Lt = L
        shape = (Lt, Lz, Ly, Lx, 4, 3, 3)
        U = _check_c128(U, shape, "links")
        mask = GAUGE_R12 if r12 else 0
        for p in precisions:
            mask |= 1 << PREC[p]
        h = ctypes.c_void_p()
        ptr, dev = _ptr(U)
        Lc = (ctypes.c_int * 4)(*L)
        if long is None:
            ctx.check(lib.stag_gauge_create(ctx.h, Lc, ptr, dev, mask, ctypes.byref(h)))
        else:
            long = _check_c128(long, shape, "long links")
            lptr, ldev = _ptr(long)
            if ldev != dev:
                raise ValueError("fat and long links must both be on the host or both on the device")
            ctx.check(lib.stag_gauge_create_improved(ctx.h, Lc, ptr, lptr, dev, mask,
                                                     ctypes.byref(h)))
        self.ctx, self.h, self.L, self.mask, self.r12 = ctx, h, L, mask, bool(r12)
        self.improved = long is not None
        self.vh = Lx * Ly * Lz * Lt // 2

    def destroy(self):
        """stag_gauge_destroy; raises StagError (EBUSY) while serving requests
        on this gauge are uncollected (the gauge then stays valid)."""
        if self.h:
            self.ctx.check(lib.stag_gauge_destroy(self.h))
            self.h = None


class Field:
    """nrhs vectors of one parity and storage precision (stag_field_*)."""

    def __init__(self, ctx: Context, gauge: Gauge, parity=0, prec="f64", nrhs=1):
        h = ctypes.c_void_p()
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        ctx.check(lib.stag_field_create(ctx.h, gauge.h, int(parity), p, int(nrhs), ctypes.byref(h)))
        self.ctx, self.gauge, self.h = ctx, gauge, h
        self.parity, self.prec, self.nrhs = int(parity), p, int(nrhs)
        self.shape = (self.nrhs, gauge.vh, 3)

    def load(self, v, stream=None):
        v = _check_c128(v, self.shape, "field import")
        ptr, dev = _ptr(v)
        self.ctx.check(lib.stag_field_import(self.h, ptr, dev, _stream(stream)))
        return self

    def store(self, out=None, stream=None):
        """Export to a new host array, or into `out` (host array or device tensor)."""
        if out is None:
            out = np.empty(self.shape, dtype=np.complex128)
        _check_c128(out, self.shape, "field export")
        ptr, dev = _ptr(out)
        self.ctx.check(lib.stag_field_export(self.h, ptr, dev, _stream(stream)))
        return out

    def destroy(self):
        if self.h:
            lib.stag_field_destroy(self.h)
            self.h = None


def stag_dslash(ctx: Context, gauge: Gauge, fin: Field, fout: Field, stream=None):
    """out = D in (Eq.5), parity p -> 1 - p."""
    return ctx.check(lib.stag_dslash(ctx.h, gauge.h, fin.h, fout.h, _stream(stream)))


def stag_apply_A(ctx: Context, gauge: Gauge, mass, fin: Field, fout: Field, stream=None):
    """out_j = m_j^2 in_j - D_eo D_oe in_j (Eq.2-3) on even fields."""
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (fin.nrhs,)).copy()
    mp = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return ctx.check(lib.stag_apply_A(ctx.h, gauge.h, mp, fin.h, fout.h, _stream(stream)))


def stag_apply_A_noalloc(ctx: Context, gauge: Gauge, mass, fin: Field, fout: Field, stream=None):
    """stag_apply_A with its intermediate in the library's device scratch
    (allocates nothing; intermediates up to NOALLOC_SCRATCH_BYTES)."""
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (fin.nrhs,)).copy()
    mp = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return ctx.check(lib.stag_apply_A_noalloc(ctx.h, gauge.h, mp, fin.h, fout.h, _stream(stream)))


def cg_params(tol=1e-8, inner="f64", max_iter=0, delta=0.1, stall_iters=0, max_stall=20,
              graph_k=0, use_graph=True, use_x0=False, escalate=True,
              mixed_variant="carry", small_lattice=True) -> CgParams:
    p = CgParams()
    lib.stag_cg_params_default(ctypes.byref(p))
    p.tol = tol
    p.max_iter = max_iter
    p.inner_prec = PREC[inner] if isinstance(inner, str) else int(inner)
    p.delta = delta
    p.stall_iters = stall_iters
    p.max_stall = max_stall
    p.graph_k = graph_k
    p.use_graph = 1 if use_graph else 0
    p.use_x0 = 1 if use_x0 else 0
    p.escalate = 1 if escalate else 0
    p.mixed_variant = {"carry": MIXED_CARRY, "restart": MIXED_RESTART, "reliable": MIXED_RELIABLE,
                       "fold_only": MIXED_FOLD_ONLY}[mixed_variant]
    p.small_lattice = 1 if small_lattice else 0
    return p


def stag_cg_solve(ctx: Context, gauge: Gauge, mass, b: Field, x: Field, params: CgParams = None,
                  stream=None):
    """Solve A_j x_j = b_j (Fig.1 / Sec.3.2). Returns (status, list of stats dicts)."""
    params = params or cg_params()
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (b.nrhs,)).copy()
    stats = (CgStats * b.nrhs)()
    rc = lib.stag_cg_solve(ctx.h, gauge.h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           b.h, x.h, ctypes.byref(params), stats, _stream(stream))
    if rc in (STAG_EINVAL, STAG_ENOMEM, STAG_EDEVICE):
        raise StagError(rc, ctx.last_error())
    return rc, [s.as_dict() for s in stats]


def stag_tune(ctx: Context, gauge: Gauge, prec="f32", nrhs=1):
    """Autotune the hop launch shape on this gauge; returns (cfg dict, ms per A)."""
    cfg = TuneCfg()
    ms = ctypes.c_double()
    ctx.check(lib.stag_tune(ctx.h, gauge.h, PREC[prec] if isinstance(prec, str) else prec,
                            int(nrhs), ctypes.byref(cfg), ctypes.byref(ms)))
    return cfg.as_dict(), ms.value


def stag_tune_counts(ctx: Context):
    """(loaded, measured): stag_tune calls answered from STAG_TUNE_CACHE / timed."""
    a, b = ctypes.c_int(), ctypes.c_int()
    ctx.check(lib.stag_tune_counts(ctx.h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def _tune_prec(prec, improved):
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    return p | (TUNE_IMPROVED if improved else 0)


def stag_tune_get(ctx: Context, prec, nrhs, vh, improved=False):
    """Launch shape for (prec, nrhs, vh) of Eq.5 gauges, or of improved-operator gauges."""
    cfg = TuneCfg()
    ctx.check(lib.stag_tune_get(ctx.h, _tune_prec(prec, improved), int(nrhs), int(vh),
                                ctypes.byref(cfg)))
    return cfg.as_dict()


def stag_tune_set(ctx: Context, prec, nrhs, vh, S1=1, S2=1, nt=1, swizzle=1, improved=False):
    cfg = TuneCfg(S1, S2, nt, swizzle)
    return ctx.check(lib.stag_tune_set(ctx.h, _tune_prec(prec, improved), int(nrhs), int(vh),
                                       ctypes.byref(cfg)))


def stag_timing_enable(ctx: Context, on=True):
    return ctx.check(lib.stag_timing_enable(ctx.h, 1 if on else 0))


def stag_timing_read(ctx: Context, kind):
    """(launch count, summed milliseconds) of one kernel kind (K_*)."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    ctx.check(lib.stag_timing_read(ctx.h, int(kind), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def stag_solver_config(ctx: Context, slots_per_batch=16, graph_k=0, queue_cap=4096):
    return ctx.check(lib.stag_solver_config(ctx.h, int(slots_per_batch), int(graph_k),
                                            int(queue_cap)))


def stag_solver_submit(ctx: Context, gauge: Gauge, mass, b, tol=1e-8, inner="f32") -> int:
    """Queue a solve of A x = b (b: complex128 (nrhs, Vh, 3) host array); returns a ticket."""
    b = np.ascontiguousarray(b, dtype=np.complex128)
    if b.ndim != 3 or b.shape[1:] != (gauge.vh, 3):
        raise ValueError(f"b must have shape (nrhs, {gauge.vh}, 3)")
    t = ctypes.c_int64()
    ctx.check(lib.stag_solver_submit(ctx.h, gauge.h, float(mass), int(b.shape[0]),
                                     ctypes.c_void_p(b.ctypes.data), float(tol),
                                     PREC[inner] if isinstance(inner, str) else int(inner),
                                     ctypes.byref(t)))
    return t.value


def stag_solver_poll(ctx: Context, ticket: int, nrhs: int, vh: int, want_x=True):
    """None while pending; else (status, x or None, stats list, latency seconds)."""
    x = np.empty((nrhs, vh, 3), dtype=np.complex128) if want_x else None
    stats = (CgStats * nrhs)()
    lat = ctypes.c_double()
    rc = lib.stag_solver_poll(ctx.h, int(ticket),
                              ctypes.c_void_p(x.ctypes.data) if want_x else None, stats,
                              ctypes.byref(lat))
    if rc == STAG_PENDING:
        return None
    if rc in (STAG_EINVAL, STAG_ENOTFOUND, STAG_EDEVICE, STAG_ENOMEM):
        raise StagError(rc, ctx.last_error())
    return rc, x, [s.as_dict() for s in stats], lat.value


def stag_time_kernels(ctx: Context, gauge: Gauge, prec="f32", nrhs=1, reps=200):
    """Average microseconds of the CG iteration's kernels: (D_oe stage, D_eo stage, update)."""
    us = (ctypes.c_double * 3)()
    ctx.check(lib.stag_time_kernels(ctx.h, gauge.h, PREC[prec] if isinstance(prec, str) else prec,
                                    int(nrhs), int(reps), us))
    return tuple(us)
