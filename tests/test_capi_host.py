"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/stag.h declares, and rejects bad arguments on the host before any
device work (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stag.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_boundary_calls():
    names = declared_functions()
    for must in ("stag_dslash", "stag_apply_A", "stag_cg_solve", "stag_solver_submit",
                 "stag_solver_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1111_0125_amd as s
    missing = [n for n in declared_functions() if not hasattr(s.lib, n)]
    assert not missing, missing


def test_null_and_bad_arguments_rejected_on_host():
    import paper_1111_0125_amd as s
    lib = s.lib
    assert lib.stag_version() >= 10000
    assert lib.stag_create(0, 0, None) == s.STAG_EINVAL
    assert lib.stag_destroy(None) == s.STAG_OK
    assert lib.stag_gauge_create(None, None, None, 0, 1, None) == s.STAG_EINVAL
    assert lib.stag_gauge_create_improved(None, None, None, None, 0, 1, None) == s.STAG_EINVAL
    assert lib.stag_field_create(None, None, 0, 0, 1, None) == s.STAG_EINVAL
    assert lib.stag_field_import(None, None, 0, None) == s.STAG_EINVAL
    assert lib.stag_dslash(None, None, None, None, None) == s.STAG_EINVAL
    assert lib.stag_apply_A(None, None, None, None, None, None) == s.STAG_EINVAL
    assert lib.stag_apply_A_noalloc(None, None, None, None, None, None) == s.STAG_EINVAL
    assert lib.stag_cg_solve(None, None, None, None, None, None, None, None) == s.STAG_EINVAL
    assert lib.stag_solver_submit(None, None, 0.1, 1, None, 1e-8, 1, None) == s.STAG_EINVAL
    assert lib.stag_solver_poll(None, 1, None, None, None) == s.STAG_EINVAL
    assert lib.stag_tune(None, None, 0, 1, None, None) == s.STAG_EINVAL
    assert isinstance(lib.stag_last_error(None), bytes)


def test_create_without_gpu_fails_cleanly():
    import paper_1111_0125_amd as s
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    rc = s.lib.stag_create(0, 0, ctypes.byref(h))
    assert rc in (s.STAG_EDEVICE, s.STAG_EINVAL)
    assert s.lib.stag_last_error(None)


ABI_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "stag.h"
#define F(T, m) printf("%s.%s %zu %zu\n", #T, #m, offsetof(T, m), sizeof(((T*)0)->m))
int main(void) {
    printf("stag_cg_params %zu\n", sizeof(stag_cg_params));
    printf("stag_cg_stats %zu\n", sizeof(stag_cg_stats));
    printf("stag_tune_cfg %zu\n", sizeof(stag_tune_cfg));
    F(stag_cg_params, tol); F(stag_cg_params, max_iter); F(stag_cg_params, inner_prec);
    F(stag_cg_params, delta); F(stag_cg_params, stall_iters); F(stag_cg_params, max_stall);
    F(stag_cg_params, graph_k); F(stag_cg_params, use_graph); F(stag_cg_params, use_x0);
    F(stag_cg_params, escalate); F(stag_cg_params, mixed_variant); F(stag_cg_params, small_lattice);
    F(stag_cg_stats, iters); F(stag_cg_stats, reliable_updates); F(stag_cg_stats, restarts);
    F(stag_cg_stats, status); F(stag_cg_stats, true_rel_res); F(stag_cg_stats, iter_rel_res);
    F(stag_cg_stats, seconds); F(stag_cg_stats, inner_final);
    F(stag_tune_cfg, S1); F(stag_tune_cfg, S2); F(stag_tune_cfg, nt); F(stag_tune_cfg, swizzle);
    printf("STAG_GAUGE_R12 %d STAG_MIXED_CARRY %d STAG_MIXED_RESTART %d STAG_MIXED_RELIABLE %d "
           "STAG_MIXED_FOLD_ONLY %d STAG_TUNE_IMPROVED %d\n", STAG_GAUGE_R12, STAG_MIXED_CARRY,
           STAG_MIXED_RESTART, STAG_MIXED_RELIABLE, STAG_MIXED_FOLD_ONLY, STAG_TUNE_IMPROVED);
    return 0;
}
"""


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the C structs have the header's layout (sizes
    and field offsets, from a C program compiled against stag.h)."""
    import shutil
    import subprocess

    import paper_1111_0125_amd as s
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "probe.c"
    src.write_text(ABI_PROBE)
    exe = tmp_path / "probe"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    sizes, fields, consts = {}, {}, {}
    for line in out:
        parts = line.split()
        if len(parts) == 2:
            sizes[parts[0]] = int(parts[1])
        elif len(parts) == 3:
            fields[parts[0]] = (int(parts[1]), int(parts[2]))
        elif line.startswith("STAG_GAUGE_R12"):
            it = iter(parts)
            consts = {k: int(v) for k, v in zip(it, it)}
    mirrors = {"stag_cg_params": s.CgParams, "stag_cg_stats": s.CgStats, "stag_tune_cfg": s.TuneCfg}
    for cname, py in mirrors.items():
        assert ctypes.sizeof(py) == sizes[cname], cname
        names = [f for f, _ in py._fields_]
        cnames = [k.split(".", 1)[1] for k in fields if k.startswith(cname + ".")]
        assert names == cnames, (cname, names, cnames)
        for f, _ in py._fields_:
            off, size = fields[f"{cname}.{f}"]
            assert getattr(py, f).offset == off and getattr(py, f).size == size, (cname, f)
    assert consts == {"STAG_GAUGE_R12": s.GAUGE_R12, "STAG_MIXED_CARRY": s.MIXED_CARRY,
                      "STAG_MIXED_RESTART": s.MIXED_RESTART,
                      "STAG_MIXED_RELIABLE": s.MIXED_RELIABLE,
                      "STAG_MIXED_FOLD_ONLY": s.MIXED_FOLD_ONLY,
                      "STAG_TUNE_IMPROVED": s.TUNE_IMPROVED}


def test_param_defaults():
    import paper_1111_0125_amd as s
    p = s.CgParams()
    s.lib.stag_cg_params_default(ctypes.byref(p))
    assert (p.tol, p.max_iter, p.inner_prec, p.delta) == (1e-8, 0, s.F64, 0.1)
    assert (p.stall_iters, p.max_stall, p.graph_k, p.use_graph) == (0, 20, 0, 1)
    assert (p.use_x0, p.escalate, p.mixed_variant, p.small_lattice) == (0, 1, s.MIXED_CARRY, 1)
    q = s.cg_params()
    assert (q.stall_iters, q.use_x0, q.escalate, q.mixed_variant) == (0, 0, 1, s.MIXED_CARRY)
    r = s.cg_params(inner="f16s", use_x0=True, mixed_variant="restart", escalate=False)
    assert (r.inner_prec, r.use_x0, r.mixed_variant, r.escalate) == (s.F16S, 1, s.MIXED_RESTART, 0)


def test_bench_refuses_more_than_one_gpu():
    """One lattice per GPU on a single GPU: --gpus N > 1 exits with a message
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "not supported" in r.stderr
    assert r.stdout == ""
