"""Write oracle_counts.json: iteration counts of the oracle's solvers on the
benchmark workloads, which the GPU tests compare against (the numpy
emulation takes minutes at these sizes, too long inside a GPU test).

Calls only the oracle and the seeded input generators:
    python3 tests/golden/make_oracle_counts.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import c as oc  # noqa: E402
from oracle import stag as ostag  # noqa: E402


def c2():
    """16^3 x 32, exp(i 0.3 H) links, m = 0.01, tol 1e-8: Fig.1 fp64 CG (C
    oracle) and the Sec.3.2 scheme with fp32 storage (numpy emulation)."""
    name = "c2_16x16x16x32"
    cfg = synth.CONFIGS[name]
    L, m, tol = cfg["L"], cfg["mass"], cfg["tol"]
    U = synth.config_links(name)
    b = synth.config_rhs(name)[0]
    _, s64 = oc.cg(U, b, L, m, tol)
    _, s32 = ostag.mixed_cg(U, L, m, b, tol, prec="f32")
    return {"workload": name, "lattice": list(L), "mass": m, "tol": tol,
            "fig1_fp64_cg": {"iters": s64["iters"], "true_rel_res": s64["true_rel_res"]},
            "sec32_fp32_mixed": {"iters": s32["iters"], "updates": s32["updates"],
                                 "true_rel_res": s32["true_rel_res"], "status": s32["status"]}}


def main():
    out = {"_source": "written by tests/golden/make_oracle_counts.py from oracle/ only",
           "c2_16x16x16x32": c2()}
    with open(os.path.join(HERE, "oracle_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
