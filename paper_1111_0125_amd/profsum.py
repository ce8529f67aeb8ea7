#!/usr/bin/env python3
"""Summaries of rocprofv3 runs of bench.py, written as the markdown files under
profiles/ (what each file says, how it was made, a JSON block bench.py reads).

Run as a script from the repository root (it does not import the package,
whose __init__ loads the GPU library):

  profsum.py aapply    --json-fetch F.json --json-write W.json --fetch DIR --write DIR
                       [--json-trace T.json --trace DIR] [--unprofiled BENCH.json]
                       --cmd "..." [--cmd ...] --out FILE
      HBM traffic (FETCH_SIZE / WRITE_SIZE, calibrated on the run's own copy
      kernel) and traced durations of every (leg, launch shape) of
      `bench.py --a-apply-only`, attributed by launch order (each run's JSON
      output lists its own).
  iteration --json RUN.json --fetch DIR --write DIR --cmd ... --out FILE
      the same counters per kernel symbol for `bench.py --kernels-only`.
  headline  --bench UNPROFILED.json --trace DIR [--reps 200] --cmd ... --out FILE
      traced durations of the dominant iteration kernel of the headline solve:
      the solves' own launches and the timing loop's, beside the unprofiled
      bench's event timing.

Counter values are KiB per dispatch. A dispatch's HBM bytes are
FETCH_SIZE x 1024 x fetch_scale + WRITE_SIZE x 1024 x write_scale, the
scales making the copy kernel's counters equal its known bytes.
"""

from __future__ import annotations

import argparse
import csv
import glob
import importlib.util
import json
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _costs():
    spec = importlib.util.spec_from_file_location("stag_costs", os.path.join(HERE, "costs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    if len(hits) > 1:
        # one profiled process per directory is expected; take the largest
        hits.sort(key=os.path.getsize)
    return hits[-1]


def _num(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return float(row[n])
    raise KeyError(names)


def read_counters(d, counter):
    """[(dispatch id, kernel name, KiB)] in dispatch order, values of one
    counter summed over the rows of a dispatch."""
    path = _find(d, "counter_collection.csv")
    per = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            did = int(_num(row, "Dispatch_Id", "Correlation_Id"))
            name = row.get("Kernel_Name", "")
            v = _num(row, "Counter_Value")
            if did in per:
                per[did][1] += v
            else:
                per[did] = [name, v]
    return [(k, per[k][0], per[k][1]) for k in sorted(per)]


def read_trace(d):
    """[(dispatch id, kernel name, microseconds)] in dispatch order."""
    path = _find(d, "kernel_trace.csv")
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            did = int(_num(row, "Dispatch_Id", "Correlation_Id"))
            dur = (_num(row, "End_Timestamp") - _num(row, "Start_Timestamp")) * 1e-3
            out.append((did, row.get("Kernel_Name", ""), dur))
    out.sort()
    return out


HOP = re.compile(r"stag::k_hop<(\d+), (\d+), (\d+), (\d+), (true|false), (\d+)>")


def hop_parts(name):
    m = HOP.search(name)
    if not m:
        return None
    p, S, N, epi, nt, npairs = m.groups()
    return {"prec": int(p), "S": int(S), "N": int(N), "epi": int(epi), "nt": nt == "true",
            "npairs": int(npairs)}


def calibration(rows, copy_bytes, n_copy):
    """Scale of a counter from the last n_copy dispatches (the copy kernel)."""
    tail = rows[-n_copy:]
    names = {r[1] for r in tail}
    if len(names) != 1:
        raise SystemExit(f"the last {n_copy} dispatches are not one copy kernel: {names}")
    kib = statistics.mean(r[2] for r in tail)
    return copy_bytes / (kib * 1024.0), kib, names.pop()


PREC_NAME = {0: "f64", 1: "f32", 2: "f16s"}
VEC = re.compile(r"stag::k_vec<(\d+), (\d+), (\d+)>")


def leg_attrs(leg):
    improved = leg.startswith("improved_")
    base = leg[len("improved_"):] if improved else leg
    r12 = base.endswith("_r12")
    prec = base[:-4] if r12 else base
    return prec, r12, improved


def attribute_a(rows, order):
    """Split the k_hop dispatches of an --a-apply-only run into its (leg,
    shape) groups: each application is a stage-1 then a stage-2 launch."""
    hops = [r for r in rows if hop_parts(r[1])]
    need = sum(2 * o["applications"] for o in order)
    if len(hops) != need:
        raise SystemExit(f"{len(hops)} hop dispatches, launch order accounts for {need}")
    groups, i = [], 0
    for o in order:
        n = o["applications"]
        g = hops[i:i + 2 * n]
        i += 2 * n
        s1, s2 = g[0::2], g[1::2]
        for stage, lst in ((0, s1), (1, s2)):
            for r in lst:
                h = hop_parts(r[1])
                if h["epi"] != stage or h["S"] != o["S"] or h["nt"] != bool(o["nt"]):
                    raise SystemExit(f"dispatch {r} does not match {o} stage {stage + 1}")
        groups.append((o, s1, s2))
    return groups


def shape_key(o):
    return f"{o['leg']} S={o['S']} nt={o['nt']} swizzle={o['swizzle']}"


def _by_shape(rows, order, skip_warm=False):
    """{(leg, shape) key: ([stage-1 values], [stage-2 values])} over every group
    of that shape (sweep and final timing)."""
    acc = {}
    for o, s1, s2 in attribute_a(rows, order):
        a1, a2 = acc.setdefault(shape_key(o), ([], []))
        k = 3 if skip_warm and len(s1) > 3 else 0
        a1.extend(r[2] for r in s1[k:])
        a2.extend(r[2] for r in s2[k:])
    return acc


def cmd_aapply(a):
    costs = _costs()
    # each profiled run prints its own launch order (its final shapes may differ)
    jf, jw = json.load(open(a.json_fetch)), json.load(open(a.json_write))
    copy_bytes = jf["copy_bytes_each_way"]
    fetch = read_counters(a.fetch, "FETCH_SIZE")
    write = read_counters(a.write, "WRITE_SIZE")
    fs, fkib, cname = calibration(fetch, copy_bytes, 23)
    ws, wkib, _ = calibration(write, copy_bytes, 23)
    gf = _by_shape(fetch, jf["launch_order"])
    gw = _by_shape(write, jw["launch_order"])
    gt = (_by_shape(read_trace(a.trace), json.load(open(a.json_trace))["launch_order"], True)
          if a.trace else {})
    unp = json.load(open(a.unprofiled)) if a.unprofiled else None
    vh = 32 * 32 * 32 * 64 // 2
    legs = {}
    for key, (f1, f2) in gf.items():
        w1, w2 = gw[key]
        leg = key.split(" ", 1)[0]
        prec, r12, improved = leg_attrs(leg)
        alg = vh * costs.a_bytes_per_site(prec, r12=r12, improved=improved)
        alg1 = vh * costs.hop_bytes_per_site(prec, 1, r12=r12, improved=improved)
        alg2 = vh * costs.hop_bytes_per_site(prec, 2, r12=r12, improved=improved)
        F1, F2 = statistics.mean(f1), statistics.mean(f2)
        W1, W2 = statistics.mean(w1), statistics.mean(w2)
        b1 = F1 * 1024 * fs + W1 * 1024 * ws
        b2 = F2 * 1024 * fs + W2 * 1024 * ws
        e = {"fetch_kib": [round(F1, 1), round(F2, 1)], "write_kib": [round(W1, 1), round(W2, 1)],
             "hbm_bytes_per_A": int(round(b1 + b2)), "algorithmic_bytes_per_A": alg,
             "ratio": round((b1 + b2) / alg, 4),
             "stage_ratio": [round(b1 / alg1, 4), round(b2 / alg2, 4)],
             "dispatches": [len(f1), len(w1)]}
        if key in gt:
            t1, t2 = gt[key]
            e["traced_us"] = [round(statistics.mean(t1), 2), round(statistics.mean(t2), 2)]
        legs[key] = e
    blob = {"workload": "32^3x64 Haar links (seed 13), A = m^2 - D_eo D_oe, one RHS",
            "kernel_src_sha256": jf["kernel_src_sha256"], "fetch_scale": round(fs, 5),
            "write_scale": round(ws, 5), "copy_kernel": cname, "legs": legs}
    lines = ["# HBM traffic of A = m^2 - D_eo D_oe on 32^3 x 64 (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             "Commands (from the repository root on one MI355X; `<repo>` is that root), one counter "
             "per run, after an unprofiled run of the same program:", ""]
    lines += ["    " + c for c in a.cmd]
    lines += ["", "`bench.py --a-apply-only` builds the 32^3 x 64 Haar links (seed 13) and, per leg "
              "(Eq.5 with full links in f64 / f32 / f16+scale, with 12-parameter links in f64 / f32, "
              "and the improved operator in f64 / f32 / f16+scale), applies A in each of the twelve "
              "launch shapes (S = 1, 2, 4 lanes per site for both stages, non-temporal link loads on "
              "or off, XCD-aware block order on or off: 3 warm-ups and 10 timed applications each), "
              "then the fastest shape in three more runs of 3 + 50 applications (3 + 30 for the improved operator; the median run is reported), and at the end "
              "a 1 GiB elementwise copy (`torch.mul`, 3 + 20 launches). Every hop dispatch is "
              "attributed to its (leg, shape) by launch order, which the program prints; the two "
              "hop kernels of each application are stage 1 (`k_hop<prec, S, 1, 0, nt, pairs>`, "
              "D_oe) and stage 2 (`k_hop<prec, S, 1, 1, nt, pairs>`, D_eo with the m^2 update).", "",
              f"Calibration on the copy kernel (`{cname}`, {copy_bytes} bytes each way): FETCH_SIZE "
              f"reads {fkib:.1f} KiB per dispatch (scale {fs:.5f}), WRITE_SIZE {wkib:.1f} KiB "
              f"(scale {ws:.5f}).", ""]
    best = {}
    if unp:
        for grp in ("a_apply_32x32x32x64", "improved_32x32x32x64"):
            for leg, v in unp.get(grp, {}).items():
                if isinstance(v, dict) and "shape" in v:
                    name = leg if grp == "a_apply_32x32x32x64" else "improved_" + leg[2:]
                    best[name] = v
    lines += ["Per leg, the launch shape the unprofiled run found fastest (its `us_per_A` and "
              "fraction of 8 TB/s from torch events around 50 back-to-back applications), with the "
              "counters of that shape; every shape's counters are in the JSON block.", "",
              "| leg | shape | compulsory MB / A | HBM MB / A (counters) | ratio (stage 1, 2) | "
              "traced us (stage 1 + 2) | unprofiled us per A | frac of 8 TB/s |",
              "|---|---|---:|---:|---|---:|---:|---:|"]
    for leg, v in best.items():
        sh = v["shape"]
        key = f"{leg} S={sh['S1']} nt={sh['nt']} swizzle={sh['swizzle']}"
        e = legs.get(key)
        if not e:
            continue
        tr = e.get("traced_us")
        lines.append(f"| {leg} | S={sh['S1']} nt={sh['nt']} sw={sh['swizzle']} | "
                     f"{e['algorithmic_bytes_per_A'] / 1e6:.1f} | {e['hbm_bytes_per_A'] / 1e6:.1f} | "
                     f"{e['ratio']:.3f} ({e['stage_ratio'][0]:.3f}, {e['stage_ratio'][1]:.3f}) | "
                     f"{'' if not tr else f'{tr[0]:.1f} + {tr[1]:.1f} = {tr[0] + tr[1]:.1f}'} | "
                     f"{v['us_per_A']:.1f} | {v['frac_of_8TBs']:.3f} |")
    lines += ["", "`bench.py` reads the block below to fill `traffic_bytes_per_A` of each A-apply "
              "leg for the shape it picks, only while `kernel_src_sha256` (sha256 over the names and "
              "contents of the device-code sources `common.h`, `launch.h`, `kern.h`, `hop.hip`, "
              "`blas.hip`, `layout.hip` in `paper_1111_0125_amd/csrc/`) matches the current sources.",
              "", "```json", json.dumps(blob, indent=1), "```", ""]
    open(a.out, "w").write("\n".join(lines))
    print(f"wrote {a.out}: {len(legs)} (leg, shape) entries")


def cmd_iteration(a):
    costs = _costs()
    run = json.load(open(a.json))
    fetch = read_counters(a.fetch, "FETCH_SIZE")
    write = read_counters(a.write, "WRITE_SIZE")
    copy_bytes = run["copy_bytes_read"]
    fs, fkib, cname = calibration(fetch, copy_bytes, 3)
    ws, wkib, _ = calibration(write, run["copy_bytes_written"], 3)
    inner, links = run.get("inner", "f32"), run.get("links", "r12")
    traced = {}
    if a.trace:
        for _, name, us in read_trace(a.trace):
            traced.setdefault(name, []).append(us)
    vh = run["vh"]
    kern = {}
    for rows, key in ((fetch, "fetch"), (write, "write")):
        for _, name, v in rows:
            if "stag::k_hop" in name or "stag::k_vec" in name:
                kern.setdefault(name, {"fetch": [], "write": []})[key].append(v)
    out = {}
    for name, d in sorted(kern.items()):
        if not d["fetch"] or not d["write"]:
            continue
        h = hop_parts(name)
        if h:
            prec = PREC_NAME[h["prec"]]
            r12p = links == "r12"
            n = h["N"]
            # blocks of 8 or more right-hand sides, and of several on lattices of
            # 131072 sites per parity or more, form the direction in a pass of
            # their own: their hop stages read d as stored
            lazy = n == 1 or (n < 8 and vh < 131072)
            if h["epi"] == 0:
                alg = vh * costs.hop_bytes_per_site(prec, 1, n, lazy=lazy, r12=r12p)
            elif h["epi"] == 2:
                alg = vh * costs.hop_bytes_per_site(prec, 2, n, lazy=lazy, r12=r12p)
            else:
                continue
        else:
            m = VEC.search(name)
            if not m or int(m.group(3)) not in (2, 3):
                continue
            prec = PREC_NAME[int(m.group(1))]
            alg = vh * int(m.group(2)) * costs.update_bytes_per_site(prec, int(m.group(3)) == 3)
        F, W = statistics.mean(d["fetch"]), statistics.mean(d["write"])
        b = F * 1024 * fs + W * 1024 * ws
        out[name] = {"fetch_kib": round(F, 1), "write_kib": round(W, 1),
                     "dispatches": [len(d["fetch"]), len(d["write"])],
                     "hbm_bytes_per_launch": int(round(b)), "algorithmic_bytes_per_launch": alg,
                     "ratio": round(b / alg, 4)}
        if traced.get(name):
            t = statistics.mean(traced[name])
            out[name]["traced_us"] = round(t, 3)
            out[name]["compulsory_GB/s_traced"] = round(alg / (t * 1e-6) / 1e9, 1)
    blob = {"workload": a.workload,
            "links": links, "kernel_src_sha256": run["kernel_src_sha256"],
            "fetch_scale": round(fs, 5), "write_scale": round(ws, 5), "kernels": out}
    lines = [f"# HBM traffic of the iteration kernels: {a.workload} (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             "Commands (from the repository root on one MI355X; `<repo>` is that root), one counter "
             "per run:", ""]
    lines += ["    " + c for c in a.cmd]
    lines += ["", a.program, "Counter values are KiB per dispatch, averaged over all "
              "dispatches of each kernel symbol (the same work every launch). Template arguments: "
              "`k_hop<prec, S, N, epilogue, nt, pairs>` (prec 0 = f64, 1 = f32, 2 = f16s; S lanes "
              "per site; N right-hand sides; epilogue 0 = stage 1, 2 = stage 2 with <d, A d>), "
              "`k_vec<prec, N, op>` (op 3 = mixed update, 2 = fp64 CG update). Compulsory bytes: "
              "`paper_1111_0125_amd/costs.py` (blocks of several right-hand sides on this many "
              "sites read the direction as stored; one right-hand side forms it in the hop "
              "stages from r and the previous d).", "",
              f"Calibration on the copy kernel (`{cname}`): FETCH_SIZE reads {fkib:.1f} KiB per "
              f"dispatch (scale {fs:.5f}), WRITE_SIZE {wkib:.1f} KiB (scale {ws:.5f}).", "",
              "HBM MB counts the bytes between L2 and the memory fabric (MALL or HBM); "
              "traced us is the mean kernel duration over every dispatch of the symbol in the "
              "`--kernel-trace` run of the same program (when given).", "",
              "| kernel | dispatches (fetch / write run) | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per "
              "launch | compulsory MB | ratio | traced us | compulsory GB/s |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name, e in out.items():
        lines.append(f"| `{name}` | {e['dispatches'][0]} / {e['dispatches'][1]} | {e['fetch_kib']} | "
                     f"{e['write_kib']} | {e['hbm_bytes_per_launch'] / 1e6:.2f} | "
                     f"{e['algorithmic_bytes_per_launch'] / 1e6:.2f} | {e['ratio']:.3f} | "
                     f"{e.get('traced_us', '')} | {e.get('compulsory_GB/s_traced', '')} |")
    lines += ["", "`bench.py` reads the block below to fill `roofline.traffic` for its dominant "
              "kernel, only while `kernel_src_sha256` matches the current device-code sources and "
              "the links match.", "", "```json", json.dumps(blob, indent=1), "```", ""]
    open(a.out, "w").write("\n".join(lines))
    print(f"wrote {a.out}: {len(out)} kernels")


def cmd_headline(a):
    bench = json.load(open(a.bench))
    sym = bench["roofline"]["kernel_symbol"]
    trace = read_trace(a.trace)
    mine = [r for r in trace if r[1] == sym]
    if len(mine) < a.reps:
        raise SystemExit(f"{len(mine)} dispatches of {sym}, fewer than the {a.reps} timing launches")
    loop = [r[2] for r in mine[-a.reps:]]
    solves = [r[2] for r in mine[:-(a.reps + 3)]]
    active = [d for d in solves if d > a.idle_us]
    ev = bench["roofline"]["avg_us"]
    byts = bench["roofline"]["bytes_per_launch"]
    rows = [("timing loop (`stag_time_kernels`, last %d launches)" % a.reps, loop),
            ("the solves' launches (warm-up and timed solves, HIP graphs; the eager solve)", solves),
            (f"the solves' launches longer than {a.idle_us} us (active slot)", active)]
    lines = [f"# rocprofv3 kernel trace: the dominant kernel of the {bench['config']['workload']}", "",
             "Commands (from the repository root on one MI355X; `<repo>` is that root), the "
             "unprofiled run first (it also writes the launch-shape table the profiled run then "
             "loads, so both run the same shapes and the trace has no autotuner sweep):", ""]
    lines += ["    " + c for c in a.cmd]
    lines += ["", f"Kernel: `{sym}` ({bench['roofline']['kernel']}), {byts} compulsory bytes per "
              "launch. In the trace its launches are the warm-up and timed solves' (graph "
              "replays; a launch whose slot is inactive, after a flag until its segment's fix-up "
              "or after convergence, reads the state and exits), one more solve's launched "
              "eagerly (`roofline.in_solve`), and last the 3 + 200 launches of "
              "`stag_time_kernels` that `roofline` is computed from.", "",
              "| launches | count | mean us | median us | GB/s at the mean | frac of 8 TB/s |",
              "|---|---:|---:|---:|---:|---:|"]
    for label, d in rows:
        if not d:
            continue
        m = statistics.mean(d)
        lines.append(f"| {label} | {len(d)} | {m:.3f} | {statistics.median(d):.3f} | "
                     f"{byts / (m * 1e-6) / 1e9:.1f} | {byts / (m * 1e-6) / 8e12:.4f} |")
    ins = bench["roofline"].get("in_solve")
    if ins:
        lines += ["", f"The unprofiled run's eager solve (`roofline.in_solve`): {ins['avg_us']} us per "
                  f"launch over {ins['launches']} launches, {ins['frac']} of 8 TB/s."]
    lines += ["", f"The unprofiled run's `roofline`: {ev} us per launch (events at the kernel's start "
              f"and end around each of the 200 launches), {bench['roofline']['achieved']} GB/s = "
              f"{bench['roofline']['frac']} of 8 TB/s; its solve took "
              f"{bench['solve']['time_to_1e-8_ms']} ms ({bench['solve']['iters']} iterations, "
              f"{bench['solve']['reliable_updates']} reliable updates).", ""]
    stats = _find(a.trace, "kernel_stats.csv")
    with open(stats, newline="") as f:
        top = list(csv.DictReader(f))[:10]
    lines += ["Top kernels of the profiled run by total time (rocprofv3 `--stats`):", "",
              "| kernel | calls | total us | avg us | min us | max us | % |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for r in top:
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['MinNs']) / 1e3:.3f} | "
                     f"{float(r['MaxNs']) / 1e3:.3f} | {float(r['Percentage']):.2f} |")
    lines.append("")
    open(a.out, "w").write("\n".join(lines))
    print(f"wrote {a.out}")


def cmd_solves(a):
    """Per-kernel durations of the 32^3x64 solves inside the solves themselves
    (graph replays), against each kernel's compulsory bytes per launch."""
    costs = _costs()
    run = json.load(open(a.json))
    vh = int(run["vh"])
    r12 = run.get("links") == "r12"
    names = {0: "f64", 1: "f32", 2: "f16s"}
    trace = read_trace(a.trace)
    per = {}
    for _, name, dur in trace:
        per.setdefault(name, []).append(dur)

    def role_bytes(name):
        h = hop_parts(name)
        if h:
            prec, n = names[h["prec"]], h["N"]
            if h["prec"] == 0:
                return ("fp64 fix-up stage %d (reliable update or check; idle launches exit early)"
                        % (1 if h["epi"] == 0 else 2)), None
            if h["epi"] == 0:
                return f"hop stage 1, {prec} (t = D_oe d)", vh * costs.hop_bytes_per_site(
                    prec, 1, n, lazy=False, r12=r12)
            if h["epi"] == 2:
                return f"hop stage 2, {prec} (Ad = m^2 d - D_eo t, <d, Ad>)", vh * costs.hop_bytes_per_site(
                    prec, 2, n, lazy=False, r12=r12)
            return f"hop {prec} epilogue {h['epi']}", None
        m = VEC.search(name)
        if m:
            prec, n, op = names[int(m.group(1))], int(m.group(2)), int(m.group(3))
            if op == 3:
                return f"update, {prec} (y += a d, r -= a Ad, |r|^2)", vh * n * costs.update_bytes_per_site(prec, True)
            if op == 5:
                return f"direction pass, {prec} (d = r + beta d)", vh * n * 3 * costs.SPINOR_BYTES[prec]
            return f"vector op {op}, {prec}", None
        if "k_finalize" in name:
            return "one-block finalisation of a reduction", None
        return None, None

    rows = []
    for name, d in per.items():
        role, byts = role_bytes(name)
        if role is None:
            continue
        med = statistics.median(d)
        rows.append((sum(d), name, role, len(d), statistics.mean(d), med, byts))
    rows.sort(reverse=True)
    lines = [f"# rocprofv3 kernel trace inside the solves: {run['workload']} Haar links, "
             f"m = {run['mass']}, {run['tol']}, fp32 and fp16+scale inner iterations", "",
             "Commands (from the repository root on one MI355X; `<repo>` is that root), the "
             "unprofiled run first (it writes the launch-shape table the traced run loads, so the "
             "trace has no autotuner sweep):", ""]
    lines += ["    " + c for c in a.cmd]
    sol = run["solves"]
    lines += ["", "`bench.py --c3-solves-only` builds the lattice with 12-parameter links and runs, per "
              "inner precision, a warm-up and a timed solve (HIP graph replays): "
              + "; ".join(f"{k}: {v['iters']} iterations, {v['reliable_updates']} reliable updates, "
                          f"{v['ms']} ms traced" for k, v in sol.items())
              + ". On this lattice an iteration is the direction pass, the two hop stages, the "
              "update and two one-block finalisations; every few iterations come the fp64 "
              "fix-up launches, idle unless a slot is flagged. The bytes are each kernel's "
              "compulsory bytes per launch (the links and every vector once); the median "
              "duration stands for an active launch (a handful of launches per solve run idle "
              "after a flag or after convergence).", "",
              "| kernel | role | launches | mean us | median us | compulsory MB | GB/s at the median | frac of 8 TB/s |",
              "|---|---|---:|---:|---:|---:|---:|---:|"]
    for tot, name, role, n, mean, med, byts in rows:
        if byts:
            gbs = byts / (med * 1e-6) / 1e9
            lines.append(f"| `{name}` | {role} | {n} | {mean:.2f} | {med:.2f} | {byts / 1e6:.1f} | "
                         f"{gbs:.1f} | {gbs / 8000:.3f} |")
        else:
            lines.append(f"| `{name}` | {role} | {n} | {mean:.2f} | {med:.2f} | | | |")
    lines.append("")
    open(a.out, "w").write("\n".join(lines))
    print(f"wrote {a.out}")


def main(argv=None):
    ap = argparse.ArgumentParser(description="rocprofv3 summaries for profiles/")
    sub = ap.add_subparsers(dest="what", required=True)
    p = sub.add_parser("aapply")
    p.add_argument("--json-fetch", required=True)
    p.add_argument("--json-write", required=True)
    p.add_argument("--json-trace")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--trace")
    p.add_argument("--unprofiled")
    p.add_argument("--cmd", action="append", default=[])
    p.add_argument("--out", required=True)
    p = sub.add_parser("iteration")
    p.add_argument("--json", required=True)
    p.add_argument("--trace")
    p.add_argument("--workload", default="16^3x32 exp(i 0.3 H) links, the CG iteration kernels "
                   "of every precision (f64: plain CG; f32, f16s: mixed), one RHS")
    p.add_argument("--program", default="`bench.py --kernels-only` builds the 16^3x32 workload, "
                   "runs the autotuner over every launch shape of the three iteration kernels (no "
                   "shapes from a table), launches them 20 more times as `stag_time_kernels` does, "
                   "then a 256 MiB elementwise copy (`torch.mul`, 3 launches).")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--cmd", action="append", default=[])
    p.add_argument("--out", required=True)
    p = sub.add_parser("solves")
    p.add_argument("--json", required=True)
    p.add_argument("--trace", required=True)
    p.add_argument("--cmd", action="append", default=[])
    p.add_argument("--out", required=True)
    p = sub.add_parser("headline")
    p.add_argument("--bench", required=True)
    p.add_argument("--trace", required=True)
    p.add_argument("--reps", type=int, default=200)
    p.add_argument("--idle-us", type=float, default=3.0)
    p.add_argument("--cmd", action="append", default=[])
    p.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    {"aapply": cmd_aapply, "iteration": cmd_iteration, "solves": cmd_solves,
     "headline": cmd_headline}[a.what](a)


if __name__ == "__main__":
    sys.exit(main())
