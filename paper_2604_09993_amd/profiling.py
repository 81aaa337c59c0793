"""Profiling helpers: HBM counter calibration and rocprofv3 summaries.

    python -m paper_2604_09993_amd.profiling copy
        one plain device copy of 64 Mi doubles (512 MiB each way), three
        dispatches: run under ``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc
        WRITE_SIZE`` to get the bytes each counter reports per byte moved.

    python -m paper_2604_09993_amd.profiling summarize --trace D --fetch D \
        --write D --cfetch D --cwrite D --md OUT.md --traffic OUT.json [--cmd-* ...]
        reads the rocprofv3 result databases under the given output folders
        (kernel trace with --stats; FETCH_SIZE and WRITE_SIZE runs of the same
        program; the two calibration runs) and writes the markdown summary and
        the per-kernel traffic record (calibrated bytes per dispatch, tied to
        the hash of the kernel sources).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sqlite3
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_ELEMS = 64 * 1024 * 1024   # doubles per calibration copy


def kernel_sources_sha256() -> str:
    """Hash of the device-code sources (the .hip files and the headers they
    include): identifies the measured kernels.  Host-only files (.cpp) and the
    ABI header's declarations do not change a kernel and are left out."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def run_copy():
    import torch
    x = torch.ones(COPY_ELEMS, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied 3 x {COPY_ELEMS * 8} bytes", flush=True)


def _dbs(folder):
    found = sorted(glob.glob(os.path.join(folder, "**", "*_results.db"), recursive=True))
    if not found:
        raise FileNotFoundError(f"no rocprofv3 results database under {folder}")
    return found


def _short(name: str) -> str:
    """Kernel name without the namespace and argument list."""
    n = name.replace("cis::", "")
    if n.startswith("void "):
        n = n[5:]
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip().replace("> >", ">>")


def kernel_stats(folder):
    rows = defaultdict(lambda: [0, 0.0])
    for db in _dbs(folder):
        c = sqlite3.connect(db).cursor()
        for name, calls, total, _avg, _pct in c.execute(
                "select name, total_calls, total_duration, average, percentage from top_kernels"):
            r = rows[_short(name)]
            r[0] += int(calls)
            r[1] += float(total)
    # the top_kernels view reports microseconds
    return {k: dict(calls=v[0], total_us=v[1], avg_us=v[1] / max(v[0], 1))
            for k, v in rows.items()}


def counter_means(folder, counter):
    vals = defaultdict(list)
    for db in _dbs(folder):
        c = sqlite3.connect(db).cursor()
        cols = [r[1] for r in c.execute("pragma table_info(counters_collection)")]
        ci = {n: i for i, n in enumerate(cols)}
        kcol = ci.get("kernel_name", ci.get("name"))
        for r in c.execute("select * from counters_collection"):
            if r[ci["counter_name"]] == counter:
                vals[_short(r[kcol])].append(float(r[ci["value"]]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


def interval_bytes(model, K, op, C=1, dsize=8):
    """Algorithmic HBM bytes of one interval (each datum moved once).

    Every operation reads X_k, X_k+1, U_k, U_k+1, s_k and the P parameters.
    discretize writes A (nx x nx), B- and B+ (nx x m), S, defect and x_prop;
    defects writes defect, x_prop and the K/C body-state checkpoints; the
    reverse sweep also reads the checkpoints and the seed, and writes gX_k,
    the two control-gradient halves, gs_k and the P parameter partials.
    """
    nx, m, n, P = model.nx, model.m, model.n, model.n_params
    read = 2 * nx + 2 * m + 1 + P
    if op == "discretize":
        return dsize * (read + nx * nx + 2 * nx * m + 3 * nx)
    if op == "defects":
        return dsize * (read + 2 * nx + (K // C) * n)
    if op == "adjoint":
        return dsize * (read + (K // C) * n + nx + nx + 2 * m + 1 + P)
    raise ValueError(op)


def _topo(model):
    return f"Topo<{model.legs}, {model.depth}"


def bench_algorithmic_bytes():
    """Algorithmic bytes per launch of the kernels bench.py runs, keyed by
    kernel-name prefix (the batch kernels by dtype and topology: every form
    the tuner tries processes the same group)."""
    from . import synth

    def auto_ckpt(K):   # a plan's default spacing: the largest divisor of K not above 8
        return max(c for c in range(1, 9) if K % c == 0)
    out = {}
    model, data, K = synth.make_workload("cheetah7_N50_K20")
    N = data["s"].shape[0]
    t = _topo(model)
    out[f"k_discretize<double, {t}"] = N * interval_bytes(model, K, "discretize")
    out[f"k_discretize<float, {t}"] = N * interval_bytes(model, K, "discretize", dsize=4)
    out[f"k_defects<double, {t}"] = N * interval_bytes(model, K, "defects", C=5)
    out[f"k_adjoint4<double, {t}"] = N * interval_bytes(model, K, "adjoint", C=5)
    out[f"k_adjoint<double, {t}"] = N * interval_bytes(model, K, "adjoint", C=5)
    groups = {}
    for m_, d, k in synth.mixed_batch():
        groups.setdefault(_topo(m_), []).append((m_, d["s"].shape[0], k))
    for t, items in groups.items():
        def tot(op, cf=lambda k: 1, items=items):
            return sum(n * interval_bytes(m_, k, op, C=cf(k)) for m_, n, k in items)
        out[f"k_discretize_batch<double, {t}"] = tot("discretize")
        out[f"k_defects_batch<double, {t}"] = tot("defects", auto_ckpt)
        out[f"k_defects_lane_batch<double, {t}"] = tot("defects", auto_ckpt)
        out[f"k_adjoint4_batch<double, {t}"] = tot("adjoint", auto_ckpt)
        out[f"k_adjoint3_batch<double, {t}"] = tot("adjoint", auto_ckpt)
        out[f"k_adjoint_batch<double, {t}"] = tot("adjoint", auto_ckpt)
    for t, items in groups.items():
        for ds, tn in ((8, "double"), (4, "float")):
            rec = sum(n * split_bytes(m_, ds)[0] for m_, n, k in items)
            tan = sum(n * split_bytes(m_, ds)[1] for m_, n, k in items)
            out[f"k_coefrec_batch<{tn}, {t}"] = rec
            out[f"k_tangent_batch<{tn}, {t}"] = tan
    imodel, idata = synth.impact_workload("quad13_x64")
    out[f"k_impact<ImpTopo<{imodel.legs}, {imodel.depth}>"] = \
        idata["Xp"].shape[0] * impact_bytes(imodel)
    qb = synth.workload_batch("quad13_N200_K20_x64")
    t = _topo(qb[0][0])
    out[f"k_discretize_batch<double, {t}"] = sum(d["s"].shape[0] * interval_bytes(m_, k, "discretize")
                                                 for m_, d, k in qb)
    out[f"k_discretize_batch<float, {t}"] = sum(d["s"].shape[0] *
                                                interval_bytes(m_, k, "discretize", dsize=4)
                                                for m_, d, k in qb)
    for ds, tn in ((8, "double"), (4, "float")):
        out[f"k_coefrec_batch<{tn}, {t}"] = sum(d["s"].shape[0] * split_bytes(m_, ds)[0]
                                               for m_, d, k in qb)
        out[f"k_tangent_batch<{tn}, {t}"] = sum(d["s"].shape[0] * split_bytes(m_, ds)[1]
                                               for m_, d, k in qb)
    return out


def split_bytes(model, dsize=8):
    """Algorithmic bytes of one interval in the two launches of the split form:
    the record launch reads the interval's inputs and writes S, the defect,
    F~ and the integral-state columns of A; the tangent launch writes the
    x-state columns of A and B-, B+ (the stage records between them are
    intermediate, not algorithmic, traffic)."""
    nx, m, n, P = model.nx, model.m, model.n, model.n_params
    rec = dsize * ((2 * nx + 2 * m + 1 + P) + 3 * nx + nx * (nx - n))
    tan = dsize * (nx * n + 2 * nx * m)
    return rec, tan


def impact_bytes(model, dsize=8):
    """Algorithmic bytes of one node of the impact map: it reads x~+, x~-,
    Phi and Gamma of the node and writes G~, Theta, Psi and the compact
    Jacobians JGv [3 nb][7 nb + 2 nc] and JTc [10 nc][14]."""
    nx, nb, nc, ny = model.nx, model.nb, model.nc, model.ny
    read = 2 * nx + 3 * nc
    write = nx + 10 * nc + ny + 3 * nb * (7 * nb + 2 * nc) + 140 * nc
    return dsize * (read + write)


PHI_FJ = {2: 300, 5: 700, 7: 1000, 13: 2000}   # per-stage RHS + Jacobian FLOP by body count


def interval_flops(model, K):
    """Algorithmic forward FLOPs of one interval, K [8 nnz(J) c + 14 nx c + 4 phi_fJ],
    and the tangent launch's share K [8 nnz(J) + 14 nx] (c - 1) in the split form."""
    nnz = 2 * 3 * model.nb + 2 * model.nb + 4 * model.nj + 4 * model.nc
    c = model.n + 2 * model.m + 1
    phi = PHI_FJ.get(model.nb, 1000)
    total = K * (8 * nnz * c + 14 * model.nx * c + 4 * phi)
    tangent = K * (8 * nnz + 14 * model.nx) * (c - 1)
    return total, tangent


def bench_algorithmic_flops():
    """Algorithmic FLOPs per launch of the forward kernels of bench.py's
    batched workloads, keyed by kernel-name prefix."""
    from . import synth
    out = {}
    groups = {}
    for m_, d, k in synth.mixed_batch():
        groups.setdefault(_topo(m_), []).append((m_, d["s"].shape[0], k))
    qb = synth.workload_batch("quad13_N200_K20_x64")
    groups[_topo(qb[0][0])] = [(m_, d["s"].shape[0], k) for m_, d, k in qb]
    for t, items in groups.items():
        tot = sum(n * interval_flops(m_, k)[0] for m_, n, k in items)
        tan = sum(n * interval_flops(m_, k)[1] for m_, n, k in items)
        for tn in ("double", "float"):
            out[f"k_discretize_batch<{tn}, {t}"] = tot
            out[f"k_coefrec_batch<{tn}, {t}"] = tot - tan
            out[f"k_tangent_batch<{tn}, {t}"] = tan
    return out


def valu_summary(a):
    """Markdown table of VALU/LDS counters per kernel: counter FLOPs against
    algorithmic FLOPs, achieved counter FLOP/s, VALU issue estimate."""
    import csv
    per = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> per-dispatch values
    for path in a.csv:
        vals = defaultdict(lambda: defaultdict(float))
        with open(path) as fh:
            for r in csv.DictReader(fh):
                vals[(_short(r["Kernel_Name"]), r["Dispatch_Id"])][r["Counter_Name"]] += \
                    float(r["Counter_Value"])
        for (k, _), cs in vals.items():
            for c, v in cs.items():
                per[k][c].append(v)
    mean = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in per.items()}
    stats = kernel_stats(a.trace) if a.trace else {}
    algo = bench_algorithmic_flops()
    clock = 2.4e9
    simds = 1024
    lines = [f"# {a.title}", "", "Box: one MI355X (gfx950). All commands run from the repository root.",
             "", "Counter passes (one rocprofv3 run each, --pmc only):", ""]
    lines += [f"    {c}" for c in a.commands]
    lines += ["", f"Kernel durations: `{a.cmd_trace}`", "",
              "Per dispatch: F64 FLOP = 64 (2 FMA + ADD + MUL) over the F64 VALU instruction counters "
              "(64 lanes per wave instruction, inactive lanes included), likewise F32; "
              "`VALU issue` = SQ_INSTS_VALU x 4 cycles (a 64-lane instruction at 16 lanes per "
              "clock) / (kernel time x 2.4 GHz x 1024 SIMDs), an estimate of the fraction of "
              "SIMD cycles spent issuing VALU instructions.", "",
              "| kernel | avg µs | F64 FLOP (counter) | algorithmic FLOP | counter / algorithmic | "
              "counter TFLOP/s | algorithmic TFLOP/s | VALU instr | VALU issue | LDS instr | "
              "LDS bank-conflict cycles | waves |",
              "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(mean, key=lambda k: -stats.get(k, {}).get("total_us", 0.0)):
        if not k.startswith("k_"):
            continue
        c = mean[k]
        f64 = 64 * (2 * c.get("SQ_INSTS_VALU_FMA_F64", 0) + c.get("SQ_INSTS_VALU_ADD_F64", 0) +
                    c.get("SQ_INSTS_VALU_MUL_F64", 0))
        f32 = 64 * (2 * c.get("SQ_INSTS_VALU_FMA_F32", 0) + c.get("SQ_INSTS_VALU_ADD_F32", 0) +
                    c.get("SQ_INSTS_VALU_MUL_F32", 0))
        fl = f64 if f64 >= f32 else f32
        al = _match(algo, k)
        us = stats.get(k, {}).get("avg_us")
        t = us * 1e-6 if us else None
        issue = c.get("SQ_INSTS_VALU", 0) * 4 / (t * clock * simds) if t else None
        fmt = lambda v, f="{:.3g}": "" if v is None else f.format(v)
        lines.append("| `{}` | {} | {} | {} | {} | {} | {} | {} | {} | {} | {} | {} |".format(
            k, fmt(us, "{:.1f}"), fmt(fl), fmt(al), fmt(fl / al if al else None, "{:.2f}"),
            fmt(fl / t / 1e12 if t else None, "{:.2f}"),
            fmt(al / t / 1e12 if (t and al) else None, "{:.2f}"),
            fmt(c.get("SQ_INSTS_VALU")), fmt(issue, "{:.2f}"), fmt(c.get("SQ_INSTS_LDS")),
            fmt(c.get("SQ_LDS_BANK_CONFLICT")), fmt(c.get("SQ_WAVES"))))
    lines += ["", "Raw counters per dispatch (means):", ""]
    names = sorted({n for cs in mean.values() for n in cs})
    lines.append("| kernel | " + " | ".join(names) + " |")
    lines.append("|---|" + "---|" * len(names))
    for k in sorted(mean):
        if not k.startswith("k_"):
            continue
        lines.append(f"| `{k}` | " + " | ".join(f"{mean[k].get(n, 0):.4g}" for n in names) + " |")
    if a.note:
        lines += ["", a.note]
    with open(a.md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {a.md}")


def _match(table, kernel):
    best = None
    for pre, v in table.items():
        if kernel.startswith(pre) and kernel[len(pre)] in ",>" and (best is None or len(pre) > len(best[0])):
            best = (pre, v)
    return None if best is None else best[1]


def summarize(a):
    stats = kernel_stats(a.trace)
    fetch = counter_means(a.fetch, "FETCH_SIZE")
    write = counter_means(a.write, "WRITE_SIZE")
    cf = counter_means(a.cfetch, "FETCH_SIZE")
    cw = counter_means(a.cwrite, "WRITE_SIZE")
    moved_kib = COPY_ELEMS * 8 / 1024.0
    copy_f = max(cf.values()) if cf else None
    copy_w = max(cw.values()) if cw else None
    sf = moved_kib / copy_f if copy_f else 1.0
    sw = moved_kib / copy_w if copy_w else 1.0
    algo = json.loads(a.algorithmic) if a.algorithmic else bench_algorithmic_bytes()
    lines = [f"# {a.title}", "", "Box: one MI355X (gfx950). All commands run from the repository root.",
             "", "## Kernel trace", "", f"    {a.cmd_trace}", "",
             "| kernel | calls | total µs | average µs |", "|---|---|---|---|"]
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["total_us"]):
        lines.append(f"| `{k}` | {v['calls']} | {v['total_us']:.1f} | {v['avg_us']:.2f} |")
    lines += ["", "## HBM traffic (PMC), per dispatch", "", f"    {a.cmd_fetch}", f"    {a.cmd_write}",
              "", "Calibration: a plain copy of 64 Mi doubles (512 MiB each way), 3 dispatches:", "",
              f"    {a.cmd_cfetch}", f"    {a.cmd_cwrite}", "",
              f"copy: FETCH_SIZE {copy_f:,.1f} KiB, WRITE_SIZE {copy_w:,.1f} KiB per dispatch for "
              f"{moved_kib:,.0f} KiB moved each way -> scale factors {sf:.3f} (fetch) and "
              f"{sw:.3f} (write).", "",
              "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read bytes | write bytes | algorithmic bytes |",
              "|---|---|---|---|---|---|"]
    rec = {"sources_sha256": kernel_sources_sha256(), "scale_fetch": sf, "scale_write": sw,
           "commands": [a.cmd_fetch, a.cmd_write, a.cmd_cfetch, a.cmd_cwrite], "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        f_kib, w_kib = fetch.get(k, 0.0), write.get(k, 0.0)
        rb, wb = f_kib * 1024 * sf, w_kib * 1024 * sw
        al = _match(algo, k)
        lines.append(f"| `{k}` | {f_kib:,.1f} | {w_kib:,.1f} | {rb:,.0f} | {wb:,.0f} | "
                     f"{'' if al is None else f'{al:,.0f}'} |")
        rec["kernels"][k] = {"fetch_bytes": rb, "write_bytes": wb, "algorithmic_bytes": al}
    if a.note:
        lines += ["", a.note]
    with open(a.md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(a.traffic, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {a.md} and {a.traffic}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    s = sub.add_parser("summarize")
    for k in ("trace", "fetch", "write", "cfetch", "cwrite", "md", "traffic"):
        s.add_argument("--" + k, required=True)
    for k in ("trace", "fetch", "write", "cfetch", "cwrite"):
        s.add_argument("--cmd-" + k, default="")
    s.add_argument("--title", default="Kernel profile")
    s.add_argument("--algorithmic", default="",
                   help="JSON {kernel-name prefix: algorithmic bytes per launch}; default: "
                        "the workloads of bench.py")
    s.add_argument("--note", default="")
    v = sub.add_parser("valu")
    v.add_argument("--csv", nargs="+", required=True, help="rocprofv3 CSV counter files")
    v.add_argument("--trace", default="", help="kernel-trace output folder (durations)")
    v.add_argument("--commands", nargs="*", default=[], help="the counter commands, for the record")
    v.add_argument("--cmd-trace", default="")
    v.add_argument("--md", required=True)
    v.add_argument("--title", default="VALU and LDS counters")
    v.add_argument("--note", default="")
    a = ap.parse_args()
    if a.cmd == "copy":
        run_copy()
    elif a.cmd == "valu":
        valu_summary(a)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
