#!/usr/bin/env python3
"""Discretized intervals/s of the CI-SCvx linearize-and-discretize step on one MI355X.

Headline workload: 64 trajectories of a planar 13-body quadruped-shaped chain
(torso + four 3-link legs, 12 revolute joints, 4 foot contacts; nx = 83,
m = 48), N = 200 intervals each (12,800 intervals), K = 20 RK4 substeps,
FP64, synthetic seeded node data resident in HBM before timing.  One step =
one replay of the batch plan's HIP graph: every interval's A, B-, B+, S,
defect and F~.

Prints one JSON line.  Extra fields: the FP32 form and the gradient step
(defects with checkpoints + reverse sweep + reduction) of the same batch;
the uneven 256-trajectory batch (hopper / cheetah7 / biped5); the
single-trajectory cheetah7 (N = 50, K = 20) and hopper (N = 20, K = 10)
calls; substep blocking with VALU and MFMA composition on one quad13
trajectory; the parity of every timed output against the CPU oracle
(sampled); the roofline of the dominant kernels; the CPU oracle baseline.
"""
import argparse
import ctypes
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12   # MI355X FP64 vector FLOP/s (AMD published)
PEAK_FP32_VALU = 157.3e12
PHI_FJ = {2: 300, 5: 700, 7: 1000, 13: 2000}   # per-stage RHS + Jacobian FLOP by body count


def algorithmic_flops_per_interval(model, K):
    """Per-interval FLOPs of the sparse forward method: K [8 nnz(J) c + 14 nx c + 4 phi_fJ].

    nnz(J) = 2 n_q + 2 n_b + 4 n_j + 4 n_c (flat ground), c = n + 2m + 1 tangent
    columns, phi_fJ = per-stage right-hand side + Jacobian cost (0.3k hopper,
    0.7k biped5, 1k cheetah7, 2k quad13).
    """
    nb, nj, nc = model.nb, model.nj, model.nc
    nnz = 2 * 3 * nb + 2 * nb + 4 * nj + 4 * nc
    c = model.n + 2 * model.m + 1
    phi = PHI_FJ.get(nb, 1000)
    return K * (8 * nnz * c + 14 * model.nx * c + 4 * phi)


def split_flops_per_interval(model, K):
    """(coefficient-record launch, tangent launch) shares of the forward
    FLOPs of one interval in the split form: the tangent launch integrates the
    c - 1 columns of Phi_x, B-, B+ (K [8 nnz(J) + 14 nx] (c - 1)); the record
    launch the right-hand side and Jacobian (4 K phi_fJ) and the dilation
    column S (K [8 nnz(J) + 14 nx])."""
    total = algorithmic_flops_per_interval(model, K)
    nb, nj, nc = model.nb, model.nj, model.nc
    nnz = 2 * 3 * nb + 2 * nb + 4 * nj + 4 * nc
    c = model.n + 2 * model.m + 1
    tangent = K * (8 * nnz + 14 * model.nx) * (c - 1)
    return total - tangent, tangent


def rkf_flops_per_interval(model, K):
    """Per-interval FLOPs of the Runge-Kutta-Fehlberg form (K steps of the 4(5)
    pair): K [10 nnz(J) c + 28 nx c + 6 phi_fJ] -- five propagated stages of
    the tangent product, 14 FMAs per tangent element and step for the stage
    inputs and the solution (partial sums), six right-hand side and Jacobian
    evaluations per step (the sixth for the estimate)."""
    nb, nj, nc = model.nb, model.nj, model.nc
    nnz = 2 * 3 * nb + 2 * nb + 4 * nj + 4 * nc
    c = model.n + 2 * model.m + 1
    phi = PHI_FJ.get(nb, 1000)
    return K * (10 * nnz * c + 28 * model.nx * c + 6 * phi)


def paper_flops_per_interval(model, K):
    """Per-interval FLOPs of the paper-faithful dynamics variant:
    4K [c (2 n_q 2 n_j + 2 nnz(J) + 14 nx) + 2 (2 n_j)^2 (2 n_j + n_q + 1)] with
    c = 6 n_b + 2 m + 1 tangent columns (m = n_j + 3 n_c, nx = 6 n_b + 4 n_c + 1):
    per stage and column the dense joint coupling Wm b, the sparse local terms
    and the RK4 combination; per stage the Gauss-Jordan elimination of
    [A | grad h M^-1 | r]."""
    nb, nj, nc = model.nb, model.nj, model.nc
    nq = 3 * nb
    nnz = 2 * nq + 2 * nb + 4 * nj + 4 * nc
    nx = 6 * nb + 4 * nc + 1
    c = 6 * nb + 2 * (nj + 3 * nc) + 1
    return 4 * K * (c * (2 * nq * 2 * nj + 2 * nnz + 14 * nx)
                    + 2 * (2 * nj) ** 2 * (2 * nj + nq + 1))


def adjoint_flops_per_interval(model, K):
    """Per-interval FLOPs of one gradient step (defects pass + reverse sweep):
    K [6 phi_fJ + 8 (nnz(J) + nnz(J_u, J_ubar) + nnz(J_p)) + 14 nx] + 2 K phi_fJ.

    The reverse sweep re-evaluates the right-hand side and Jacobian at every
    stage (4 phi_fJ per substep), recomputes the stage states from the
    checkpoints (4 phi_f ~ 2 phi_fJ), applies the transposed products (four
    stages, one FMA per nonzero of J, of the control Jacobians J_u (10 n_j +
    9 n_c) and J_ubar (3 n_c), and of J_p (3 n_b + n_c)) and the RK4 adjoint
    combination (14 nx); the defects pass is the nominal RK4 (2 K phi_fJ).
    """
    nb, nj, nc = model.nb, model.nj, model.nc
    nnz = 2 * 3 * nb + 2 * nb + 4 * nj + 4 * nc
    nnz_u = 10 * nj + 12 * nc
    nnz_p = 3 * nb + nc
    phi = PHI_FJ.get(nb, 1000)
    return K * (6 * phi + 8 * (nnz + nnz_u + nnz_p) + 14 * model.nx) + 2 * K * phi


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter record, or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2604_09993_amd.profiling import kernel_sources_sha256
    if rec.get("sources_sha256") != kernel_sources_sha256():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return {"fetch_bytes": k["fetch_bytes"], "write_bytes": k["write_bytes"],
            "total_bytes": k["fetch_bytes"] + k["write_bytes"],
            "algorithmic_bytes": k.get("algorithmic_bytes"), "source": "profiles/hbm_traffic.json"}


def upload_batch(api, batch, dev, dtype):
    import torch
    cms, trajs = {}, []
    for model, data, K in batch:
        cm = cms.get(id(model)) or cms.setdefault(id(model), api.CisModel(model))
        N = data["s"].shape[0]
        trajs.append(dict(cm=cm, K=K, X=api.to_device_soa(data["X"], dev, dtype, ld=N + 1),
                          U=api.to_device_soa(data["U"], dev, dtype, ld=N + 1),
                          s=torch.tensor(data["s"], device=dev, dtype=dtype),
                          params=torch.tensor(data["p"], device=dev, dtype=dtype)))
    return trajs


def batch_kernel_name(model, group, dtype):
    """rocprofv3 short name of a batch group's discretize kernel (the tangent
    launch for the split form)."""
    t = "double" if dtype == "f64" else "float"
    topo = f"Topo<{model.legs}, {model.depth}, 6, 1, false>"
    if group.get("split"):
        return f"k_tangent_batch<{t}, {topo}, {group['waves_per_simd']}>"
    pers = "true" if group["persist_blocks"] > 0 else "false"
    return f"k_discretize_batch<{t}, {topo}, {pers}, {group['waves_per_simd']}>"


def coefrec_kernel_name(model, dtype):
    t = "double" if dtype == "f64" else "float"
    return f"k_coefrec_batch<{t}, Topo<{model.legs}, {model.depth}, 6, 1, false>>"


def host_cpu():
    """CPU model, logical CPUs, CPUs this process may run on, and the cgroup quota."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()[:2]
            if q != "max":
                quota = float(q) / float(per)
    except (OSError, ValueError):
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    usable = affinity if quota is None else max(1, min(affinity, int(quota)))
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity_cpus": affinity,
            "cgroup_cpu_quota": quota, "usable_cpus": usable}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the headline workload only (profiling runs)")
    ap.add_argument("--extra-steps", type=int, default=20)
    ap.add_argument("--scp-max-iter", type=int, default=1500,
                    help="iteration cap of the end-to-end SCP run on the monoped")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs every kernel on a single GPU "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2604_09993_amd import _lib, api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = _lib.load(build_if_missing=False)
    stream = torch.cuda.current_stream()

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def timed(launch, steps, warmup):
        """Average ms per step over `steps` launches on `stream`, bracketed by HIP
        events recorded on that stream (after `warmup` untimed launches)."""
        for _ in range(warmup):
            launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            launch()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / steps, wall

    # Parity of the timed outputs: sampled GPU outputs are copied to the host
    # here and compared with the oracle in the CPU-baseline leg at the end
    # (the only part of this script that runs the oracle).
    parity, pending = {}, []
    sys.path.insert(0, os.path.join(ROOT, "tests"))

    def check_intervals(key, batch, plan, windows, fp32):
        """Queue an oracle check of contiguous windows of intervals."""
        if args.no_cpu_baseline:
            return
        got_all = []
        for t, k0, n in windows:
            sl = slice(k0, k0 + n)
            got = api.as_interval_major({k: v[..., sl] for k, v in plan.out[t].items()
                                         if k in ("A", "Bm", "Bp", "S", "d", "xprop")})
            got_all.append({k: v.double().cpu().numpy() for k, v in got.items()})

        def run():
            import oracle
            from parity import PHI32, PHI64, block_err
            r = (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)) if fp32 else \
                (lambda a: np.asarray(a, dtype=np.float64))
            worst = 0.0
            for (t, k0, n), got in zip(windows, got_all):
                model, data, K = batch[t]
                ref = oracle.discretize(model, r(data["X"][k0:k0 + n + 1]),
                                        r(data["U"][k0:k0 + n + 1]), r(data["s"][k0:k0 + n]),
                                        r(data["p"]), K)
                for k in ("A", "Bm", "Bp", "S", "d", "xprop"):
                    if model.m == 0 and k in ("Bm", "Bp"):
                        continue
                    worst = max(worst, block_err(got[k], ref[k], PHI32 if fp32 else PHI64))
            parity[key] = {"max_rel_err_vs_oracle": worst,
                           "metric": "normwise" if fp32 else "per-entry (phi = 1e-3)",
                           "bar": 1e-4 if fp32 else 1e-10,
                           "sample": "; ".join(f"trajectory {t} intervals {k0}..{k0 + n - 1}"
                                               for t, k0, n in windows)}
        pending.append(run)

    def check_adjoint(key, batch, plan, lams, picks):
        """Queue an oracle check of the gradients of whole trajectories."""
        if args.no_cpu_baseline:
            return
        got_all = []
        for t in picks:
            model, data, K = batch[t]
            N = data["s"].shape[0]
            o = plan.out[t]
            got_all.append((o["gX"][:, :N + 1].cpu().numpy().T, o["gs"].cpu().numpy(),
                            o["gp"].cpu().numpy(), o["gU"][:model.m, :N + 1].cpu().numpy().T))

        def run():
            import oracle
            from parity import PHI64, block_err
            worst = 0.0
            for t, (gX, gs, gp, gU) in zip(picks, got_all):
                model, data, K = batch[t]
                ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K,
                                     lams[t])
                pairs = [(gX, ref["gX"]), (gs.reshape(1, -1), ref["gs"].reshape(1, -1)),
                         (gp.reshape(1, -1), ref["gp"].reshape(1, -1))]
                if model.m:
                    pairs.append((gU, ref["gU"]))
                for g, r in pairs:
                    worst = max(worst, block_err(g, r, PHI64))
            parity[key] = {"max_rel_err_vs_oracle": worst, "metric": "per-entry (phi = 1e-3)",
                           "bar": 1e-10,
                           "sample": f"whole trajectories {picks} (gX, gU, gs, gp)"}
        pending.append(run)

    def merit_seeds(plan, cms):
        """Seeds of the merit 1/2 sum ||d_k||^2 + sum of integral increments:
        dJ/dF~_k = d_k + [0; 1] (from the plan's own defects pass)."""
        lams = []
        for o, cm in zip(plan.out, cms):
            sd = o["d"].clone()
            sd[cm.n:] += 1.0
            o["seed"].copy_(sd)
            lams.append(sd.cpu().numpy().T.copy())
        return lams

    # ---------------- headline: quad13 x 64, FP64 forward ----------------
    qb = synth.workload_batch("quad13_N200_K20_x64")
    qmodel = qb[0][0]
    q_int = sum(d["s"].shape[0] for _, d, _ in qb)
    q_flops = sum(algorithmic_flops_per_interval(m, k) * d["s"].shape[0] for m, d, k in qb)
    q_adj_flops = sum(adjoint_flops_per_interval(m, k) * d["s"].shape[0] for m, d, k in qb)
    trajs = upload_batch(api, qb, dev, torch.float64)
    plan64 = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=True,
                           stream=stream)
    g64 = plan64.groups()[0]
    ms_q64, wall_q64 = timed(lambda: plan64.run("discretize", graph=True, stream=stream),
                             args.steps, args.warmup)
    progress(f"quad13 x64 fp64 discretize {ms_q64:.3f} ms/step ({g64})")
    # the launches of the step one by one (HIP events on the launch stream)
    ms_part0, _ = timed(lambda: plan64.run_part("discretize", 0, stream=stream),
                        max(args.steps // 5, 3), 1)
    ms_part1 = None
    if g64.get("split"):
        ms_part1, _ = timed(lambda: plan64.run_part("discretize", 1, stream=stream),
                            max(args.steps // 5, 3), 1)
    progress(f"  launches: {ms_part0:.3f} ms" + (f" + {ms_part1:.3f} ms" if ms_part1 else ""))
    check_intervals("quad13x64_f64_discretize", qb, plan64, [(0, 0, 8), (37, 192, 8)], False)
    # gradient step of the same batch (merit seeds from its own defects pass)
    plan64.run("adjoint", graph=True, stream=stream)
    torch.cuda.synchronize()
    lams = merit_seeds(plan64, [t["cm"] for t in trajs])
    ms_qadj, _ = timed(lambda: plan64.run("adjoint", graph=True, stream=stream),
                       max(args.steps // 2, 5), args.warmup)
    progress(f"quad13 x64 fp64 gradient step {ms_qadj:.3f} ms/step")
    check_adjoint("quad13x64_f64_adjoint", qb, plan64, lams, [0, 21, 42, 63])
    plan64.close()
    del plan64, trajs
    torch.cuda.empty_cache()

    kname = batch_kernel_name(qmodel, g64, "f64")
    if g64.get("split"):
        # dominant kernel: the tangent launch, timed alone
        rec_fl = sum(split_flops_per_interval(m, k)[0] * d["s"].shape[0] for m, d, k in qb)
        tan_fl = q_flops - rec_fl
        achieved = tan_fl / (ms_part1 * 1e-3)
        kflops, kms = tan_fl, ms_part1
    else:
        achieved = q_flops / (ms_part0 * 1e-3)
        kflops, kms = q_flops, ms_part0
    line = {
        "metric": "discretized intervals/s (x+STM+B±) at 1e-10 rel vs oracle",
        "value": q_int / (ms_q64 * 1e-3),
        "unit": "intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_q64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "quad13 x 64: 64 trajectories of a planar 13-body chain "
                               "(torso + four 3-link legs, 12 joints, 4 contacts), N=200 "
                               "intervals each, K=20 RK4 substeps, FP64 forward, one batch "
                               "plan replayed as a HIP graph",
                   "trajectories": len(qb), "intervals": q_int, "N": 200, "substeps": 20,
                   "nx": qmodel.nx, "m": qmodel.m, "launch": g64},
        "roofline": {"bound": "alu", "kernel": kname,
                     "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "traffic": committed_traffic(kname),
                     "algorithmic_flop_per_launch": kflops, "ms_per_launch": kms,
                     "timing": "HIP events on the launch stream around launches of this "
                               "kernel alone (cis_batch_run_part)",
                     "step": {"achieved": q_flops / (ms_q64 * 1e-3) / 1e12,
                              "frac": q_flops / (ms_q64 * 1e-3) / PEAK_FP64_VALU,
                              "algorithmic_flop_per_step": q_flops,
                              "kernels": ([coefrec_kernel_name(qmodel, "f64"), kname]
                                          if g64.get("split") else [kname]),
                              "ms_per_launch": ([ms_part0, ms_part1] if g64.get("split")
                                                else [ms_part0])}},
        "gradient_step": {"value": q_int / (ms_qadj * 1e-3), "unit": "interval grads/s",
                          "ms_per_step": ms_qadj,
                          "roofline_frac": q_adj_flops / (ms_qadj * 1e-3) / PEAK_FP64_VALU,
                          "algorithmic_flop_per_step": q_adj_flops,
                          "step": "defects with checkpoints + reverse sweep + reduction, "
                                  "graph replay; merit 1/2 sum ||d||^2 + integral increments"},
        "wall_s_timed_region": wall_q64,
    }

    extras = {}
    if not args.no_extras:
        # FP32 forward of the same batch
        trajs = upload_batch(api, qb, dev, torch.float32)
        plan32 = api.BatchPlan(trajs, ("discretize",), sched="tune", graph=True, stream=stream)
        g32 = plan32.groups()[0]
        ms_q32, _ = timed(lambda: plan32.run("discretize", graph=True, stream=stream),
                          args.extra_steps, 2)
        progress(f"quad13 x64 fp32 discretize {ms_q32:.3f} ms/step")
        check_intervals("quad13x64_f32_discretize", qb, plan32, [(0, 0, 8), (37, 192, 8)], True)
        extras["quad13x64_f32"] = {"value": q_int / (ms_q32 * 1e-3), "unit": "intervals/s",
                                   "ms_per_step": ms_q32, "launch": g32,
                                   "kernel": batch_kernel_name(qmodel, g32, "f32"),
                                   "roofline_frac": q_flops / (ms_q32 * 1e-3) / PEAK_FP32_VALU}
        plan32.close()
        del plan32, trajs
        torch.cuda.empty_cache()

        # node-level impact map over every node of the headline batch (64 x 201
        # nodes, one launch): G~, Theta, Psi and the compact Jacobians
        from paper_2604_09993_amd.profiling import impact_bytes
        imodel, idata = synth.impact_workload("quad13_x64")
        icm = api.CisModel(imodel)
        soa = lambda a: torch.from_numpy(np.ascontiguousarray(a.T)).to(dev)
        iin = [soa(idata[k]) for k in ("Xp", "Xm", "Phi", "Gamma")]
        ip = torch.tensor(idata["p"], device=dev)
        n_nodes = iin[0].shape[1]
        iout = api.impact_linearize(icm, *iin, ip, 1e-2, 1e-4, stream=stream)
        iargv = ([icm.handle, n_nodes, iin[0].stride(0)]
                 + [ctypes.c_void_p(t.data_ptr()) for t in iin + [ip]] + [1e-2, 1e-4]
                 + [ctypes.c_void_p(iout[k].data_ptr()) for k in ("G", "Theta", "JGv", "JTc", "Psi")]
                 + [ctypes.c_void_p(stream.cuda_stream)])

        def launch_impact():
            st = lib.cis_impact_linearize(*iargv)
            if st != 0:
                _lib.check(st)
        ms_imp, _ = timed(launch_impact, 5 * args.extra_steps, 5)
        ibytes = n_nodes * impact_bytes(imodel)
        iname = f"k_impact<ImpTopo<{imodel.legs}, {imodel.depth}>>"
        progress(f"impact map quad13 {n_nodes} nodes {ms_imp * 1e3:.1f} us/launch")
        extras["impact_quad13x64_f64"] = {
            "value": n_nodes / (ms_imp * 1e-3), "unit": "nodes/s", "ms_per_launch": ms_imp,
            "nodes": n_nodes, "kernel": iname,
            "roofline": {"bound": "hbm", "achieved": ibytes / (ms_imp * 1e-3) / 1e9,
                         "peak": 8000.0, "unit": "GB/s",
                         "frac": ibytes / (ms_imp * 1e-3) / 8e12,
                         "traffic": committed_traffic(iname),
                         "algorithmic_bytes_per_launch": ibytes},
            "timing": "HIP events on the launch stream around cis_impact_linearize calls"}
        if not args.no_cpu_baseline:
            picks = [0, 5000, n_nodes - 1]
            got_i = {k: iout[k][picks].cpu().numpy() for k in ("G", "Theta", "JGv", "JTc")}

            def run_impact():
                from oracle import impact as oimp
                from parity import PHI64, block_err
                import impact_layout
                lin = oimp.linearize(imodel, idata["Xp"][picks], idata["Xm"][picks],
                                     idata["Phi"][picks], idata["Gamma"][picks], idata["p"], 1e-2)
                JGv, JTc = impact_layout.compact_from_dense(imodel, lin["JG"], lin["JT"])
                ref = dict(G=lin["G"], Theta=lin["Theta"], JGv=JGv, JTc=JTc)
                worst = max(block_err(got_i[k], ref[k], PHI64) for k in ref)
                parity["impact_quad13x64_f64"] = {
                    "max_rel_err_vs_oracle": worst, "metric": "per-entry (phi = 1e-3)",
                    "bar": 1e-10, "sample": f"nodes {picks} (G, Theta, JGv, JTc)"}
            pending.append(run_impact)
        del iin, iout
        torch.cuda.empty_cache()

        # Runge-Kutta-Fehlberg form: the 12800 quad13 intervals of the batch as
        # one trajectory (cis_discretize_rkf), beside the RK4 split form on the
        # same intervals (cis_discretize_split)
        rmodel, rdata, rK = synth.make_workload("quad13_N12800_K20")
        rN = rdata["s"].shape[0]
        rcm = api.CisModel(rmodel)
        rX = api.to_device_soa(rdata["X"], dev)
        rU = api.to_device_soa(rdata["U"], dev)
        rs = torch.tensor(rdata["s"], device=dev)
        rp = torch.tensor(rdata["p"], device=dev)
        rout = api.discretize_rkf(rcm, rX, rU, rs, rp, rK, stream=stream)
        rws = torch.empty((api.rkf_workspace_bytes(rcm, rN, rK),), device=dev, dtype=torch.uint8)
        rsh = _lib.Shape(rN, rK, _lib.CIS_F64, 0, rX.stride(0), rN)
        vpr = lambda t: ctypes.c_void_p(None if t is None else t.data_ptr())
        rargs = [vpr(t) for t in (rX, rU, rs, rp)]
        routs = [vpr(rout[k]) for k in ("A", "Bm", "Bp", "S", "d", "xprop")]
        st_r = ctypes.c_void_p(stream.cuda_stream)

        def launch_rkf(waves=1):
            _lib.check(lib.cis_discretize_rkf(rcm.handle, ctypes.byref(rsh), *rargs, waves,
                                              *routs, vpr(rout["err"]), vpr(rws), rws.numel(),
                                              st_r))

        def launch_rk4_split():   # the register budget the batch tuner picks for quad13
            _lib.check(lib.cis_discretize_split(rcm.handle, ctypes.byref(rsh), *rargs, 2, *routs,
                                                vpr(rws), rws.numel(), st_r))
        # both register budgets of the tangent launch; the faster is reported
        rkf_by_waves = {w: timed(lambda: launch_rkf(w), args.extra_steps, 2)[0] for w in (1, 2)}
        rkf_w = min(rkf_by_waves, key=rkf_by_waves.get)
        ms_rkf = rkf_by_waves[rkf_w]
        ms_rk4s, _ = timed(launch_rk4_split, args.extra_steps, 2)
        launch_rkf(rkf_w)
        torch.cuda.synchronize()
        rkf_fl = rkf_flops_per_interval(rmodel, rK) * rN
        progress(f"rkf quad13 N={rN} K={rK}: {ms_rkf:.3f} ms (rk4 split {ms_rk4s:.3f} ms)")
        extras["rkf_quad13_N12800_K20_f64"] = {
            "value": rN / (ms_rkf * 1e-3), "unit": "intervals/s", "ms_per_step": ms_rkf,
            "rk4_split_ms_same_intervals": ms_rk4s,
            "tangent_waves_per_simd": {"rkf": rkf_w, "rk4_split": 2},
            "rkf_ms_by_tangent_waves": {str(w): v for w, v in rkf_by_waves.items()},
            "roofline": {"bound": "alu", "achieved": rkf_fl / (ms_rkf * 1e-3) / 1e12,
                         "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": rkf_fl / (ms_rkf * 1e-3) / PEAK_FP64_VALU,
                         "algorithmic_flop_per_step": rkf_fl,
                         "traffic": {"records": committed_traffic(
                                         f"k_rkf_rec<double, Topo<{rmodel.legs}, {rmodel.depth}, 6, 1, false>>"),
                                     "tangent": committed_traffic(
                                         f"k_rkf_tan<double, Topo<{rmodel.legs}, {rmodel.depth}, 6, 1, false>, {rkf_w}>")}},
            "step": "cis_discretize_rkf: Fehlberg 4(5), K=20 steps, records + tangent launches"}
        if not args.no_cpu_baseline:
            rks = [0, 6400, rN - 1]
            got_r = {k: api.as_interval_major({k: rout[k]})[k][rks].double().cpu().numpy()
                     for k in ("A", "Bm", "Bp", "S", "d", "xprop")}

            def run_rkf():
                import oracle
                from parity import PHI64, block_err
                worst = 0.0
                for i, kk in enumerate(rks):
                    ref = oracle.discretize_rkf(rmodel, rdata["X"][kk:kk + 2], rdata["U"][kk:kk + 2],
                                                rdata["s"][kk:kk + 1], rdata["p"], rK)
                    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
                        worst = max(worst, block_err(got_r[key][i:i + 1], ref[key], PHI64))
                parity["rkf_quad13_N12800_K20_f64"] = {
                    "max_rel_err_vs_oracle": worst, "metric": "per-entry (phi = 1e-3)",
                    "bar": 1e-10, "sample": f"intervals {rks}"}
            pending.append(run_rkf)
        del rout, rws, rX, rU
        torch.cuda.empty_cache()

        # paper-faithful dynamics variant (joint forces eliminated): 12800
        # quad13 intervals as one trajectory, K = 20
        pmodel = rmodel
        prng = np.random.default_rng(8)
        pdata = synth.gen_paper_nodes(pmodel, rN, prng, T=64.0)
        pcm = api.CisModel(pmodel)
        pX = api.to_device_soa(pdata["X"], dev)
        pU = api.to_device_soa(pdata["U"], dev)
        ps = torch.tensor(pdata["s"], device=dev)
        pp = torch.tensor(pdata["p"], device=dev)
        pout = api.discretize_paper(pcm, pX, pU, ps, pp, rK, stream=stream)
        psh = _lib.Shape(rN, rK, _lib.CIS_F64, 0, pX.stride(0), rN)
        pnb = ctypes.c_size_t()
        _lib.check(lib.cis_paper_workspace_size(pcm.handle, ctypes.byref(psh), ctypes.byref(pnb)))
        pws = torch.empty((pnb.value,), device=dev, dtype=torch.uint8)
        pargs = [vpr(t) for t in (pX, pU, ps, pp)]
        pouts = [vpr(pout[k]) for k in ("A", "Bm", "Bp", "S", "d", "xprop")]

        def launch_paper():
            _lib.check(lib.cis_discretize_paper(pcm.handle, ctypes.byref(psh), *pargs, *pouts,
                                                vpr(pws), pws.numel(), st_r))
        ms_pap, _ = timed(launch_paper, max(args.extra_steps // 4, 3), 1)
        pap_fl = paper_flops_per_interval(pmodel, rK) * rN
        progress(f"paper dynamics quad13 N={rN} K={rK}: {ms_pap:.3f} ms")
        extras["paper_dynamics_quad13_N12800_K20_f64"] = {
            "value": rN / (ms_pap * 1e-3), "unit": "intervals/s", "ms_per_step": ms_pap,
            "roofline": {"bound": "alu", "achieved": pap_fl / (ms_pap * 1e-3) / 1e12,
                         "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": pap_fl / (ms_pap * 1e-3) / PEAK_FP64_VALU,
                         "algorithmic_flop_per_step": pap_fl,
                         "traffic": {"records": committed_traffic(
                                         f"k_paper_rec<PTopo<{rmodel.legs}, {rmodel.depth}>>"),
                                     "tangent": committed_traffic(
                                         f"k_paper_tan<PTopo<{rmodel.legs}, {rmodel.depth}>>")}},
            "step": "cis_discretize_paper: joint forces eliminated, RK4 K=20, record + tangent "
                    "launches"}
        if not args.no_cpu_baseline:
            pks = [0, rN - 1]
            got_p = {k: api.as_interval_major({k: pout[k]})[k][pks].cpu().numpy()
                     for k in ("A", "Bm", "Bp", "S", "d", "xprop")}

            def run_paper():
                from oracle import paper_dynamics as pdyn
                from parity import PHI64, block_err
                worst = 0.0
                for i, kk in enumerate(pks):
                    ref = pdyn.discretize(pmodel, pdata["X"][kk:kk + 2], pdata["U"][kk:kk + 2],
                                          pdata["s"][kk:kk + 1], pdata["p"], rK)
                    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
                        worst = max(worst, block_err(got_p[key][i:i + 1], ref[key], PHI64))
                parity["paper_dynamics_quad13_N12800_K20_f64"] = {
                    "max_rel_err_vs_oracle": worst, "metric": "per-entry (phi = 1e-3)",
                    "bar": 1e-10, "sample": f"intervals {pks}"}
            pending.append(run_paper)
        del pout, pws, pX, pU
        torch.cuda.empty_cache()

        # uneven batch of 256 trajectories over three models
        mb = synth.mixed_batch()
        m_int = sum(d["s"].shape[0] for _, d, _ in mb)
        m_flops = sum(algorithmic_flops_per_interval(m, k) * d["s"].shape[0] for m, d, k in mb)
        m_adj = sum(adjoint_flops_per_interval(m, k) * d["s"].shape[0] for m, d, k in mb)
        trajs = upload_batch(api, mb, dev, torch.float64)
        planm = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=True,
                              stream=stream)
        ms_m, _ = timed(lambda: planm.run("discretize", graph=True, stream=stream),
                        args.extra_steps, 2)
        first = {}
        for i, (m_, _, _) in enumerate(mb):
            first.setdefault(id(m_), i)
        check_intervals("mixed256_f64_discretize", mb, planm,
                        [(i, 0, 6) for i in sorted(first.values())], False)
        planm.run("adjoint", graph=True, stream=stream)
        torch.cuda.synchronize()
        lams_m = merit_seeds(planm, [t["cm"] for t in trajs])
        ms_madj, _ = timed(lambda: planm.run("adjoint", graph=True, stream=stream),
                           args.extra_steps, 2)
        check_adjoint("mixed256_f64_adjoint", mb, planm, lams_m,
                      sorted(set(first.values()) | {5, 100, 200}))
        # each model's trajectories alone (same kernels, tuned the same way): the
        # mixed graph runs the groups concurrently, so its time against the
        # slowest group alone bounds what one launch switching on the model
        # could still gain by overlapping them
        alone = {}
        by_model = {}
        for i, (m_, _, _) in enumerate(mb):
            by_model.setdefault(m_.name, []).append(i)
        for name_, idx in by_model.items():
            pl = api.BatchPlan([trajs[i] for i in idx], ("discretize",), sched="tune", graph=True,
                               stream=stream)
            alone[name_], _ = timed(lambda: pl.run("discretize", graph=True, stream=stream),
                                    args.extra_steps, 2)
            pl.close()
        progress(f"mixed256 fp64 discretize {ms_m:.3f} ms, gradient step {ms_madj:.3f} ms; "
                 f"groups alone {alone}")
        extras["mixed256_f64"] = {
            "trajectories": len(mb), "intervals": m_int,
            "discretize": {"value": m_int / (ms_m * 1e-3), "unit": "intervals/s",
                           "ms_per_step": ms_m,
                           "roofline_frac": m_flops / (ms_m * 1e-3) / PEAK_FP64_VALU},
            "gradient_step": {"value": m_int / (ms_madj * 1e-3), "unit": "interval grads/s",
                              "ms_per_step": ms_madj,
                              "roofline_frac": m_adj / (ms_madj * 1e-3) / PEAK_FP64_VALU},
            "groups": planm.groups(),
            "groups_alone_ms": alone, "sum_alone_ms": sum(alone.values()),
            "max_alone_ms": max(alone.values())}
        planm.close()
        del planm, trajs
        torch.cuda.empty_cache()

        # single trajectories: cheetah7 N=50 K=20 (FP64, FP32, gradient), hopper N=20 K=10
        def single(name, dtype):
            model, data, K = synth.make_workload(name)
            N = data["s"].shape[0]
            cm = api.CisModel(model)
            X = api.to_device_soa(data["X"], dev, dtype)
            U = api.to_device_soa(data["U"], dev, dtype)
            s = torch.tensor(data["s"], device=dev, dtype=dtype)
            p = torch.tensor(data["p"], device=dev, dtype=dtype)
            kw = dict(device=dev, dtype=dtype)
            out = dict(A=torch.empty((cm.nx, cm.nx, N), **kw), Bm=torch.empty((cm.nx, cm.m, N), **kw),
                       Bp=torch.empty((cm.nx, cm.m, N), **kw), S=torch.empty((cm.nx, N), **kw),
                       d=torch.empty((cm.nx, N), **kw), xprop=torch.empty((cm.nx, N), **kw))
            api.discretize_into(cm, X, U, s, p, K, out)
            sh = _lib.Shape(N, K, api._dtype_code(dtype), 0, X.stride(0), N)
            argv = [cm.handle, ctypes.byref(sh)] + [ctypes.c_void_p(t.data_ptr()) for t in
                    (X, U, s, p, out["A"], out["Bm"], out["Bp"], out["S"], out["d"], out["xprop"])]
            argv.append(ctypes.c_void_p(stream.cuda_stream))

            def launch():
                st = lib.cis_discretize(*argv)
                if st != 0:
                    _lib.check(st)
            ms, _ = timed(launch, 200, 20)
            wrap = [(model, data, K)]
            fake = type("P", (), {"out": [out]})()
            check_intervals(f"{name}_{'f64' if dtype == torch.float64 else 'f32'}", wrap, fake,
                            [(0, 0, N)], dtype == torch.float32)
            # the tuner's pick among layouts and forms on these inputs (best of three)
            _, ch = api.single_tune(cm, X, U, s, p, K, stream=stream)
            tuned = {k: ch[k] for k in ("form", "layout", "waves", "blocks", "compose", "ms")}
            return dict(value=N / (ms * 1e-3), unit="intervals/s", ms_per_step=ms,
                        roofline_frac=algorithmic_flops_per_interval(model, K) * N / (ms * 1e-3) /
                        (PEAK_FP64_VALU if dtype == torch.float64 else PEAK_FP32_VALU),
                        tuned=tuned), (cm, X, U, s, p, N, K)

        extras["cheetah7_N50_K20_f64"], keep = single("cheetah7_N50_K20", torch.float64)
        extras["cheetah7_N50_K20_f32"], _ = single("cheetah7_N50_K20", torch.float32)
        extras["hopper_N20_K10_f64"], _ = single("hopper_N20_K10", torch.float64)
        cm, X, U, s, p, N, K = keep
        C = 5
        fw = api.defects(cm, X, U, s, p, K, ckpt_every=C)
        seed = fw["d"].clone()
        seed[cm.n:] += 1.0
        nbytes = api.adjoint_workspace_bytes(cm, N, K)
        ws = torch.empty((nbytes,), device=dev, dtype=torch.uint8)
        gX = torch.empty((cm.nx, N + 1), device=dev, dtype=torch.float64)
        gU = torch.empty((cm.m, N + 1), device=dev, dtype=torch.float64)
        gs = torch.empty((N,), device=dev, dtype=torch.float64)
        gp = torch.empty((cm.np,), device=dev, dtype=torch.float64)
        sh_adj = _lib.Shape(N, K, _lib.CIS_F64, 0, X.stride(0), N)
        vp = lambda t: ctypes.c_void_p(t.data_ptr())
        st_ptr = ctypes.c_void_p(stream.cuda_stream)

        def launch_grad():
            _lib.check(lib.cis_defects(cm.handle, ctypes.byref(sh_adj), vp(X), vp(U), vp(s), vp(p),
                                       vp(fw["d"]), vp(fw["xprop"]), vp(fw["ckpt"]), C, st_ptr))
            _lib.check(lib.cis_discretize_adjoint(cm.handle, ctypes.byref(sh_adj), vp(X), vp(U),
                                                  vp(s), vp(p), vp(fw["ckpt"]), C, vp(seed),
                                                  vp(gX), vp(gU), vp(gs), vp(gp), vp(ws), nbytes,
                                                  st_ptr))
        ms_g, _ = timed(launch_grad, 100, 20)
        cmodel = cm.model
        extras["cheetah7_N50_K20_gradient_step"] = {
            "value": N / (ms_g * 1e-3), "unit": "interval grads/s", "ms_per_step": ms_g,
            "roofline_frac": adjoint_flops_per_interval(cmodel, K) * N / (ms_g * 1e-3) /
            PEAK_FP64_VALU,
            "step": "cis_defects (checkpoints every 5 substeps) + cis_discretize_adjoint"}
        progress("single trajectories: " + ", ".join(
            f"{k} {v['ms_per_step']:.4f} ms" for k, v in extras.items() if k.startswith(("cheetah", "hopper"))))

        # substep blocking on one quad13 trajectory (N = 200): fused kernel
        # against B blocks chained by dense VALU or MFMA products
        model, data, K = qb[0]
        cmq = api.CisModel(model)
        Xq = api.to_device_soa(data["X"], dev)
        Uq = api.to_device_soa(data["U"], dev)
        sq = torch.tensor(data["s"], device=dev)
        pq = torch.tensor(data["p"], device=dev)
        blk = {}
        ms_f, _ = timed(lambda: api.discretize(cmq, Xq, Uq, sq, pq, K, stream=stream), 10, 2)
        blk["fused_ms"] = ms_f
        ms_s, _ = timed(lambda: api.discretize_split(cmq, Xq, Uq, sq, pq, K, stream=stream), 10, 2)
        blk["split_ms"] = ms_s
        for B in (2, 4, 5):
            nb_ = api.blocked_workspace_bytes(cmq, data["s"].shape[0], K, B)
            wsb = torch.empty((nb_,), device=dev, dtype=torch.uint8)
            for mode in ("valu", "mfma"):
                ms_b, _ = timed(lambda: api.discretize_blocked(cmq, Xq, Uq, sq, pq, K, B, mode,
                                                               ws=wsb, stream=stream), 10, 2)
                blk[f"B{B}_{mode}_ms"] = ms_b
        for lay in ("latency", "latency_s", "narrow", "throughput"):
            ms_l, _ = timed(lambda: api.discretize(cmq, Xq, Uq, sq, pq, K, layout=lay,
                                                   stream=stream), 10, 2)
            blk[f"layout_{lay}_ms"] = ms_l
        _, ch = api.single_tune(cmq, Xq, Uq, sq, pq, K, stream=stream)
        blk["tuned"] = {k: ch[k] for k in ("form", "layout", "waves", "blocks", "compose")}
        blk["tuned"]["candidates"] = ("one-launch layouts, split form with 1 and 2 waves, blocks "
                                      "2..8 dividing K with VALU and MFMA composition, timed on "
                                      "these inputs (cis_single_tune)")
        extras["quad13_N200_K20_single_blocking"] = blk
        progress("blocking: " + ", ".join(f"{k} {v:.3f}" for k, v in blk.items()
                                          if isinstance(v, float)) + f"; tuned {blk['tuned']}")

        # the SCP driver end to end on the monoped (hopper; the paper's grid of
        # 15 nodes, 10 integration steps per interval): GPU transcription, host
        # assembly and interior-point QP solve, delta-homotopy of Alg. 1
        from paper_2604_09993_amd import scp
        hmodel = synth.make_hopper(np.random.default_rng(0))
        hx0, hx1 = synth.standing_state(hmodel, 0.0), synth.standing_state(hmodel, 0.3)
        hpb = scp.CitoProblem(hmodel, 14, hx0, hx1, K=10)
        hg = synth.scp_initial_guess(hmodel, 14, hx0, hx1, 0.05, np.random.default_rng(1))
        hz0 = hpb.pack(hg["Xp"], hg["Xm"], hg["Phi"], hg["Gamma"], hg["Ua"], hg["Ub"], hg["S"])
        for integ, key in (("rk4", "scp_monoped_N14_K10"), ("rkf", "scp_monoped_N14_K10_rkf")):
            htr = scp.GpuTranscriber(hpb, integ)
            htr(hpb.unpack(hz0), 1.0)                   # warm-up transcription
            hdrv = scp.ScpDriver(hpb, htr)
            t_scp = time.perf_counter()
            hdrv.run(hz0, max_iter=args.scp_max_iter,
                     callback=lambda rec, z: rec.j % 100 == 99 and progress(
                         f"scp ({integ}) iteration {rec.j + 1}: delta {rec.delta:.3g}, "
                         f"J_px {rec.J_px:.2e}, J_ep {rec.J_ep:.2e}"))
            t_scp = time.perf_counter() - t_scp
            hh = hdrv.history
            ms_it = 1e3 * t_scp / len(hh)
            ex = {
                "value": len(hh) / t_scp, "unit": "SCP iterations/s", "ms_per_iteration": ms_it,
                "iterations": len(hh), "converged": bool(hdrv.hom.done()), "wall_s": t_scp,
                "integrator": {"rk4": "classical RK4", "rkf": "Fehlberg 4(5)"}[integ],
                "final": {"delta": hdrv.hom.delta[-1], "J_px": hh[-1].J_px, "J_ep": hh[-1].J_ep,
                          "cost": hh[-1].cost},
                "qp_status_counts": {st: sum(r.qp_status == st for r in hh)
                                     for st in sorted({r.qp_status for r in hh})},
                "transcribe_ms": 1e3 * float(np.mean([r.t_transcribe for r in hh])),
                "assemble_ms": 1e3 * float(np.mean([r.t_assemble for r in hh])),
                "qp_solve_ms": 1e3 * float(np.mean([r.t_solve for r in hh])),
                "qp_iterations_mean": float(np.mean([r.qp_iters for r in hh])),
                "step": "transcription (cis_discretize or cis_discretize_rkf over the "
                        "node-doubled discontinuous hold + cis_impact_linearize, host copies "
                        "included), subproblem assembly, QP solve, Alg. 1 update"}
            extras[key] = ex
            progress(f"scp monoped ({integ}): {len(hh)} iterations in {t_scp:.1f} s (converged "
                     f"{ex['converged']}), {ms_it:.1f} ms/iteration (transcribe "
                     f"{ex['transcribe_ms']:.2f}, assemble {ex['assemble_ms']:.2f}, solve "
                     f"{ex['qp_solve_ms']:.2f} ms)")
            if not args.no_cpu_baseline:
                got_h = htr(hpb.unpack(hz0), 0.5)

                def run_scp(got_h=got_h, integ=integ, key=key):
                    from parity import PHI64, block_err
                    from scp_oracle import oracle_transcriber
                    ref = oracle_transcriber(hpb, integ)(hpb.unpack(hz0), 0.5)
                    worst = max(block_err(got_h[k], ref[k], PHI64) for k in ref)
                    parity[key + "_transcription"] = {
                        "max_rel_err_vs_oracle": worst, "metric": "per-entry (phi = 1e-3)",
                        "bar": 1e-10, "sample": "initial iterate, every interval and node "
                        "(A, B-, B+, S, d, G~, Theta, Psi and their node Jacobians), delta = 0.5"}
                pending.append(run_scp)

    line["extras"] = extras

    bad = []
    if not args.no_cpu_baseline:
        for run in pending:
            run()
        line["parity"] = parity
        bad = [k for k, v in parity.items() if not v["max_rel_err_vs_oracle"] <= v["bar"]]
        line["parity_ok"] = not bad
        line["max_rel_err_vs_oracle"] = parity["quad13x64_f64_discretize"]["max_rel_err_vs_oracle"]
        progress(f"parity checked on {len(parity)} outputs; above the bar: {bad}")
        # CPU-baseline leg: the plain FP64 oracle on the host cores, on a bounded
        # sample of the headline workload (consecutive quad13 intervals, K = 20).
        import oracle
        cpu = host_cpu()
        nthr = cpu["usable_cpus"]
        # all usable threads: whole trajectories 1.. of the batch (5000 intervals
        # with 16 or more threads, about 10 s); one thread: one whole
        # trajectory (200 intervals, about 7 s)
        n_tr = max(1, min(25, (25 * nthr) // 16))
        n_all = 0
        t0 = time.perf_counter()
        for t in range(1, 1 + n_tr):
            model, data, K = qb[t]
            oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K,
                              nthreads=nthr)
            n_all += data["s"].shape[0]
        dt_all = time.perf_counter() - t0
        model, data, K = qb[1]
        n_one = 200   # one whole trajectory
        t0 = time.perf_counter()
        oracle.discretize(model, data["X"][:n_one + 1], data["U"][:n_one + 1], data["s"][:n_one],
                          data["p"], K, nthreads=1)
        dt_one = time.perf_counter() - t0
        progress(f"cpu baseline: {n_all} intervals on {nthr} threads in {dt_all:.1f} s, "
                 f"{n_one} on 1 thread in {dt_one:.1f} s")
        line["cpu_baseline"] = {
            "value": n_all / dt_all, "unit": "intervals/s", "cores": nthr, "kind": "oracle",
            "sample": f"{n_all} intervals ({n_tr} whole quad13 trajectories of the headline "
                      f"batch, K=20, FP64), OpenMP over intervals on {nthr} threads, "
                      f"{dt_all:.1f} s",
            "one_thread": {"value": n_one / dt_one, "unit": "intervals/s", "cores": 1,
                           "sample": f"{n_one} intervals on 1 thread, {dt_one:.1f} s"},
            "host": cpu}
    print(json.dumps(line), flush=True)
    if bad:
        print(f"bench.py: parity above the bar for {bad}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
