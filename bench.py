#!/usr/bin/env python3
"""Discretized intervals/s of the CI-SCvx linearize-and-discretize step on one MI355X.

Workload: HalfCheetah-shaped planar chain (7 bodies, 6 joints, 2 contacts;
nx = 45, m = 24), N = 50 intervals, K = 20 RK4 substeps, FP64, synthetic
seeded node data (inputs resident in HBM before timing).  One step = one call
of cis_discretize over all 50 intervals (A, B-, B+, S, defects, F~).

Prints one JSON line.  Extra fields: the FP32 form of the same step, the
adjoint gradient step, batched multiple shooting (256 mixed trajectories;
64 quad13 trajectories of N = 200), the parity error of the timed output
against the CPU oracle, the roofline of the dominant kernel (k_discretize)
and the CPU oracle baseline.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12   # MI355X FP64 vector FLOP/s (AMD published)
PEAK_FP32_VALU = 157.3e12


def algorithmic_flops_per_interval(model, K):
    """Per-interval FLOPs of the sparse method: K [8 nnz(J) c + 14 nx c + 4 phi_fJ].

    nnz(J) = 2 n_q + 2 n_b + 4 n_j + 4 n_c (flat ground), c = n + 2m + 1 tangent
    columns, phi_fJ = per-stage right-hand side + Jacobian cost (0.3k hopper,
    0.7k biped5, 1k cheetah7, 2k quad13).
    """
    nb, nj, nc = model.nb, model.nj, model.nc
    nnz = 2 * 3 * nb + 2 * nb + 4 * nj + 4 * nc
    c = model.n + 2 * model.m + 1
    phi = {2: 300, 5: 700, 7: 1000, 13: 2000}.get(nb, 1000)
    return K * (8 * nnz * c + 14 * model.nx * c + 4 * phi)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workloads")
    ap.add_argument("--batch-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus must be 1 (the kernels run on a single GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2604_09993_amd import _lib, api, synth

    model, data, K = synth.make_workload("cheetah7_N50_K20")
    N = data["s"].shape[0]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cm = api.CisModel(model)
    lib = _lib.load(build_if_missing=False)

    def prepare(dtype):
        X = api.to_device_soa(data["X"], dev, dtype)
        U = api.to_device_soa(data["U"], dev, dtype)
        s = torch.tensor(data["s"], device=dev, dtype=dtype)
        p = torch.tensor(data["p"], device=dev, dtype=dtype)
        kw = dict(device=dev, dtype=dtype)
        nx, m = cm.nx, cm.m
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw), xprop=torch.empty((nx, N), **kw))
        api.discretize_into(cm, X, U, s, p, K, out)   # validates shapes once
        stream = torch.cuda.current_stream()
        sh = _lib.Shape(N, K, api._dtype_code(dtype), 0, X.stride(0), N)
        argv = [cm.handle, ctypes.byref(sh)] + [ctypes.c_void_p(t.data_ptr()) for t in
                (X, U, s, p, out["A"], out["Bm"], out["Bp"], out["S"], out["d"], out["xprop"])]
        argv.append(ctypes.c_void_p(stream.cuda_stream))
        fn = lib.cis_discretize

        def launch():
            st = fn(*argv)
            if st != 0:
                _lib.check(st)
        keep = (X, U, s, p, sh)
        return launch, out, stream, keep

    def timed(launch, stream, steps, warmup):
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

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    launch64, out64, stream, keep64 = prepare(torch.float64)
    ms64, wall64 = timed(launch64, stream, args.steps, args.warmup)
    progress(f"fp64 discretize {ms64:.4f} ms/step")
    launch32, out32, _, keep32 = prepare(torch.float32)
    ms32, _ = timed(launch32, stream, args.steps, args.warmup)
    progress(f"fp32 discretize {ms32:.4f} ms/step")

    # adjoint form on the same workload (checkpoints every 5 substeps): one
    # gradient step = forward defects with checkpoints + reverse sweep + reduce
    C = 5
    X64, U64, s64, p64 = keep64[:4]
    fw = api.defects(cm, X64, U64, s64, p64, K, ckpt_every=C)
    seed = fw["d"].clone()
    seed[cm.n:] += 1.0          # d(1/2 ||d||^2 + sum of integral increments)/dF~
    nbytes = api.adjoint_workspace_bytes(cm, N, K)
    ws = torch.empty((nbytes,), device=dev, dtype=torch.uint8)
    gX = torch.empty((cm.nx, N + 1), device=dev, dtype=torch.float64)
    gU = torch.empty((cm.m, N + 1), device=dev, dtype=torch.float64)
    gs = torch.empty((N,), device=dev, dtype=torch.float64)
    gp = torch.empty((cm.np,), device=dev, dtype=torch.float64)
    sh_adj = _lib.Shape(N, K, _lib.CIS_F64, 0, X64.stride(0), N)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    d_fw, xp_fw, ck = fw["d"], fw["xprop"], fw["ckpt"]
    st_ptr = ctypes.c_void_p(stream.cuda_stream)

    def launch_grad():
        _lib.check(lib.cis_defects(cm.handle, ctypes.byref(sh_adj), vp(X64), vp(U64), vp(s64), vp(p64),
                                   vp(d_fw), vp(xp_fw), vp(ck), C, st_ptr))
        _lib.check(lib.cis_discretize_adjoint(cm.handle, ctypes.byref(sh_adj), vp(X64), vp(U64),
                                              vp(s64), vp(p64), vp(ck), C, vp(seed), vp(gX),
                                              vp(gU), vp(gs), vp(gp), vp(ws), nbytes, st_ptr))
    ms_grad, _ = timed(launch_grad, stream, max(args.steps // 2, 10), args.warmup)
    progress(f"gradient step {ms_grad:.4f} ms")

    flops = algorithmic_flops_per_interval(model, K) * N
    achieved = flops / (ms64 * 1e-3)
    kname = "k_discretize<double, Topo<2, 3, 1, 2, true>>"

    batch = {}
    if not args.no_batch:
        # multiple shooting over many trajectories: one plan per workload,
        # replayed as a HIP graph (one kernel per model, run concurrently)
        for name, make, ops, dtypes in (
                ("mixed256", lambda: synth.mixed_batch(), ("discretize", "adjoint"),
                 (torch.float64,)),
                ("quad13x64", lambda: synth.workload_batch("quad13_N200_K20_x64"), ("discretize",),
                 (torch.float64, torch.float32))):
            bl = make()
            nint = sum(d["s"].shape[0] for _, d, _ in bl)
            bflops = sum(algorithmic_flops_per_interval(m, k) * d["s"].shape[0] for m, d, k in bl)
            for dt in dtypes:
                trajs = upload_batch(api, bl, dev, dt)
                plan = api.BatchPlan(trajs, ops if dt == torch.float64 else ("discretize",),
                                     sched="tune", graph=True, stream=stream)
                res = {}
                for op in (ops if dt == torch.float64 else ("discretize",)):
                    ms_b, _ = timed(lambda: plan.run(op, graph=True, stream=stream), stream,
                                    args.batch_steps, 2)
                    res[op] = {"value": nint / (ms_b * 1e-3),
                               "unit": "intervals/s" if op == "discretize" else "interval grads/s",
                               "ms_per_step": ms_b}
                    if op == "discretize":
                        peak = PEAK_FP64_VALU if dt == torch.float64 else PEAK_FP32_VALU
                        res[op]["roofline_frac"] = bflops / (ms_b * 1e-3) / peak
                key = f"{name}_{'f64' if dt == torch.float64 else 'f32'}"
                progress(f"batch {key}: " + ", ".join(f"{o} {r['ms_per_step']:.3f} ms"
                                                      for o, r in res.items()))
                batch[key] = dict(trajectories=len(bl), intervals=nint, **res,
                                  groups=plan.groups())
                plan.close()
                del trajs

    line = {
        "metric": "discretized intervals/s (x+STM+B±) at 1e-10 rel vs oracle",
        "value": N / (ms64 * 1e-3),
        "unit": "intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cheetah7 planar chain (7 bodies, 6 joints, 2 contacts), "
                               "N=50 intervals, K=20 RK4 substeps, FP64 forward",
                   "N": N, "substeps": K, "nx": cm.nx, "m": cm.m},
        "fp32": {"value": N / (ms32 * 1e-3), "unit": "intervals/s", "ms_per_step": ms32},
        "adjoint": {"value": N / (ms_grad * 1e-3), "unit": "interval grads/s",
                    "ms_per_step": ms_grad,
                    "step": "cis_defects with checkpoints every 5 substeps + cis_discretize_adjoint"},
        "roofline": {"bound": "alu", "kernel": kname,
                     "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                     "traffic": committed_traffic(kname),
                     "algorithmic_flop_per_launch": flops},
        "batch": batch,
        "wall_s_timed_region": wall64,
    }
    if not args.no_cpu_baseline:
        # CPU-baseline leg: the plain FP64 oracle on the host cores, on the same
        # seeded inputs; its result also gives the parity of the timed outputs.
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import PHI32, PHI64, block_err
        ref = oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K)
        v64 = api.as_interval_major(out64)
        line["max_rel_err_vs_oracle"] = max(
            block_err(v64[k].double().cpu().numpy(), ref[k], PHI64)
            for k in ("A", "Bm", "Bp", "S", "d", "xprop"))
        r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        ref32 = oracle.discretize(model, r32(data["X"]), r32(data["U"]), r32(data["s"]),
                                  r32(data["p"]), K)
        v32 = api.as_interval_major(out32)
        line["fp32"]["max_rel_err_vs_oracle_normwise"] = max(
            block_err(v32[k].double().cpu().numpy(), ref32[k], PHI32)
            for k in ("A", "Bm", "Bp", "S", "d", "xprop"))
        ncores = os.cpu_count() or 1
        ncores = min(ncores, 16)
        reps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K, nthreads=ncores)
            reps += 1
        dt = time.perf_counter() - t0
        progress(f"cpu baseline {reps} repetitions in {dt:.1f} s")
        line["cpu_baseline"] = {"value": reps * N / dt, "unit": "intervals/s", "cores": ncores,
                                "kind": "oracle",
                                "sample": f"{reps} repetitions of the same 50-interval workload "
                                          f"({reps * N} intervals, {dt:.1f} s, OpenMP over intervals)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
