"""Split discretize form (coefficient records + leg-wave tangent kernel) vs the oracle (GPU).

cis_discretize_split computes the same discrete map as cis_discretize in two
launches.  Bars as for the fused kernel: FP64 per-block error <= 1e-10
(phi = 1e-3), FP32 normwise <= 1e-4 with the oracle on the FP32-rounded
inputs; structural entries A[:, n:] = [0; I] exact.  Cases span one and
several 64-column blocks (hopper 24 tangent columns, biped5 66, cheetah7 90,
quad13 174), both register budgets of the tangent kernel, padded leading
dimensions (untouched padding), and the quad13 N = 200, K = 20 workload
(sampled intervals).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2604_09993_amd import synth
from parity import PHI32, PHI64, TOL32, TOL64, block_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("A", "Bm", "Bp", "S", "d", "xprop")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _model(name, seed):
    rng = np.random.default_rng(seed)
    if name == "chain3":
        return synth.legged_model("chain3", 1, 2, rng), rng
    if name == "biped3":
        return synth.legged_model("biped3", 2, 1, rng, terrain="sinusoid"), rng
    return synth.MODEL_MAKERS[name](rng), rng


def run_split(model, data, K, dtype, waves, ld_int_pad=0):
    from paper_2604_09993_amd import _lib, api
    import ctypes
    dev = torch.device("cuda:0")
    N = data["s"].shape[0]
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev, dtype)
    U = api.to_device_soa(data["U"], dev, dtype)
    s = torch.tensor(data["s"], device=dev, dtype=dtype)
    p = torch.tensor(data["p"], device=dev, dtype=dtype)
    if not ld_int_pad:
        out = api.discretize_split(cm, X, U, s, p, K, waves=waves)
        torch.cuda.synchronize()
        return {k: v.double().cpu().numpy() for k, v in api.as_interval_major(out).items()}, cm
    ldi = N + ld_int_pad
    kw = dict(device=dev, dtype=dtype)
    nx, m = cm.nx, cm.m
    full = dict(A=torch.full((nx, nx, ldi), np.nan, **kw), Bm=torch.full((nx, m, ldi), np.nan, **kw),
                Bp=torch.full((nx, m, ldi), np.nan, **kw), S=torch.full((nx, ldi), np.nan, **kw),
                d=torch.full((nx, ldi), np.nan, **kw), xprop=torch.full((nx, ldi), np.nan, **kw))
    nb = api.split_workspace_bytes(cm, N, K, dtype)
    ws = torch.empty((nb,), device=dev, dtype=torch.uint8)
    sh = _lib.Shape(N, K, api._dtype_code(dtype), 0, X.stride(0), ldi)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    _lib.check(_lib.load().cis_discretize_split(
        cm.handle, ctypes.byref(sh), vp(X), vp(U), vp(s), vp(p), waves, vp(full["A"]),
        vp(full["Bm"]), vp(full["Bp"]), vp(full["S"]), vp(full["d"]), vp(full["xprop"]), vp(ws),
        nb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    for k, v in full.items():
        assert torch.isnan(v[..., N:]).all(), k
    out = {k: v[..., :N] for k, v in full.items()}
    return {k: v.double().cpu().numpy() for k, v in api.as_interval_major(out).items()}, cm


def check(model, data, K, res, fp32, ks=None):
    X, U, s, p = data["X"], data["U"], data["s"], data["p"]
    phi, tol = (PHI32, TOL32) if fp32 else (PHI64, TOL64)
    if fp32:
        X, U, s, p = _r32(X), _r32(U), _r32(s), _r32(p)
    if ks is None:
        ref = oracle.discretize(model, X, U, s, p, K)
        got = res
    else:
        refs = [oracle.discretize(model, X[k:k + 2], U[k:k + 2], s[k:k + 1], p, K) for k in ks]
        ref = {key: np.concatenate([r[key] for r in refs]) for key in KEYS}
        got = {key: res[key][ks] for key in KEYS}
    errs = {key: block_err(got[key], ref[key], phi) for key in KEYS
            if not (model.m == 0 and key in ("Bm", "Bp"))}
    n, ny = model.n, model.ny
    assert np.all(got["A"][:, :n, n:] == 0.0)
    assert np.all(got["A"][:, n:, n:] == np.eye(ny)[None])
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, (bad, errs)
    return errs


CASES = [("hopper", 5, 3), ("chain3", 3, 3), ("biped3", 3, 3), ("biped5", 4, 3),
         ("cheetah7", 4, 3), ("quad13", 3, 2)]


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("name,N,K", CASES)
def test_split_small_fp64(name, N, K, waves):
    """quad13 on intervals of the configurations' length (s ~ 0.02 s): with
    the default 0.26-0.37 s intervals and K = 2 a one-ulp perturbation of the
    inputs already moves the oracle by ~8e-11, the order of the bar
    (tests/test_conditioning.py measures it)."""
    _say(f"[gpu] split fp64 {name} N={N} K={K} waves={waves} seed=300")
    model, rng = _model(name, 300)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N) if name == "quad13" else \
        synth.gen_nodes(model, N, rng)
    res, _ = run_split(model, data, K, torch.float64, waves)
    check(model, data, K, res, False)


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("name,N,K", [("hopper", 3, 2), ("biped5", 3, 2), ("cheetah7", 3, 2),
                                      ("quad13", 2, 2)])
def test_split_small_fp32(name, N, K, waves):
    """Intervals of the configurations' length (s ~ 0.02 s), as for the fused kernel."""
    _say(f"[gpu] split fp32 {name} N={N} K={K} waves={waves} seed=301")
    model, rng = _model(name, 301)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    res, _ = run_split(model, data, K, torch.float32, waves)
    check(model, data, K, res, True)


@pytest.mark.parametrize("name", ["biped5", "quad13"])
def test_split_padded_leading_dimension(name):
    _say(f"[gpu] split fp64 {name} N=7 K=2 ld_int=N+5 seed=302")
    model, rng = _model(name, 302)
    data = synth.gen_nodes(model, 7, rng, T=0.14)
    res, _ = run_split(model, data, 2, torch.float64, 1, ld_int_pad=5)
    check(model, data, 2, res, False)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("waves", [1, 2])
def test_split_quad13_workload_sampled(dtype, waves):
    """The quad13 N = 200, K = 20 trajectory of the batched workload: 6 sampled
    intervals (first, last and four drawn) against the oracle."""
    fp32 = dtype == "fp32"
    _say(f"[gpu] split {dtype} quad13 N=200 K=20 waves={waves} (sampled)")
    model, data, K = synth.workload_batch("quad13_N200_K20_x64")[5]
    res, _ = run_split(model, data, K, torch.float32 if fp32 else torch.float64, waves)
    rng = np.random.default_rng(303)
    ks = sorted({0, 199} | set(int(v) for v in rng.choice(200, size=4, replace=False)))
    check(model, data, K, res, fp32, ks=ks)


def test_split_matches_fused_cheetah7():
    """Same map as cis_discretize: on cheetah7 N = 50, K = 20 the two forms
    agree to within the FP64 bar of each other (sums ordered differently)."""
    from paper_2604_09993_amd import api
    _say("[gpu] split vs fused cheetah7 N=50 K=20")
    model, data, K = synth.make_workload("cheetah7_N50_K20")
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    a = api.as_interval_major(api.discretize(cm, X, U, s, p, K))
    b = api.as_interval_major(api.discretize_split(cm, X, U, s, p, K))
    torch.cuda.synchronize()
    for key in KEYS:
        e = block_err(b[key].cpu().numpy(), a[key].cpu().numpy(), PHI64)
        assert e <= 1e-12, (key, e)


def test_batch_run_parts_equal_run():
    """cis_batch_run_part: the split form's two launches enqueued one by one
    give exactly the outputs of cis_batch_run (same kernels, same order)."""
    from paper_2604_09993_amd import api
    _say("[gpu] batch run parts vs run: 3 cheetah7 trajectories N=12 K=4, split form")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(304)
    model = synth.make_cheetah7(rng)
    cm = api.CisModel(model)
    trajs = []
    for _ in range(3):
        data = synth.gen_nodes(model, 12, rng, T=0.24)
        trajs.append(dict(cm=cm, K=4, X=api.to_device_soa(data["X"], dev),
                          U=api.to_device_soa(data["U"], dev),
                          s=torch.tensor(data["s"], device=dev),
                          params=torch.tensor(data["p"], device=dev)))
    plan = api.BatchPlan(trajs, ("discretize",), sched="grid", graph=False, form="split")
    assert plan.groups()[0]["split"] == 1
    plan.run("discretize")
    torch.cuda.synchronize()
    ref = [{k: o[k].clone() for k in KEYS} for o in plan.out]
    for o in plan.out:
        for k in KEYS:
            o[k].fill_(float("nan"))
    plan.run_part("discretize", 0)
    plan.run_part("discretize", 1)
    torch.cuda.synchronize()
    for o, r in zip(plan.out, ref):
        for k in KEYS:
            assert torch.equal(o[k], r[k]), k
    plan.close()
