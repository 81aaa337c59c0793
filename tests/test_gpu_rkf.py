"""Runge-Kutta-Fehlberg discretize form (cis_discretize_rkf) vs the oracle (GPU).

The same outputs as the RK4 forms, from K steps of Fehlberg's 4(5) pair per
interval, against oracle.discretize_rkf: FP64 per-block error <= 1e-10
(phi = 1e-3), FP32 normwise <= 1e-4 with the oracle on the FP32-rounded
inputs; the structural entries A[:, n:] = [0; I] exact.  The embedded
estimate err is a difference of the two solutions of a step (cancellation of
terms |h K| against a result |e|), so it is held to 1e-9 relative plus
1e-13 absolute in FP64 and checked only for sign and finiteness in FP32.
Cases: every compiled topology with legs with links, both register budgets,
padded leading dimensions, and the quad13 N = 200, K = 20 trajectory of the
batched workload (sampled intervals).
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


def run_rkf(model, data, K, dtype, waves, ld_int_pad=0):
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
        out = api.discretize_rkf(cm, X, U, s, p, K, waves=waves)
        torch.cuda.synchronize()
        return {k: v.double().cpu().numpy() for k, v in api.as_interval_major(out).items()}
    ldi = N + ld_int_pad
    kw = dict(device=dev, dtype=dtype)
    nx, m = cm.nx, cm.m
    full = dict(A=torch.full((nx, nx, ldi), np.nan, **kw), Bm=torch.full((nx, m, ldi), np.nan, **kw),
                Bp=torch.full((nx, m, ldi), np.nan, **kw), S=torch.full((nx, ldi), np.nan, **kw),
                d=torch.full((nx, ldi), np.nan, **kw), xprop=torch.full((nx, ldi), np.nan, **kw))
    err = torch.full((N,), np.nan, **kw)
    nb = api.rkf_workspace_bytes(cm, N, K, dtype)
    ws = torch.empty((nb,), device=dev, dtype=torch.uint8)
    sh = _lib.Shape(N, K, api._dtype_code(dtype), 0, X.stride(0), ldi)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    _lib.check(_lib.load().cis_discretize_rkf(
        cm.handle, ctypes.byref(sh), vp(X), vp(U), vp(s), vp(p), waves, vp(full["A"]),
        vp(full["Bm"]), vp(full["Bp"]), vp(full["S"]), vp(full["d"]), vp(full["xprop"]), vp(err),
        vp(ws), nb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    for k, v in full.items():
        assert torch.isnan(v[..., N:]).all(), k
    out = {k: v[..., :N] for k, v in full.items()}
    out["err"] = err
    return {k: v.double().cpu().numpy() for k, v in api.as_interval_major(out).items()}


def check(model, data, K, res, fp32, ks=None):
    X, U, s, p = data["X"], data["U"], data["s"], data["p"]
    phi, tol = (PHI32, TOL32) if fp32 else (PHI64, TOL64)
    if fp32:
        X, U, s, p = _r32(X), _r32(U), _r32(s), _r32(p)
    if ks is None:
        ref = oracle.discretize_rkf(model, X, U, s, p, K)
        got = res
    else:
        refs = [oracle.discretize_rkf(model, X[k:k + 2], U[k:k + 2], s[k:k + 1], p, K) for k in ks]
        ref = {key: np.concatenate([r[key] for r in refs]) for key in KEYS + ("err",)}
        got = {key: res[key][ks] for key in KEYS + ("err",)}
    errs = {key: block_err(got[key], ref[key], phi) for key in KEYS
            if not (model.m == 0 and key in ("Bm", "Bp"))}
    n, ny = model.n, model.ny
    assert np.all(got["A"][:, :n, n:] == 0.0)
    assert np.all(got["A"][:, n:, n:] == np.eye(ny)[None])
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, (bad, errs)
    e_got, e_ref = got["err"], ref["err"]
    assert np.all(np.isfinite(e_got)) and np.all(e_got >= 0.0)
    if not fp32:
        dev = np.abs(e_got - e_ref)
        assert np.all(dev <= 1e-9 * e_ref + 1e-13), (dev, e_ref)
    return errs


CASES = [("hopper", 5, 3), ("chain3", 3, 3), ("biped3", 3, 3), ("biped5", 4, 3),
         ("cheetah7", 4, 3), ("quad13", 3, 2)]


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("name,N,K", CASES)
def test_rkf_small_fp64(name, N, K, waves):
    """Intervals of the configurations' length (s ~ 0.02 s)."""
    _say(f"[gpu] rkf fp64 {name} N={N} K={K} waves={waves} seed=500")
    model, rng = _model(name, 500)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    res = run_rkf(model, data, K, torch.float64, waves)
    check(model, data, K, res, False)


@pytest.mark.parametrize("name,N,K", [("hopper", 3, 2), ("biped5", 3, 2), ("cheetah7", 3, 2),
                                      ("quad13", 2, 2)])
def test_rkf_small_fp32(name, N, K):
    _say(f"[gpu] rkf fp32 {name} N={N} K={K} seed=501")
    model, rng = _model(name, 501)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    res = run_rkf(model, data, K, torch.float32, 1)
    check(model, data, K, res, True)


@pytest.mark.parametrize("name", ["biped5", "quad13"])
def test_rkf_padded_leading_dimension(name):
    _say(f"[gpu] rkf fp64 {name} N=7 K=2 ld_int=N+5 seed=502")
    model, rng = _model(name, 502)
    data = synth.gen_nodes(model, 7, rng, T=0.14)
    res = run_rkf(model, data, 2, torch.float64, 1, ld_int_pad=5)
    check(model, data, 2, res, False)


@pytest.mark.parametrize("waves", [1, 2])
def test_rkf_quad13_workload_sampled(waves):
    """The quad13 N = 200, K = 20 trajectory of the batched workload: 6 sampled
    intervals (first, last and four drawn) against the oracle."""
    _say(f"[gpu] rkf fp64 quad13 N=200 K=20 waves={waves} (sampled)")
    model, data, K = synth.workload_batch("quad13_N200_K20_x64")[5]
    res = run_rkf(model, data, K, torch.float64, waves)
    rng = np.random.default_rng(503)
    ks = sorted({0, 199} | set(int(v) for v in rng.choice(200, size=4, replace=False)))
    check(model, data, K, res, False, ks=ks)


def test_rkf_is_not_rk4():
    """The two integrators give different maps on the same intervals (so the
    RKF parity above is not RK4 parity by accident), and both converge."""
    from paper_2604_09993_amd import api
    _say("[gpu] rkf vs rk4 cheetah7 N=50 K=20")
    model, data, K = synth.make_workload("cheetah7_N50_K20")
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    a = api.discretize_split(cm, X, U, s, p, K)
    b = api.discretize_rkf(cm, X, U, s, p, K)
    torch.cuda.synchronize()
    gap = (a["xprop"] - b["xprop"]).abs().max().item()
    assert gap > 1e-12
    assert gap < 1e-2 * max(1.0, a["xprop"].abs().max().item())
