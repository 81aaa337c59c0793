"""The allocation-free reverse sweep against the workspace form (GPU, through the C ABI).

cis_discretize_adjoint_noalloc runs the kernels of cis_discretize_adjoint with
a device array inside the library as the workspace.  Two calls in a row on one
stream, the second on a smaller input (fewer intervals, another model), must
each give exactly the outputs of cis_discretize_adjoint on the same inputs
(same kernels, same order of every sum), and the first call's results must
also sit within the parity bar of the oracle's reverse sweep.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2604_09993_amd import synth
from parity import PHI64, TOL64, block_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs(name, N, seed):
    rng = np.random.default_rng(seed)
    model = synth.MODEL_MAKERS[name](rng)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    lam = rng.normal(size=(N, model.nx))
    return model, data, lam


def _run_both(model, data, K, C, lam, stream):
    """(workspace form, no-alloc form) outputs on the same device inputs."""
    from paper_2604_09993_amd import _lib, api
    dev = torch.device("cuda:0")
    lib = _lib.load()
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    N = s.shape[0]
    fw = api.defects(cm, X, U, s, p, K, ckpt_every=C, stream=stream)
    seed = torch.tensor(np.ascontiguousarray(lam.T), device=dev)
    sh = _lib.Shape(N, K, _lib.CIS_F64, 0, X.stride(0), N)
    vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    sp = ctypes.c_void_p(stream.cuda_stream)
    outs = []
    for form in ("ws", "noalloc"):
        kw = dict(device=dev, dtype=torch.float64)
        gX = torch.full((cm.nx, X.stride(0)), np.nan, **kw)
        gU = torch.full((max(cm.m, 1), X.stride(0)), np.nan, **kw)
        gs = torch.full((N,), np.nan, **kw)
        gp = torch.full((cm.np,), np.nan, **kw)
        if form == "ws":
            nb = api.adjoint_workspace_bytes(cm, N, K)
            ws = torch.empty((nb,), device=dev, dtype=torch.uint8)
            st = lib.cis_discretize_adjoint(cm.handle, ctypes.byref(sh), vp(X), vp(U), vp(s),
                                            vp(p), vp(fw["ckpt"]), C, vp(seed), vp(gX),
                                            vp(gU if cm.m else None), vp(gs), vp(gp), vp(ws),
                                            nb, sp)
        else:
            st = lib.cis_discretize_adjoint_noalloc(cm.handle, ctypes.byref(sh), vp(X), vp(U),
                                                    vp(s), vp(p), vp(fw["ckpt"]), C, vp(seed),
                                                    vp(gX), vp(gU if cm.m else None), vp(gs),
                                                    vp(gp), sp)
        _lib.check(st)
        stream.synchronize()
        outs.append(dict(gX=gX[:, :N + 1].cpu().numpy(), gU=gU[:cm.m, :N + 1].cpu().numpy(),
                         gs=gs.cpu().numpy(), gp=gp.cpu().numpy()))
        if form == "ws":
            del ws
    return outs


def test_noalloc_adjoint_matches_workspace_form_twice():
    stream = torch.cuda.current_stream()
    cases = [("cheetah7", 24, 10, 5, 901), ("biped5", 7, 6, 2, 902)]   # second call smaller
    for i, (name, N, K, C, seed) in enumerate(cases):
        _say(f"[gpu] no-alloc adjoint call {i + 1}: {name} N={N} K={K} C={C} seed={seed}")
        model, data, lam = _inputs(name, N, seed)
        ref, got = _run_both(model, data, K, C, lam, stream)
        for key in ("gX", "gU", "gs", "gp"):
            assert np.array_equal(got[key], ref[key]), (i, key)
            assert np.all(np.isfinite(got[key])), (i, key)
        if i == 0:
            o = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, lam)
            assert block_err(got["gX"].T, o["gX"], PHI64) <= TOL64
            assert block_err(got["gU"].T, o["gU"], PHI64) <= TOL64
            assert block_err(got["gs"].reshape(1, -1), o["gs"].reshape(1, -1), PHI64) <= TOL64
            assert block_err(got["gp"].reshape(1, -1), o["gp"].reshape(1, -1), PHI64) <= TOL64
