"""Debug mode of the single-trajectory entry points (CIS_DEBUG_FINITE): a call
counts the non-finite values of its inputs and outputs after the launch and
returns CIS_ERR_NONFINITE naming them; on finite data it changes nothing.
Without the variable a NaN input propagates to the outputs and the call
succeeds.  The NaN and inf inputs only flow through arithmetic with fixed
control flow (no value-dependent indexing), so every kernel runs as usual.
"""
import sys

import numpy as np
import pytest

from paper_2604_09993_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(dtype=torch.float64, name="cheetah7", N=5, K=4, seed=51):
    from paper_2604_09993_amd import api
    rng = np.random.default_rng(seed)
    model = synth.MODEL_MAKERS[name](rng)
    d = synth.gen_nodes(model, N, rng, T=0.02 * N)
    cm = api.CisModel(model)
    X = api.to_device_soa(d["X"], dtype=dtype)
    U = api.to_device_soa(d["U"], dtype=dtype)
    s = torch.tensor(d["s"], device="cuda", dtype=dtype)
    p = torch.tensor(d["p"], device="cuda", dtype=dtype)
    return api, cm, X, U, s, p, K


def _same(a, b):
    return all(torch.equal(a[k], b[k]) for k in a if a[k] is not None)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_debug_mode_leaves_finite_results_unchanged(monkeypatch, dtype):
    _say(f"debug finite: clean inputs {dtype}")
    api, cm, X, U, s, p, K = _setup(dtype)
    ref = api.discretize(cm, X, U, s, p, K)
    ref_split = api.discretize_split(cm, X, U, s, p, K)
    monkeypatch.setenv("CIS_DEBUG_FINITE", "1")
    assert _same(api.discretize(cm, X, U, s, p, K), ref)
    assert _same(api.discretize_split(cm, X, U, s, p, K), ref_split)
    if dtype == torch.float64:
        fw = api.defects(cm, X, U, s, p, K, ckpt_every=2)
        seed = torch.ones((cm.nx, s.shape[0]), device="cuda", dtype=dtype)
        g = api.adjoint(cm, X, U, s, p, K, fw["ckpt"], 2, seed)
        monkeypatch.setenv("CIS_DEBUG_FINITE", "0")
        g0 = api.adjoint(cm, X, U, s, p, K, fw["ckpt"], 2, seed)
        assert _same(g, g0)


def test_debug_mode_names_the_non_finite_arrays(monkeypatch):
    from paper_2604_09993_amd import _lib
    _say("debug finite: NaN in X, inf in params")
    api, cm, X, U, s, p, K = _setup()
    X[3, 2] = float("nan")
    # without debug mode the NaN propagates and the call succeeds
    out = api.discretize(cm, X, U, s, p, K)
    torch.cuda.synchronize()
    assert torch.isnan(out["A"]).any()
    monkeypatch.setenv("CIS_DEBUG_FINITE", "1")
    for call in (lambda: api.discretize(cm, X, U, s, p, K),
                 lambda: api.discretize_split(cm, X, U, s, p, K),
                 lambda: api.discretize_rkf(cm, X, U, s, p, K),
                 lambda: api.defects(cm, X, U, s, p, K)):
        with pytest.raises(_lib.CisError) as ei:
            call()
        assert ei.value.status == _lib.CIS_ERR_NONFINITE
        msg = str(ei.value)
        assert "input X 1" in msg and "output defect" in msg, msg
        assert "input U" not in msg and "input params" not in msg, msg
    X[3, 2] = 0.1
    p[0] = float("inf")
    with pytest.raises(_lib.CisError) as ei:
        api.discretize(cm, X, U, s, p, K)
    assert "input params 1" in str(ei.value) and "input X" not in str(ei.value)
    p[0] = 0.8
    assert api.discretize(cm, X, U, s, p, K)["A"].isfinite().all()
