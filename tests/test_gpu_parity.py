"""HIP path vs the CPU oracle, element by element (GPU).

Bar: FP64 per-block error <= 1e-10 (phi = 1e-3), FP32 normwise <= 1e-4 with
the oracle in FP64 on the FP32-rounded inputs (metric in tests/parity.py).
Structural entries (A[:, n:] = [0; I]) must match exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2604_09993_amd import synth
from parity import PHI32, PHI64, TOL32, TOL64, block_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _api():
    from paper_2604_09993_amd import api
    return api


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model(name, seed):
    rng = np.random.default_rng(seed)
    if name == "point1s":
        return synth.make_point_contact(rng, terrain="sinusoid"), rng
    if name == "chain3":
        return synth.legged_model("chain3", 1, 2, rng), rng
    if name == "biped3":
        return synth.legged_model("biped3", 2, 1, rng, terrain="sinusoid"), rng
    return synth.MODEL_MAKERS[name](rng), rng


def run_gpu(model, data, K, dtype=torch.float64, ld_node_pad=0, ld_int_pad=0, with_xprop=True):
    api = _api()
    dev = torch.device("cuda:0")
    N = data["s"].shape[0]
    cm = api.CisModel(model)
    ld = N + 1 + ld_node_pad
    X = api.to_device_soa(data["X"], dev, dtype, ld=ld)
    U = api.to_device_soa(data["U"], dev, dtype, ld=ld)
    s = torch.tensor(data["s"], device=dev, dtype=dtype)
    p = torch.tensor(data["p"], device=dev, dtype=dtype)
    if ld_int_pad:
        ldi = N + ld_int_pad
        kw = dict(device=dev, dtype=dtype)
        nx, m = cm.nx, cm.m
        full = dict(A=torch.full((nx, nx, ldi), np.nan, **kw), Bm=torch.full((nx, m, ldi), np.nan, **kw),
                    Bp=torch.full((nx, m, ldi), np.nan, **kw), S=torch.full((nx, ldi), np.nan, **kw),
                    d=torch.full((nx, ldi), np.nan, **kw), xprop=torch.full((nx, ldi), np.nan, **kw))
        api.discretize_into(cm, X, U, s, p, K, full)
        torch.cuda.synchronize()
        # padding untouched
        assert torch.isnan(full["A"][..., N:]).all() and torch.isnan(full["d"][:, N:]).all()
        out = {k: v[..., :N] for k, v in full.items()}
    else:
        out = api.discretize(cm, X, U, s, p, K, with_xprop=with_xprop)
        torch.cuda.synchronize()
    res = {}
    for k, v in api.as_interval_major(out).items():
        res[k] = None if v is None else v.double().cpu().numpy()
    return res, cm


def check_against_oracle(model, data, K, res, dtype=torch.float64):
    X, U, s, p = data["X"], data["U"], data["s"], data["p"]
    if dtype == torch.float32:
        r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        X, U, s, p = r32(X), r32(U), r32(s), r32(p)
        tol, phi = TOL32, PHI32
    else:
        tol, phi = TOL64, PHI64
    ref = oracle.discretize(model, X, U, s, p, K)
    errs = {}
    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
        if res.get(key) is None:
            continue
        errs[key] = block_err(res[key], ref[key], phi)
    n, ny = model.n, model.ny
    A = res["A"]
    assert np.all(A[:, :n, n:] == 0.0)
    assert np.all(A[:, n:, n:] == np.eye(ny)[None])
    bad = {k: e for k, e in errs.items() if not e <= tol}
    assert not bad, (bad, errs)
    return errs


SMALL = [("free1", 3, 4), ("point1", 3, 4), ("point1s", 4, 3), ("hopper", 5, 3),
         ("chain3", 3, 3), ("biped3", 3, 3), ("biped5", 4, 3), ("cheetah7", 4, 3), ("quad13", 3, 2)]


@pytest.mark.parametrize("name,N,K", SMALL)
def test_discretize_small_fp64(name, N, K):
    _say(f"[gpu] discretize fp64 {name} N={N} K={K} seed=100")
    model, rng = _model(name, 100)
    data = synth.gen_nodes(model, N, rng)
    res, _ = run_gpu(model, data, K)
    check_against_oracle(model, data, K, res)


@pytest.mark.parametrize("name,N,K", [("hopper", 3, 2), ("biped5", 3, 2), ("cheetah7", 3, 2),
                                      ("quad13", 2, 2)])
def test_discretize_small_fp32(name, N, K):
    """FP32 on intervals of the configurations' length (s ~ 0.02 s).

    On long intervals with few substeps the map itself is ill-conditioned: for
    quad13 with N=2, K=2 over 1 s, perturbing the inputs at FP32 rounding
    (6e-8) moves the FP64 oracle outputs by ~2e-3 normwise, so no FP32
    evaluation can meet 1e-4 there.
    """
    _say(f"[gpu] discretize fp32 {name} N={N} K={K} seed=101")
    model, rng = _model(name, 101)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    res, _ = run_gpu(model, data, K, dtype=torch.float32)
    check_against_oracle(model, data, K, res, dtype=torch.float32)


@pytest.mark.parametrize("N", [300, 200, 110, 70, 30, 22])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("name", [n for n, _, _ in SMALL])
def test_discretize_many_intervals_sampled(name, dtype, N):
    """More intervals than the small cases above, which take the latency
    layout with the S column in a group of its own.  With 256 CUs (FP64 column
    groups: latency / latency with S on leg lanes / narrow = 4 / 3 / 2 for
    biped5 and cheetah7, 12 / 11 / 6 for quad13, 2 / 1 / 1 for hopper):
    N = 300 takes the throughput layout for every model; N = 200 the latency
    layout with S on leg lanes for hopper (and FP32 models); N = 110 the
    narrow layout for biped5 / cheetah7; N = 70 the latency layout with S on
    leg lanes for them; N = 30 the narrow layout and N = 22 the latency layout
    with S on leg lanes for quad13.  4 sampled intervals vs the oracle."""
    K = 2
    _say(f"[gpu] discretize {dtype} {name} N={N} K={K} seed=102 (sampled)")
    dt = torch.float64 if dtype == "fp64" else torch.float32
    model, rng = _model(name, 102)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    res, _ = run_gpu(model, data, K, dtype=dt)
    for k in (0, 1, N // 2, N - 1):
        sub = dict(X=data["X"][k:k + 2], U=data["U"][k:k + 2], s=data["s"][k:k + 1], p=data["p"])
        one = {key: (None if v is None else v[k:k + 1]) for key, v in res.items()}
        check_against_oracle(model, sub, K, one, dtype=dt)


def test_edge_single_interval_single_substep():
    _say("[gpu] discretize fp64 cheetah7 N=1 K=1")
    model, rng = _model("cheetah7", 102)
    data = synth.gen_nodes(model, 1, rng)
    res, _ = run_gpu(model, data, 1)
    check_against_oracle(model, data, 1, res)


def test_edge_padded_leading_dimensions_and_no_xprop():
    _say("[gpu] discretize fp64 biped5 N=5 K=2 ld padding")
    model, rng = _model("biped5", 103)
    data = synth.gen_nodes(model, 5, rng)
    res, _ = run_gpu(model, data, 2, ld_node_pad=3, ld_int_pad=7)
    check_against_oracle(model, data, 2, res)
    res, _ = run_gpu(model, data, 2, with_xprop=False)
    assert res["xprop"] is None
    check_against_oracle(model, data, 2, res)


def test_workload_hopper_N20_K10_full():
    _say("[gpu] workload hopper N=20 K=10 fp64")
    model, data, K = synth.make_workload("hopper_N20_K10")
    res, _ = run_gpu(model, data, K)
    check_against_oracle(model, data, K, res)


def test_workload_cheetah7_N50_K20_full_fp64_fp32():
    _say("[gpu] workload cheetah7 N=50 K=20 fp64")
    model, data, K = synth.make_workload("cheetah7_N50_K20")
    res, _ = run_gpu(model, data, K)
    check_against_oracle(model, data, K, res)
    _say("[gpu] workload cheetah7 N=50 K=20 fp32")
    res, _ = run_gpu(model, data, K, dtype=torch.float32)
    check_against_oracle(model, data, K, res, dtype=torch.float32)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_workload_quad13_N200_K20_sampled(dtype):
    """Full N=200, K=20 trajectory on the GPU; 6 sampled intervals recomputed by the oracle."""
    _say(f"[gpu] workload quad13 N=200 K=20 {dtype} (sampled)")
    dt = torch.float64 if dtype == "fp64" else torch.float32
    model, data, K = synth.make_workload("quad13_N200_K20_x64")
    res, _ = run_gpu(model, data, K, dtype=dt)
    for k in (0, 1, 77, 128, 198, 199):
        sub = dict(X=data["X"][k:k + 2], U=data["U"][k:k + 2], s=data["s"][k:k + 1], p=data["p"])
        one = {key: (None if v is None else v[k:k + 1]) for key, v in res.items()}
        check_against_oracle(model, sub, K, one, dtype=dt)


def test_defects_match_discretize_and_oracle():
    _say("[gpu] defects fp64 cheetah7 N=6 K=4 ckpt 2")
    api = _api()
    model, rng = _model("cheetah7", 104)
    data = synth.gen_nodes(model, 6, rng)
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    out = api.defects(cm, X, U, s, p, 4, ckpt_every=2)
    full = api.discretize(cm, X, U, s, p, 4)
    torch.cuda.synchronize()
    ref = oracle.defects(model, data["X"], data["U"], data["s"], data["p"], 4)
    assert block_err(out["d"].t().cpu().numpy(), ref["d"], PHI64) <= TOL64
    assert block_err(out["xprop"].t().cpu().numpy(), ref["xprop"], PHI64) <= TOL64
    # the two kernels evaluate the same right-hand side (in different summation orders)
    assert block_err(out["xprop"].t().cpu().numpy(), full["xprop"].t().cpu().numpy(), PHI64) <= 1e-13
    # checkpoint 0 is the node state; checkpoint 1 is the state after 2 substeps
    ck = out["ckpt"].cpu().numpy()
    np.testing.assert_array_equal(ck[0].T, data["X"][:6, :model.n])
    mid = np.stack([oracle.integrate(model, data["X"][k], data["U"][k], data["U"][k + 1], data["s"][k],
                                     data["p"], 2, 0.0, 0.5)["xf"][:model.n] for k in range(6)])
    assert block_err(ck[1].T, mid, PHI64) <= TOL64
