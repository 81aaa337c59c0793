"""Substep-blocked discretization (GPU): block sensitivities integrated in
parallel and chained by dense products on the vector ALUs or FP64 MFMA.

The result is the chain rule applied over the block boundaries, so it must
meet the same parity bar as the fused kernel against the CPU oracle (FP64
1e-10, phi = 1e-3), for several block counts and both compositions, and
agree with the fused kernel to rounding (1e-12 relative per block).
"""
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


CASES = [("hopper", 5, 4, 2), ("hopper", 5, 4, 4), ("biped5", 4, 6, 3), ("cheetah7", 6, 4, 2),
         ("cheetah7", 6, 8, 4), ("quad13", 3, 4, 2), ("point1", 3, 4, 2), ("free1", 2, 2, 2)]


@pytest.mark.parametrize("compose", ["valu", "mfma"])
@pytest.mark.parametrize("name,N,K,B", CASES)
def test_blocked_matches_oracle_and_fused(name, N, K, B, compose):
    from paper_2604_09993_amd import api
    _say(f"[gpu] blocked {compose} {name} N={N} K={K} B={B} seed=110")
    rng = np.random.default_rng(110)
    model = synth.MODEL_MAKERS[name](rng) if name in synth.MODEL_MAKERS else None
    if model is None:
        model = (synth.make_point_contact(rng) if name == "point1" else synth.make_free_body(rng))
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    got = api.discretize_blocked(cm, X, U, s, p, K, B, compose)
    fused = api.discretize(cm, X, U, s, p, K)
    torch.cuda.synchronize()
    ref = oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K)
    g = api.as_interval_major(got)
    f = api.as_interval_major(fused)
    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
        if model.m == 0 and key in ("Bm", "Bp"):
            continue
        gk = g[key].cpu().numpy()
        e = block_err(gk, ref[key], PHI64)
        assert e <= TOL64, (key, e)
        fk = f[key].cpu().numpy()
        scale = max(np.max(np.abs(fk)), 1e-300)
        assert np.max(np.abs(gk - fk)) / scale <= 1e-12, key


def test_blocked_rejects_bad_block_counts():
    from paper_2604_09993_amd import api, _lib
    model = synth.make_hopper(np.random.default_rng(0))
    data = synth.gen_nodes(model, 3, np.random.default_rng(1))
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    for B in (1, 3):   # 1 is not blocked, 3 does not divide 4
        with pytest.raises(_lib.CisError):
            api.discretize_blocked(cm, X, U, s, p, 4, B)
    with pytest.raises(_lib.CisError):
        api.discretize_blocked(cm, X.float(), U.float(), s.float(), p.float(), 4, 2)


def _check_choice(choice, K, dtype):
    if choice["form"] == "one_launch":
        assert choice["layout"] in ("latency", "latency_s", "narrow", "throughput")
    elif choice["form"] == "split":
        assert choice["waves"] in (1, 2)
    else:
        assert dtype == torch.float64 and 2 <= choice["blocks"] <= 8
        assert K % choice["blocks"] == 0 and choice["compose"] in ("valu", "mfma")


@pytest.mark.parametrize("name,dtype", [("cheetah7", torch.float64), ("cheetah7", torch.float32),
                                        ("point1", torch.float64)])
def test_single_tuner_choice_matches_the_oracle_and_is_cached(tmp_path, monkeypatch, name, dtype):
    """The single-trajectory tuner (one-launch layouts, split form, blocked
    forms) returns one of its candidates, its outputs are that
    configuration's (checked against the oracle), and a second call reads the
    same choice back from the CIS_TUNE_CACHE file."""
    import oracle
    from paper_2604_09993_amd import api, synth
    from parity import PHI32, PHI64, TOL32, TOL64, block_err
    print(f"single tune {name} N=8 K=8 {dtype}", flush=True)
    rng = np.random.default_rng(41)
    model = synth.MODEL_MAKERS[name](rng)
    d = synth.gen_nodes(model, 8, rng, T=0.16)
    K = 8
    cm = api.CisModel(model)
    X, U = api.to_device_soa(d["X"], dtype=dtype), api.to_device_soa(d["U"], dtype=dtype)
    s = torch.tensor(d["s"], device="cuda", dtype=dtype)
    p = torch.tensor(d["p"], device="cuda", dtype=dtype)
    monkeypatch.setenv("CIS_TUNE_CACHE", str(tmp_path / "tune.json"))
    out, choice = api.single_tune(cm, X, U, s, p, K)
    assert not choice["from_cache"] and choice["ms"] > 0
    _check_choice(choice, K, dtype)
    if model.nb == 1:
        assert choice["form"] != "split"   # no legs with links: no split candidate
    # FP32: the oracle runs on the same FP32-rounded inputs
    r = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 \
        else (lambda a: a)
    ref = oracle.discretize(model, r(d["X"]), r(d["U"]), r(d["s"]), r(d["p"]), K)
    got = api.as_interval_major(out)
    phi, tol = (PHI64, TOL64) if dtype == torch.float64 else (PHI32, TOL32)
    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
        assert block_err(got[key].double().cpu().numpy(), ref[key], phi) <= tol, key
    out2, choice2 = api.single_tune(cm, X, U, s, p, K)
    assert choice2["from_cache"]
    for f in ("form", "layout", "waves", "blocks", "compose"):
        assert choice2[f] == choice[f], f
    got2 = api.as_interval_major(out2)
    for key in ("A", "S", "d"):
        assert torch.equal(got2[key], got[key]), key
    path = tmp_path / "tune.json"
    assert '"form"' in path.read_text()
    # an entry naming a configuration that does not exist for this shape is
    # ignored (the shape is tuned again); a damaged file counts as empty
    import json
    cache = json.loads(path.read_text())
    for entry in cache["entries"].values():
        entry.update(form=2, blocks=3, compose=0)     # 3 does not divide K = 8
    path.write_text(json.dumps(cache))
    _, choice3 = api.single_tune(cm, X, U, s, p, K)
    assert not choice3["from_cache"]
    _check_choice(choice3, K, dtype)
    path.write_text("{not json")
    _, choice4 = api.single_tune(cm, X, U, s, p, K)
    assert not choice4["from_cache"] and '"form"' in path.read_text()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("layout", ["latency", "latency_s", "narrow", "throughput"])
def test_every_one_launch_layout_matches_the_oracle(layout, dtype):
    """cis_shape.layout forces each workgroup layout of the one-launch kernel;
    every one gives the oracle's results (quadruped with a ragged N; FP32
    against the oracle on the same FP32-rounded inputs)."""
    import oracle
    from paper_2604_09993_amd import api, synth
    from parity import PHI32, PHI64, TOL32, TOL64, block_err
    print(f"layout {layout} quad13 N=7 K=6 {dtype}", flush=True)
    rng = np.random.default_rng(43)
    model = synth.make_quad13(rng)
    d = synth.gen_nodes(model, 7, rng, T=0.14)
    K = 6
    cm = api.CisModel(model)
    X = api.to_device_soa(d["X"], dtype=dtype)
    U = api.to_device_soa(d["U"], dtype=dtype)
    s = torch.tensor(d["s"], device="cuda", dtype=dtype)
    p = torch.tensor(d["p"], device="cuda", dtype=dtype)
    got = api.as_interval_major(api.discretize(cm, X, U, s, p, K, layout=layout))
    r = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 \
        else (lambda a: a)
    ref = oracle.discretize(model, r(d["X"]), r(d["U"]), r(d["s"]), r(d["p"]), K)
    phi, tol = (PHI64, TOL64) if dtype == torch.float64 else (PHI32, TOL32)
    for key in ("A", "Bm", "Bp", "S", "d", "xprop"):
        assert block_err(got[key].double().cpu().numpy(), ref[key], phi) <= tol, key
