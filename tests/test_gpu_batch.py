"""Batched multi-trajectory path (work lists, persistent grids, HIP graphs) (GPU).

Every trajectory of a batch must give what the single-trajectory entry
points give for it (same kernels' arithmetic; compared at 1e-13 relative per
block), and sampled trajectories are compared with the CPU oracle at the
parity bar (FP64 1e-10, FP32 1e-4 normwise).  Graph replays are checked
against the eager run after eager work in between, and a persistent plan is
run twice over NaN-filled outputs to show the device cursor resets.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2604_09993_amd import synth
from parity import PHI32, PHI64, TOL32, TOL64, block_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAME = 1e-13   # batch vs single-trajectory launch of the same arithmetic


def _api():
    from paper_2604_09993_amd import api
    return api


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small_batch(n_traj, seed, N_range=(3, 12), K_range=(2, 6)):
    """Mixed hopper / cheetah7 / biped5 batch with short intervals (T = 0.02 N)."""
    out = []
    for model, data, K in synth.mixed_batch(n_traj, seed, N_range, K_range):
        N = data["s"].shape[0]
        r = np.random.default_rng([seed, 99, N, K])
        data = dict(data)
        data["s"] = r.uniform(0.5, 2.0, size=N) * 0.02
        out.append((model, data, K))
    return out


def _upload(batch, dtype):
    api = _api()
    dev = torch.device("cuda:0")
    cms = {}
    trajs = []
    for model, data, K in batch:
        cm = cms.get(id(model))
        if cm is None:
            cm = cms[id(model)] = api.CisModel(model)
        N = data["s"].shape[0]
        trajs.append(dict(cm=cm, K=K, X=api.to_device_soa(data["X"], dev, dtype, ld=N + 1),
                          U=api.to_device_soa(data["U"], dev, dtype, ld=N + 1),
                          s=torch.tensor(data["s"], device=dev, dtype=dtype),
                          params=torch.tensor(data["p"], device=dev, dtype=dtype)))
    return trajs


def _single(t):
    api = _api()
    return api.discretize(t["cm"], t["X"], t["U"], t["s"], t["params"], t["K"])


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale) if b.size else 0.0


def _compare_to_single(plan, trajs, keys=("A", "Bm", "Bp", "S", "d", "xprop"), tol=SAME):
    worst = 0.0
    for i, t in enumerate(trajs):
        ref = _single(t)
        for k in keys:
            if t["cm"].m == 0 and k in ("Bm", "Bp"):
                continue
            e = _rel(plan.out[i][k], ref[k])
            assert e <= tol, (i, k, e)
            worst = max(worst, e)
    return worst


@pytest.mark.parametrize("sched,waves", [("grid", None), ("persistent", None), ("tune", None),
                                         ("grid", 2), ("persistent", 2), ("tune", 1)])
def test_batch_discretize_matches_single_and_oracle(sched, waves):
    """waves: register budget of the discretize kernel (None: default or tuned)."""
    api = _api()
    batch = _small_batch(9, seed=11)
    _say(f"batch discretize fp64 sched={sched} waves={waves} trajs={len(batch)}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize",), sched=sched, graph=False, waves_per_simd=waves)
    groups = plan.groups()
    assert len(groups) == 3 and sum(g["n_traj"] for g in groups) == 9
    if sched == "persistent":
        assert all(g["persist_blocks"] > 0 for g in groups)
    if sched == "grid":
        assert all(g["persist_blocks"] == 0 for g in groups)
    want = waves if waves is not None else (None if sched == "tune" else 1)
    assert all(g["waves_per_simd"] == want if want else g["waves_per_simd"] in (1, 2)
               for g in groups), groups
    plan.run("discretize")
    torch.cuda.synchronize()
    _compare_to_single(plan, trajs)
    # oracle on two trajectories of different models
    for i in (0, 4):
        model, data, K = batch[i]
        ref = oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K)
        got = api.as_interval_major({k: plan.out[i][k] for k in ("A", "Bm", "Bp", "S", "d",
                                                                    "xprop")})
        for k in ("A", "Bm", "Bp", "S", "d", "xprop"):
            e = block_err(got[k].cpu().numpy(), ref[k], PHI64)
            assert e <= TOL64, (i, k, e)
    plan.close()


def test_persistent_cursor_resets_between_launches():
    api = _api()
    batch = _small_batch(7, seed=12)
    _say("persistent plan twice over NaN-filled outputs")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize",), sched="persistent", graph=True)
    plan.run("discretize")
    torch.cuda.synchronize()
    first = [{k: v.clone() for k, v in o.items() if k in ("A", "Bm", "Bp", "S", "d")}
             for o in plan.out]
    for rep in range(2):
        for o in plan.out:
            for k in ("A", "Bm", "Bp", "S", "d"):
                o[k].fill_(float("nan"))
        plan.run("discretize", graph=bool(rep))
        torch.cuda.synchronize()
        for o, f in zip(plan.out, first):
            for k, v in f.items():
                assert torch.equal(o[k], v), (rep, k)
    plan.close()


def test_graph_replays_match_eager():
    api = _api()
    batch = _small_batch(8, seed=13)
    _say("graph replays vs eager")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize",), sched="grid", graph=True)
    plan.run("discretize")
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in o.items() if k in ("A", "Bm", "Bp", "S", "d", "xprop")}
             for o in plan.out]
    for rep in range(3):
        for o in plan.out:
            o["A"].zero_()
            o["d"].fill_(float("nan"))
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        plan.run("discretize", graph=True)
        torch.cuda.synchronize()
        for o, e in zip(plan.out, eager):
            for k, v in e.items():
                assert torch.equal(o[k], v), (rep, k)
    plan.close()


def test_batch_fp32_matches_single_and_oracle():
    api = _api()
    batch = _small_batch(6, seed=14)
    _say("batch discretize fp32")
    trajs = _upload(batch, torch.float32)
    plan = api.BatchPlan(trajs, ("discretize",), sched="tune", graph=True)
    assert all(g["waves_per_simd"] == 1 for g in plan.groups())   # one FP32 form
    plan.run("discretize", graph=True)
    torch.cuda.synchronize()
    _compare_to_single(plan, trajs, tol=1e-6)
    model, data, K = batch[1]
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    ref = oracle.discretize(model, r32(data["X"]), r32(data["U"]), r32(data["s"]),
                            r32(data["p"]), K)
    got = api.as_interval_major({k: plan.out[1][k] for k in ("A", "Bm", "Bp", "S", "d")})
    for k in ("A", "Bm", "Bp", "S", "d"):
        e = block_err(got[k].double().cpu().numpy(), ref[k], PHI32)
        assert e <= TOL32, (k, e)
    plan.close()


@pytest.mark.parametrize("graph,sched,spacing,waves", [
    (False, "grid", 0, None), (True, "grid", 0, 4), (True, "grid", 0, 3), (True, "grid", 0, 2),
    (True, "grid", 0, 1), (True, "tune", 0, None), (True, "grid", 10, None),
    (True, "grid", 10, 1), (True, "grid", 10, 4)])
def test_batch_adjoint_matches_single(graph, sched, spacing, waves):
    """spacing 0: checkpoints at most 8 substeps apart; 10: every 10 substeps with
    K in {10, 20} (chunked replay).  waves: forced form of the reverse sweep."""
    api = _api()
    batch = _small_batch(7, seed=15, K_range=(2, 8))
    if spacing:
        batch = [(m, d, 10 * (1 + i % 2)) for i, (m, d, _) in enumerate(batch)]
    _say(f"batch adjoint graph={graph} sched={sched} spacing={spacing} waves={waves}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize", "adjoint"), sched=sched, ckpt_every=spacing,
                         graph=graph, adjoint_waves=waves)
    chosen = {g["adjoint_waves"] for g in plan.groups()}
    if waves is not None:
        assert chosen == {min(waves, 2) if spacing > 8 else waves}, chosen
    gen = torch.Generator(device="cpu").manual_seed(5)
    for o in plan.out:
        o["seed"].copy_(torch.randn(o["seed"].shape, generator=gen, dtype=torch.float64))
    plan.run("adjoint", graph=graph)
    torch.cuda.synchronize()
    for i, t in enumerate(trajs):
        K = t["K"]
        C = spacing if spacing else max(c for c in range(1, 9) if K % c == 0)
        d = api.defects(t["cm"], t["X"], t["U"], t["s"], t["params"], K, ckpt_every=C)
        assert _rel(plan.out[i]["xprop"], d["xprop"]) <= SAME
        assert _rel(plan.out[i]["d"], d["d"]) <= SAME
        g = api.adjoint(t["cm"], t["X"], t["U"], t["s"], t["params"], K, d["ckpt"], C,
                        plan.out[i]["seed"])
        N = t["s"].shape[0]
        assert _rel(plan.out[i]["gX"][:, :N + 1], g["gX"]) <= SAME, i
        if t["cm"].m:
            assert _rel(plan.out[i]["gU"][:t["cm"].m, :N + 1], g["gU"]) <= SAME, i
        assert _rel(plan.out[i]["gs"], g["gs"]) <= SAME, i
        assert _rel(plan.out[i]["gp"], g["gp"]) <= SAME, i
    # the adjoint seeds against the oracle's reverse sweep for one trajectory
    model, data, K = batch[2]
    seed = plan.out[2]["seed"].cpu().numpy().T
    ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, seed)
    N = data["s"].shape[0]
    for key, got in (("gX", plan.out[2]["gX"][:, :N + 1].T), ("gs", plan.out[2]["gs"]),
                     ("gp", plan.out[2]["gp"])):
        got = got.cpu().numpy()
        scale = max(np.max(np.abs(ref[key])), 1e-300)
        assert np.max(np.abs(got - ref[key])) / scale <= TOL64, key
    plan.close()
