"""Parity of the batched plans the benchmark times, on the benchmark's own inputs (GPU).

The benchmark replays plans over two batched workloads: 64 quad13
trajectories (N = 200, K = 20; FP64 and FP32 discretize, FP64 defects +
reverse sweep) and the uneven 256-trajectory mix (hopper / cheetah7 / biped5,
N in 20..100, K in 10..30; FP64 discretize and reverse sweep).  These tests
build the same plans (tuned, and with every schedule and register budget
fixed) from the same seeded inputs and compare with the oracle:

* discretize: sampled (trajectory, interval) pairs, at least 8 per plan and
  per model, each interval recomputed by the oracle on its own nodes (the
  intervals are independent given X_k, X_k+1, U_k, U_k+1, s_k), all six
  output blocks through the per-interval block metric;
* reverse sweep: whole trajectories (gX, gU, gs, gp) against the oracle's
  reverse sweep with the same cotangent seeds, at least 8 trajectories per
  plan covering every model, through the same metric (gU included).

Bars: FP64 1e-10 (phi = 1e-3), FP32 1e-4 normwise (oracle on the
FP32-rounded inputs).
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


def _api():
    from paper_2604_09993_amd import api
    return api


def _upload(batch, dtype):
    api = _api()
    dev = torch.device("cuda:0")
    cms, trajs = {}, []
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


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _oracle_interval(model, data, K, k, fp32):
    """Oracle outputs of interval k alone ([1, ...] arrays)."""
    X, U, s, p = data["X"][k:k + 2], data["U"][k:k + 2], data["s"][k:k + 1], data["p"]
    if fp32:
        X, U, s, p = _r32(X), _r32(U), _r32(s), _r32(p)
    return oracle.discretize(model, X, U, s, p, K)


def _samples(batch, per_model, seed):
    """(trajectory, interval) pairs: per model `per_model` pairs drawn without
    repeats, always including the first and last interval of some trajectory."""
    rng = np.random.default_rng(seed)
    by_model = {}
    for i, (model, data, K) in enumerate(batch):
        by_model.setdefault(id(model), []).append(i)
    out = []
    for trajs in by_model.values():
        picks = set()
        t0, t1 = trajs[0], trajs[-1]
        picks.add((t0, 0))
        picks.add((t1, batch[t1][1]["s"].shape[0] - 1))
        while len(picks) < per_model:
            t = int(rng.choice(trajs))
            picks.add((t, int(rng.integers(batch[t][1]["s"].shape[0]))))
        out.extend(sorted(picks))
    return out


def _interval_view(o, k):
    """Interval k of a plan's SoA outputs as [1, ...] numpy arrays."""
    return {"A": o["A"][:, :, k].double().cpu().numpy()[None],
            "Bm": o["Bm"][:, :, k].double().cpu().numpy()[None],
            "Bp": o["Bp"][:, :, k].double().cpu().numpy()[None],
            "S": o["S"][:, k].double().cpu().numpy()[None],
            "d": o["d"][:, k].double().cpu().numpy()[None],
            "xprop": o["xprop"][:, k].double().cpu().numpy()[None]}


def _check_sampled(plan, batch, refs, fp32):
    phi, tol = (PHI32, TOL32) if fp32 else (PHI64, TOL64)
    worst = 0.0
    for (t, k), ref in refs.items():
        got = _interval_view(plan.out[t], k)
        for key in KEYS:
            if batch[t][0].m == 0 and key in ("Bm", "Bp"):
                continue
            e = block_err(got[key], ref[key], phi)
            assert e <= tol, (t, k, key, e)
            worst = max(worst, e)
    return worst


@pytest.fixture(scope="module")
def quad13():
    batch = synth.workload_batch("quad13_N200_K20_x64")
    picks = _samples(batch, 8, seed=501)
    _say(f"quad13 x64: oracle on {len(picks)} sampled intervals (FP64 and FP32 inputs)")
    ref64 = {(t, k): _oracle_interval(*batch[t], k, False) for t, k in picks}
    ref32 = {(t, k): _oracle_interval(*batch[t], k, True) for t, k in picks}
    return batch, ref64, ref32


@pytest.mark.parametrize("sched,waves,form", [("tune", None, None), ("grid", 1, "fused"),
                                              ("grid", 2, "fused"), ("persistent", 1, "fused"),
                                              ("persistent", 2, "fused"), ("grid", 1, "split"),
                                              ("grid", 2, "split")])
def test_quad13x64_fp64_discretize_plans(quad13, sched, waves, form):
    api = _api()
    batch, ref64, _ = quad13
    _say(f"quad13 x64 fp64 discretize sched={sched} waves={waves} form={form}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize",), sched=sched, graph=True, waves_per_simd=waves,
                         form=form)
    g = plan.groups()
    assert len(g) == 1 and g[0]["n_items"] == 64 * 200
    if waves is not None:
        assert g[0]["waves_per_simd"] == waves
    if form is not None:
        assert g[0]["split"] == (form == "split")
    # NaN-filled outputs first, so a unit the plan skips cannot pass
    for o in plan.out:
        for key in KEYS:
            o[key].fill_(float("nan"))
    plan.run("discretize", graph=True)
    torch.cuda.synchronize()
    for o in plan.out:
        for key in KEYS:
            assert bool(torch.isfinite(o[key]).all()), key
    worst = _check_sampled(plan, batch, ref64, fp32=False)
    _say(f"  worst block error {worst:.3e}")
    plan.close()


@pytest.mark.parametrize("sched,form,waves", [("tune", None, None), ("grid", "fused", None),
                                              ("persistent", "fused", None),
                                              ("grid", "split", 1), ("grid", "split", 2)])
def test_quad13x64_fp32_discretize_plans(quad13, sched, form, waves):
    api = _api()
    batch, _, ref32 = quad13
    _say(f"quad13 x64 fp32 discretize sched={sched} form={form} waves={waves}")
    trajs = _upload(batch, torch.float32)
    plan = api.BatchPlan(trajs, ("discretize",), sched=sched, graph=True, form=form,
                         waves_per_simd=waves)
    if form is not None:
        assert plan.groups()[0]["split"] == (form == "split")
    for o in plan.out:
        for key in KEYS:
            o[key].fill_(float("nan"))
    plan.run("discretize", graph=True)
    torch.cuda.synchronize()
    for o in plan.out:
        for key in KEYS:
            assert bool(torch.isfinite(o[key]).all()), key
    worst = _check_sampled(plan, batch, ref32, fp32=True)
    _say(f"  worst block error {worst:.3e}")
    plan.close()


def _seeds(plan, seed):
    gen = torch.Generator(device="cpu").manual_seed(seed)
    lams = []
    for o in plan.out:
        lam = torch.randn(o["seed"].shape, generator=gen, dtype=torch.float64)
        o["seed"].copy_(lam)
        lams.append(lam.numpy().T.copy())
    return lams


def _check_adjoint_trajs(plan, batch, lams, picks):
    worst = 0.0
    for t in picks:
        model, data, K = batch[t]
        N = data["s"].shape[0]
        ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, lams[t])
        o = plan.out[t]
        got = {"gX": o["gX"][:, :N + 1].cpu().numpy().T,
               "gU": o["gU"][:model.m, :N + 1].cpu().numpy().T,
               "gs": o["gs"].cpu().numpy().reshape(1, -1),
               "gp": o["gp"].cpu().numpy().reshape(1, -1)}
        want = {"gX": ref["gX"], "gU": ref["gU"], "gs": ref["gs"].reshape(1, -1),
                "gp": ref["gp"].reshape(1, -1)}
        for key in ("gX", "gU", "gs", "gp"):
            if key == "gU" and model.m == 0:
                continue
            e = block_err(got[key], want[key], PHI64)
            assert e <= TOL64, (t, key, e)
            worst = max(worst, e)
        assert float(got["gp"][0, 1]) == 0.0   # restitution does not enter the interval map
    return worst


def _traj_picks(batch, per_model, seed):
    rng = np.random.default_rng(seed)
    by_model = {}
    for i, (model, _, _) in enumerate(batch):
        by_model.setdefault(id(model), []).append(i)
    out = []
    for trajs in by_model.values():
        k = min(per_model, len(trajs))
        out.extend(int(t) for t in rng.choice(trajs, size=k, replace=False))
    return sorted(out)


@pytest.mark.parametrize("defects_waves", [None, 2, 1])
def test_quad13x64_adjoint_plan(quad13, defects_waves):
    api = _api()
    batch, ref64, _ = quad13
    _say(f"quad13 x64 fp64 discretize + adjoint plan, defects form {defects_waves}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=True,
                         defects_waves=defects_waves)
    g = plan.groups()
    if defects_waves is not None:
        assert g[0]["defects_waves"] == defects_waves
    lams = _seeds(plan, 7)
    plan.run("discretize", graph=True)
    plan.run("adjoint", graph=True)
    torch.cuda.synchronize()
    if defects_waves is None:
        _check_sampled(plan, batch, ref64, fp32=False)
    worst = _check_adjoint_trajs(plan, batch, lams, _traj_picks(batch, 8, seed=502))
    _say(f"  worst gradient block error {worst:.3e}")
    plan.close()


@pytest.fixture(scope="module")
def mixed():
    batch = synth.mixed_batch()
    picks = _samples(batch, 8, seed=503)
    _say(f"mixed 256: oracle on {len(picks)} sampled intervals")
    refs = {(t, k): _oracle_interval(*batch[t], k, False) for t, k in picks}
    return batch, refs


@pytest.mark.parametrize("sched,waves,form", [("tune", None, None), ("grid", 2, "fused"),
                                              ("persistent", 1, "fused"), ("grid", 1, "split"),
                                              ("grid", 2, "split")])
def test_mixed256_discretize_plans(mixed, sched, waves, form):
    api = _api()
    batch, refs = mixed
    _say(f"mixed 256 fp64 discretize sched={sched} waves={waves} form={form}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize",), sched=sched, graph=True, waves_per_simd=waves,
                         form=form)
    g = plan.groups()
    assert len(g) == 3
    if form is not None:
        assert all(x["split"] == (form == "split") for x in g), g
    for o in plan.out:
        for key in KEYS:
            o[key].fill_(float("nan"))
    plan.run("discretize", graph=True)
    torch.cuda.synchronize()
    for o in plan.out:
        for key in KEYS:
            assert bool(torch.isfinite(o[key]).all()), key
    worst = _check_sampled(plan, batch, refs, fp32=False)
    _say(f"  worst block error {worst:.3e}")
    plan.close()


@pytest.mark.parametrize("defects_waves,adjoint_waves", [(None, None), (2, None), (1, None),
                                                         (1, 1), (2, 4)])
def test_mixed256_adjoint_plans(mixed, defects_waves, adjoint_waves):
    api = _api()
    batch, _ = mixed
    _say(f"mixed 256 fp64 adjoint plan, defects form {defects_waves}, "
         f"reverse sweep {adjoint_waves}")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=True,
                         defects_waves=defects_waves, adjoint_waves=adjoint_waves)
    g = plan.groups()
    if defects_waves is not None:
        assert all(x["defects_waves"] == defects_waves for x in g), g
    lams = _seeds(plan, 9)
    plan.run("adjoint", graph=True)
    torch.cuda.synchronize()
    picks = _traj_picks(batch, 4, seed=504)
    assert len(picks) >= 8
    worst = _check_adjoint_trajs(plan, batch, lams, picks)
    # the defects pass: d and F~ of the sampled trajectories against the oracle
    for t in picks[:3]:
        model, data, K = batch[t]
        ref = oracle.defects(model, data["X"], data["U"], data["s"], data["p"], K)
        for key in ("d", "xprop"):
            e = block_err(plan.out[t][key].cpu().numpy().T, ref[key], PHI64)
            assert e <= TOL64, (t, key, e)
    _say(f"  worst gradient block error {worst:.3e}")
    plan.close()


@pytest.mark.parametrize("defects_waves", [2, 1])
def test_defects_forms_checkpoints_match_single(defects_waves):
    """Both defects forms of a batch feed the reverse sweep the checkpoints of
    the single-trajectory cis_defects: the gradients of a plan forced to either
    form agree with cis_defects + cis_discretize_adjoint on each trajectory (the
    two forms sum the right-hand side in different orders, hence 1e-12), its d
    and F~ with the oracle, and its gradients with the oracle."""
    api = _api()
    batch = synth.mixed_batch(12, seed=21, N_range=(5, 14), K_range=(4, 16))
    batch = [(m, d, K) for m, d, K in batch]
    _say(f"defects form {defects_waves} vs single-trajectory checkpoints")
    trajs = _upload(batch, torch.float64)
    plan = api.BatchPlan(trajs, ("adjoint",), sched="grid", graph=False,
                         defects_waves=defects_waves)
    assert all(x["defects_waves"] == defects_waves for x in plan.groups())
    lams = _seeds(plan, 11)
    plan.run("adjoint")
    torch.cuda.synchronize()

    def rel(a, b):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0

    for i, t in enumerate(trajs):
        K = t["K"]
        C = max(c for c in range(1, 9) if K % c == 0)   # the plan's default spacing
        d = api.defects(t["cm"], t["X"], t["U"], t["s"], t["params"], K, ckpt_every=C)
        g = api.adjoint(t["cm"], t["X"], t["U"], t["s"], t["params"], K, d["ckpt"], C,
                        plan.out[i]["seed"])
        N = t["s"].shape[0]
        assert rel(plan.out[i]["gX"][:, :N + 1], g["gX"]) <= 1e-12, i
        assert rel(plan.out[i]["gs"], g["gs"]) <= 1e-12, i
        assert rel(plan.out[i]["gp"], g["gp"]) <= 1e-12, i
        if t["cm"].m:
            assert rel(plan.out[i]["gU"][:t["cm"].m, :N + 1], g["gU"]) <= 1e-12, i
        model, data, _ = batch[i]
        ref = oracle.defects(model, data["X"], data["U"], data["s"], data["p"], K)
        for key in ("d", "xprop"):
            e = block_err(plan.out[i][key].cpu().numpy().T, ref[key], PHI64)
            assert e <= TOL64, (i, key, e)
    _check_adjoint_trajs(plan, batch, lams, list(range(len(batch))))
    plan.close()
