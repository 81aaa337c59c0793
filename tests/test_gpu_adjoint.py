"""Reverse-mode kernel vs the oracle's reverse sweep, and through autograd (GPU).

Bar: per-block error <= 1e-10 (phi = 1e-3) for gX, gU, gs and gp against
oracle.adjoint on the same inputs; dJ/de is exactly 0; central finite
differences of the merit (h = 1e-6 relative) agree to 1e-6.
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


def _dev_inputs(api, data, dev):
    X = api.to_device_soa(data["X"], dev)
    U = api.to_device_soa(data["U"], dev)
    s = torch.tensor(data["s"], device=dev)
    p = torch.tensor(data["p"], device=dev)
    return X, U, s, p


def _vec_err(g, o):
    g = np.asarray(g, dtype=np.float64).reshape(1, -1)
    o = np.asarray(o, dtype=np.float64).reshape(1, -1)
    return block_err(g, o, PHI64)


def run_adjoint(model, data, K, C, lam):
    from paper_2604_09993_amd import api
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X, U, s, p = _dev_inputs(api, data, dev)
    fw = api.defects(cm, X, U, s, p, K, ckpt_every=C)
    seed = torch.tensor(np.ascontiguousarray(lam.T), device=dev)
    g = api.adjoint(cm, X, U, s, p, K, fw["ckpt"], C, seed)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


def check(model, data, K, C, lam):
    g = run_adjoint(model, data, K, C, lam)
    ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, lam)
    errs = {"gX": block_err(g["gX"].T, ref["gX"], PHI64),
            "gU": block_err(g["gU"].T, ref["gU"], PHI64) if model.m else 0.0,
            "gs": _vec_err(g["gs"], ref["gs"]),
            "gp": _vec_err(g["gp"], ref["gp"])}
    assert g["gp"][1] == 0.0
    assert np.all(g["gX"][:, -1] == 0.0)
    bad = {k: e for k, e in errs.items() if not e <= TOL64}
    assert not bad, errs
    return g


CASES = [("free1", 3, 4, 2), ("point1", 3, 4, 4), ("hopper", 4, 6, 3), ("biped5", 3, 4, 1),
         ("cheetah7", 4, 6, 2), ("quad13", 2, 4, 4)]


@pytest.mark.parametrize("name,N,K,C", CASES)
def test_adjoint_matches_oracle(name, N, K, C):
    """Intervals of ~0.02 s, as in the configurations.  (With 0.1-0.2 s intervals
    the light quad13 links tumble and a 1-ulp input perturbation already moves
    the oracle's own gradients by ~2.5e-10, above the 1e-10 bar.)"""
    _say(f"[gpu] adjoint {name} N={N} K={K} C={C} seed=200")
    rng = np.random.default_rng(200)
    model = synth.MODEL_MAKERS[name](rng)
    data = synth.gen_nodes(model, N, rng, T=0.02 * N)
    lam = rng.normal(size=(N, model.nx))
    check(model, data, K, C, lam)


def test_adjoint_long_segment_replay():
    """ckpt_every = K = 20 > the 8-substep LDS chunk: the segment is replayed in chunks."""
    _say("[gpu] adjoint hopper N=3 K=20 C=20 (chunked replay)")
    rng = np.random.default_rng(201)
    model = synth.make_hopper(rng)
    data = synth.gen_nodes(model, 3, rng, T=0.3)
    lam = rng.normal(size=(3, model.nx))
    check(model, data, 20, 20, lam)
    check(model, data, 20, 10, lam)


def _merit_seed(model, d):
    """R15 merit J = 1/2 sum ||d_k||^2 + sum_k sum_i (F~_k - X_k)_{n+i}: dJ/dF~_k = d_k + [0; 1]."""
    lam = d.copy()
    lam[:, model.n:] += 1.0
    return lam


def test_workload_cheetah7_ckpt5_merit_gradients_via_autograd():
    """Cheetah N=50, K=20, checkpoints every 5 substeps, merit through torch.autograd."""
    from paper_2604_09993_amd import api
    _say("[gpu] workload cheetah7 N=50 K=20 C=5: adjoint via autograd")
    model, data, K = synth.make_workload("cheetah7_N50_K20_ckpt5")
    C = synth.WORKLOADS["cheetah7_N50_K20_ckpt5"]["ckpt"]
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X, U, s, p = _dev_inputs(api, data, dev)
    X.requires_grad_(True)
    U.requires_grad_(True)
    s.requires_grad_(True)
    p.requires_grad_(True)
    N = data["s"].shape[0]
    F = api.CisDefects.apply(X, U, s, p, cm, K, C)
    d = F - X[:, 1:N + 1]
    J = 0.5 * (d[:model.n] ** 2).sum() + 0.5 * (d[model.n:] ** 2).sum() + \
        (F[model.n:] - X[model.n:, :N]).sum()
    J.backward()
    torch.cuda.synchronize()
    # reference: oracle reverse sweep with dJ/dF~ = d + [0;1], plus the explicit X terms
    ref_d = oracle.defects(model, data["X"], data["U"], data["s"], data["p"], K)["d"]
    lam = _merit_seed(model, ref_d)
    ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, lam)
    gX = ref["gX"].copy()
    gX[1:] -= ref_d                      # d_k = F~_k - X_{k+1}
    gX[:N, model.n:] -= 1.0              # - X_k in the increment term
    errs = {"gX": block_err(X.grad.t().cpu().numpy(), gX, PHI64),
            "gU": block_err(U.grad.t().cpu().numpy(), ref["gU"], PHI64),
            "gs": _vec_err(s.grad.cpu().numpy(), ref["gs"]),
            "gp": _vec_err(p.grad.cpu().numpy(), ref["gp"])}
    assert all(e <= TOL64 for e in errs.values()), errs
    assert p.grad[1].item() == 0.0
    # FD of the merit w.r.t. mu and two masses on the GPU defects path (h = 1e-6 relative)
    def merit(pp):
        with torch.no_grad():
            out = api.defects(cm, X.detach(), U.detach(), s.detach(), pp, K)
            dd = out["d"]
            inc = out["xprop"][model.n:] - X.detach()[model.n:, :N]
            return float(0.5 * (dd ** 2).sum() + inc.sum())
    # central-difference error bound: 1e-6 relative (truncation at h = 1e-6
    # relative) plus the rounding of the merit itself, ~ eps |J| / h.
    J0 = merit(p.detach())
    for c in (0, 2, 5):
        h = 1e-6 * abs(float(p.detach()[c]))
        pp, pm = p.detach().clone(), p.detach().clone()
        pp[c] += h
        pm[c] -= h
        fd = (merit(pp) - merit(pm)) / (2 * h)
        g = float(p.grad[c])
        tol = 1e-6 * max(1.0, abs(g)) + 64 * 2.2e-16 * abs(J0) / h
        assert abs(fd - g) <= tol, (c, fd, g, tol, J0)


def test_adjoint_contraction_of_forward_sensitivities():
    """gX = A^T lam, gs = S^T lam and gU = B-^T lam_k + B+^T lam_k-1 from the GPU forward kernel."""
    from paper_2604_09993_amd import api
    _say("[gpu] adjoint vs forward contraction biped5 N=5 K=4")
    rng = np.random.default_rng(202)
    model = synth.make_biped5(rng)
    data = synth.gen_nodes(model, 5, rng, T=0.5)
    lam = rng.normal(size=(5, model.nx))
    g = run_adjoint(model, data, 4, 2, lam)
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X, U, s, p = _dev_inputs(api, data, dev)
    fw = api.as_interval_major(api.discretize(cm, X, U, s, p, 4))
    A = fw["A"].cpu().numpy()
    S = fw["S"].cpu().numpy()
    Bm = fw["Bm"].cpu().numpy()
    Bp = fw["Bp"].cpu().numpy()
    gX = np.einsum("kij,ki->kj", A, lam)
    gU = np.zeros((6, model.m))
    gU[:5] += np.einsum("kij,ki->kj", Bm, lam)
    gU[1:] += np.einsum("kij,ki->kj", Bp, lam)
    assert block_err(g["gX"].T[:5], gX, PHI64) <= 1e-12 * 100
    assert block_err(g["gU"].T, gU, PHI64) <= 1e-12 * 100
    assert _vec_err(g["gs"], np.einsum("ki,ki->k", S, lam)) <= 1e-12 * 100


def _merit_autograd(api, cm, model, data, K, C, dev):
    """Gradients of the R15 merit through CisDefects (reverse-mode kernel)."""
    X, U, s, p = _dev_inputs(api, data, dev)
    for t in (X, U, s, p):
        t.requires_grad_(True)
    N = data["s"].shape[0]
    F = api.CisDefects.apply(X, U, s, p, cm, K, C)
    d = F - X[:, 1:N + 1]
    J = 0.5 * (d ** 2).sum() + (F[model.n:] - X[model.n:, :N]).sum()
    J.backward()
    torch.cuda.synchronize()
    return X, U, s, p


def test_merit_gradients_match_central_differences_of_nodes_controls_dilations():
    """Central differences (h = 1e-6 relative, absolute 1e-6 for entries below
    one) of the merit, evaluated with the GPU defects kernel, against the
    reverse-mode gradients on 10 sampled entries each of X, U and s
    (cheetah7 N = 50, K = 20, checkpoints every 5 substeps)."""
    from paper_2604_09993_amd import api
    _say("[gpu] merit FD on X, U, s: cheetah7 N=50 K=20 C=5, 10 entries each, seed 205")
    model, data, K = synth.make_workload("cheetah7_N50_K20_ckpt5")
    C = synth.WORKLOADS["cheetah7_N50_K20_ckpt5"]["ckpt"]
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X, U, s, p = _merit_autograd(api, cm, model, data, K, C, dev)
    N = data["s"].shape[0]

    def merit(Xv, Uv, sv):
        with torch.no_grad():
            out = api.defects(cm, Xv, Uv, sv, p.detach(), K)
            inc = out["xprop"][model.n:] - Xv[model.n:, :N]
            return float(0.5 * (out["d"] ** 2).sum() + inc.sum())

    Xd, Ud, sd = X.detach(), U.detach(), s.detach()
    J0 = merit(Xd, Ud, sd)
    rng = np.random.default_rng(205)
    picks = ([("X", (int(rng.integers(model.nx)), int(rng.integers(N + 1)))) for _ in range(10)] +
             [("U", (int(rng.integers(model.m)), int(rng.integers(N + 1)))) for _ in range(10)] +
             [("s", (int(rng.integers(N)),)) for _ in range(10)])
    grads = {"X": X.grad, "U": U.grad, "s": s.grad}
    base = {"X": Xd, "U": Ud, "s": sd}
    worst = 0.0
    for name, idx in picks:
        v = float(base[name][idx])
        h = 1e-6 * max(1.0, abs(v))
        args_p = {k: t.clone() for k, t in base.items()}
        args_m = {k: t.clone() for k, t in base.items()}
        args_p[name][idx] += h
        args_m[name][idx] -= h
        fd = (merit(args_p["X"], args_p["U"], args_p["s"]) -
              merit(args_m["X"], args_m["U"], args_m["s"])) / (2 * h)
        g = float(grads[name][idx])
        tol = 1e-6 * max(1.0, abs(g)) + 64 * 2.2e-16 * abs(J0) / h
        assert abs(fd - g) <= tol, (name, idx, fd, g, tol)
        worst = max(worst, abs(fd - g) / max(1.0, abs(g)))
    _say(f"  worst |FD - grad| / max(1, |grad|) = {worst:.2e}")


def test_adjoint_bitwise_reproducible():
    """Run-to-run: the reverse sweep and its reductions in fixed order give
    bit-identical gX, gU, gs and gp on repeated calls, single trajectory and
    batch plan."""
    from paper_2604_09993_amd import api
    _say("[gpu] adjoint run-to-run bitwise: cheetah7 N=50 K=20 C=5; mixed plan of 6 trajectories")
    model, data, K = synth.make_workload("cheetah7_N50_K20_ckpt5")
    C = synth.WORKLOADS["cheetah7_N50_K20_ckpt5"]["ckpt"]
    dev = torch.device("cuda:0")
    cm = api.CisModel(model)
    X, U, s, p = _dev_inputs(api, data, dev)
    fw = api.defects(cm, X, U, s, p, K, ckpt_every=C)
    seed = torch.randn(fw["d"].shape, generator=torch.Generator().manual_seed(5),
                       dtype=torch.float64).to(dev)
    runs = [api.adjoint(cm, X, U, s, p, K, fw["ckpt"], C, seed) for _ in range(3)]
    torch.cuda.synchronize()
    for r in runs[1:]:
        for key in ("gX", "gU", "gs", "gp"):
            assert torch.equal(r[key], runs[0][key]), key
    batch = synth.mixed_batch()[:6]
    trajs = []
    for m_, d_, k_ in batch:
        c_ = api.CisModel(m_)
        Nt = d_["s"].shape[0]
        trajs.append(dict(cm=c_, K=k_, X=api.to_device_soa(d_["X"], dev, ld=Nt + 1),
                          U=api.to_device_soa(d_["U"], dev, ld=Nt + 1),
                          s=torch.tensor(d_["s"], device=dev),
                          params=torch.tensor(d_["p"], device=dev)))
    plan = api.BatchPlan(trajs, ("adjoint",), sched="tune", graph=True)
    gen = torch.Generator().manual_seed(6)
    for o in plan.out:
        o["seed"].copy_(torch.randn(o["seed"].shape, generator=gen, dtype=torch.float64))
    outs = []
    for _ in range(3):
        plan.run("adjoint", graph=True)
        torch.cuda.synchronize()
        outs.append([{k: o[k].clone() for k in ("gX", "gU", "gs", "gp")} for o in plan.out])
    for o in outs[1:]:
        for a_, b_ in zip(o, outs[0]):
            for key in a_:
                assert torch.equal(a_[key], b_[key]), key
    plan.close()
