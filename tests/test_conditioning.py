"""Conditioning of the discrete map at the parity test inputs (CPU only).

The GPU parity tests compare against the FP64 oracle at 1e-10 (FP64) and at
1e-4 normwise (FP32, oracle on the FP32-rounded inputs).  Those bars only
mean something where the map itself is well conditioned: a computation in
another rounding order is, at best, the exact map of inputs perturbed at the
level of one rounding.  These tests measure that sensitivity with the oracle
alone, at the inputs the GPU tests use and at the longer intervals (whole
trajectory T = 1 s over N = 2 intervals, and 0.1 s intervals for the adjoint)
where the quad13 cases first ran:

* at the long intervals a perturbation of every input by one unit in the last
  place (FP64) or by one FP32 rounding moves the oracle itself by more than the
  bar, so no implementation with a different rounding order can be held to
  the bar there;
* at the intervals of the configurations (about 0.02 s) the same perturbation
  moves it far below the bar, so the GPU tests there are meaningful.

The perturbation multiplies every nonzero input entry by (1 + sign * u) with
random signs, u = 2^-53 (FP64) or 2^-24 (FP32).
"""
import numpy as np

import oracle
from paper_2604_09993_amd import synth
from parity import PHI32, PHI64, TOL32, TOL64, block_err

KEYS = ("A", "Bm", "Bp", "S", "d", "xprop")


def _perturb(data, u, seed):
    r = np.random.default_rng(seed)
    out = {}
    for key in ("X", "U", "s", "p"):
        a = np.asarray(data[key], dtype=np.float64)
        sign = r.choice([-1.0, 1.0], size=a.shape)
        out[key] = a * (1.0 + sign * u)
    out["p"][1] = data["p"][1]
    return out


def _r32(data):
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in data.items()}


def _fwd_spread(model, data, K, u, phi):
    ref = oracle.discretize(model, data["X"], data["U"], data["s"], data["p"], K)
    worst = 0.0
    for seed in range(3):
        pd = _perturb(data, u, seed)
        o = oracle.discretize(model, pd["X"], pd["U"], pd["s"], pd["p"], K)
        worst = max(worst, max(block_err(o[k], ref[k], phi) for k in KEYS))
    return worst


def _quad13_fp32_case(T):
    # the model and nodes of the quad13 FP32 parity case (seed 101, N = 2, K = 2)
    rng = np.random.default_rng(101)
    model = synth.make_quad13(rng)
    return model, _r32(synth.gen_nodes(model, 2, rng, T=T))


def test_quad13_fp32_long_intervals_ill_conditioned():
    model, data = _quad13_fp32_case(T=1.0)
    spread = _fwd_spread(model, data, 2, 2.0 ** -24, PHI32)
    assert spread > TOL32, spread


def test_quad13_fp32_configuration_intervals_well_conditioned():
    model, data = _quad13_fp32_case(T=0.04)
    spread = _fwd_spread(model, data, 2, 2.0 ** -24, PHI32)
    assert spread < 0.1 * TOL32, spread


def _adj_spread(model, data, K, lam, u):
    ref = oracle.adjoint(model, data["X"], data["U"], data["s"], data["p"], K, lam)
    worst = 0.0
    for seed in range(3):
        pd = _perturb(data, u, seed)
        o = oracle.adjoint(model, pd["X"], pd["U"], pd["s"], pd["p"], K, lam)
        for key in ("gX", "gU"):
            worst = max(worst, block_err(o[key], ref[key], PHI64))
        for key in ("gs", "gp"):
            worst = max(worst, block_err(o[key].reshape(1, -1), ref[key].reshape(1, -1), PHI64))
    return worst


def _quad13_adjoint_case(T):
    # the model, nodes and seed of the quad13 adjoint parity case (seed 200, N = 2, K = 4)
    rng = np.random.default_rng(200)
    model = synth.make_quad13(rng)
    data = synth.gen_nodes(model, 2, rng, T=T)
    lam = rng.normal(size=(2, model.nx))
    return model, data, lam


def test_quad13_adjoint_long_intervals_ill_conditioned():
    for T in (1.0, 0.2):
        model, data, lam = _quad13_adjoint_case(T)
        spread = _adj_spread(model, data, 4, lam, 2.0 ** -53)
        assert spread > TOL64, (T, spread)


def test_quad13_adjoint_configuration_intervals_well_conditioned():
    model, data, lam = _quad13_adjoint_case(T=0.04)
    spread = _adj_spread(model, data, 4, lam, 2.0 ** -53)
    assert spread < 0.1 * TOL64, spread


def _quad13_split_case(T):
    # the model and nodes of the quad13 FP64 case of the split-form tests
    # (seed 300, N = 3, K = 2)
    rng = np.random.default_rng(300)
    model = synth.make_quad13(rng)
    data = synth.gen_nodes(model, 3, rng) if T is None else synth.gen_nodes(model, 3, rng, T=T)
    return model, data


def test_quad13_split_case_conditioning():
    """With the default 1 s over 3 intervals (0.26-0.37 s each, K = 2) a one-ulp
    input perturbation moves the oracle by the order of the FP64 bar; at the
    configurations' 0.02 s intervals by less than a thousandth of it."""
    model, data = _quad13_split_case(None)
    long_spread = _fwd_spread(model, data, 2, 2.0 ** -53, PHI64)
    assert long_spread > 0.3 * TOL64, long_spread
    model, data = _quad13_split_case(0.06)
    short_spread = _fwd_spread(model, data, 2, 2.0 ** -53, PHI64)
    assert short_spread < 1e-3 * TOL64, short_spread
