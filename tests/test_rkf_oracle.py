"""Pins of the Runge-Kutta-Fehlberg oracle (CPU only).

The Fehlberg transcription of the oracle (explicit Runge-Kutta with the 4(5)
pair, fourth-order solution propagated, embedded estimate from the fifth) is
checked against things other than itself: the order conditions of rooted
trees up to order 5 on its tableau, the already pinned RK4 oracle (the same
generic code fed the classical tableau), observed convergence orders, the
exact ballistic solution, the interval semigroup and the chain rule of the
sensitivities, and central differences of its own discrete map.
"""
import numpy as np
import pytest

import oracle
from paper_2604_09993_amd import synth

RK4_C = np.array([0.0, 0.5, 0.5, 1.0])
RK4_A = np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]])
RK4_B = np.array([1.0, 2.0, 2.0, 1.0]) / 6.0


def _order_conditions(b, A, c):
    """Residuals of the order conditions of the rooted trees with 1..5 nodes."""
    Ac = A @ c
    return [
        (b.sum(), 1.0),
        (b @ c, 1 / 2),
        (b @ c**2, 1 / 3), (b @ Ac, 1 / 6),
        (b @ c**3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ (A @ c**2), 1 / 12), (b @ (A @ Ac), 1 / 24),
        (b @ c**4, 1 / 5), (b @ (c**2 * Ac), 1 / 10), (b @ (c * (A @ c**2)), 1 / 15),
        (b @ (c * (A @ Ac)), 1 / 30), (b @ (Ac**2), 1 / 20), (b @ (A @ c**3), 1 / 20),
        (b @ (A @ (c * Ac)), 1 / 40), (b @ (A @ (A @ c**2)), 1 / 60),
        (b @ (A @ (A @ Ac)), 1 / 120),
    ]


def test_fehlberg_tableau_is_a_4_5_pair():
    c, a, b, bh = oracle.rkf_tableau()
    assert np.all(np.triu(a) == 0.0)                       # explicit
    np.testing.assert_allclose(a.sum(axis=1), c, rtol=0, atol=1e-15)
    conds_b = _order_conditions(b, a, c)
    conds_bh = _order_conditions(bh, a, c)
    for got, want in conds_b[:8]:                          # order 4: trees with <= 4 nodes
        assert abs(got - want) <= 1e-14, (got, want)
    assert max(abs(g - w) for g, w in conds_b[8:]) > 1e-4  # and not order 5
    for got, want in conds_bh:                             # order 5: all 17 trees
        assert abs(got - want) <= 1e-14, (got, want)
    assert b[5] == 0.0 and b[1] == 0.0 and bh[1] == 0.0   # K2 enters no solution


def _interval(name, seed, airborne=False, T=0.04):
    rng = np.random.default_rng(seed)
    model = synth.MODEL_MAKERS[name](rng)
    d = synth.gen_nodes(model, 2, rng, T=T)
    X = d["X"].copy()
    if airborne:   # every contact well above the ground: a smooth right-hand side
        nb = model.nb
        X[:, 1:3 * nb:3] += 1.0
    return model, X, d["U"], d["s"], d["p"]


def test_generic_stages_with_the_classical_tableau_reproduce_the_rk4_oracle():
    model, X, U, s, p = _interval("cheetah7", 20)
    ref = oracle.integrate(model, X[0], U[0], U[1], s[0], p, 3)
    got = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 3, RK4_C, RK4_A, RK4_B)
    for k in ("xf", "Phi", "Bm", "Bp", "S"):
        scale = max(1.0, np.max(np.abs(ref[k])))
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-13 * scale, k


def test_rkf_converges_with_order_four_and_the_estimate_with_order_five():
    model, X, U, s, p = _interval("hopper", 21, airborne=True, T=0.02)
    c, a, b, bh = oracle.rkf_tableau()
    exact = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 256, c, a, b)["xf"]
    errs, ests = [], []
    for K in (2, 4, 8):
        r = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, K, c, a, b, bh)
        errs.append(np.max(np.abs(r["xf"] - exact)))
        ests.append(r["err"])
    for e0, e1 in zip(errs, errs[1:]):
        assert 13.0 < e0 / e1 < 21.0, errs          # 2^4 = 16
    for e0, e1 in zip(ests, ests[1:]):
        assert 26.0 < e0 / e1 < 40.0, ests          # local error of one step, 2^5 = 32
    assert 0.0 < ests[-1]


def test_rkf_integrates_ballistic_motion_exactly():
    """A free body under gravity: q(tau) is quadratic in tau, which every
    method of order >= 2 integrates exactly (and the estimate vanishes)."""
    model, X, U, s, p = _interval("free1", 22)
    c, a, b, bh = oracle.rkf_tableau()
    r = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 3, c, a, b, bh)
    nb, g, S = model.nb, model.gravity, s[0]
    q0, v0 = X[0, :3 * nb], X[0, 3 * nb:6 * nb]
    acc = np.tile([0.0, -g, 0.0], nb)
    np.testing.assert_allclose(r["xf"][:3 * nb], q0 + S * v0 + 0.5 * S * S * acc, rtol=0,
                               atol=1e-14)
    np.testing.assert_allclose(r["xf"][3 * nb:6 * nb], v0 + S * acc, rtol=0, atol=1e-14)
    assert r["err"] <= 1e-15


def test_rkf_semigroup_and_chain_rule():
    """Two steps over [0, 1] are one step over [0, 1/2] then one over [1/2, 1];
    the sensitivities compose by the chain rule."""
    model, X, U, s, p = _interval("biped5", 23)
    c, a, b, _ = oracle.rkf_tableau()
    args = (model, X[0], U[0], U[1], s[0], p)
    full = oracle.integrate_erk(*args[:1], X[0], U[0], U[1], s[0], p, 2, c, a, b)
    h1 = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 1, c, a, b, tau0=0.0, tau1=0.5)
    h2 = oracle.integrate_erk(model, h1["xf"], U[0], U[1], s[0], p, 1, c, a, b, tau0=0.5,
                              tau1=1.0)
    np.testing.assert_allclose(h2["xf"], full["xf"], rtol=0, atol=1e-13)
    P2 = h2["Phi"]
    for key, comp in (("Phi", P2 @ h1["Phi"]), ("Bm", P2 @ h1["Bm"] + h2["Bm"]),
                      ("Bp", P2 @ h1["Bp"] + h2["Bp"]), ("S", P2 @ h1["S"] + h2["S"])):
        scale = max(1.0, np.max(np.abs(full[key])))
        assert np.max(np.abs(comp - full[key])) <= 1e-12 * scale, key


def test_rkf_sensitivities_are_central_differences_of_the_map():
    model, X, U, s, p = _interval("cheetah7", 24)
    K = 2
    out = oracle.discretize_rkf(model, X[:2], U[:2], s[:1], p, K)
    rng = np.random.default_rng(25)

    def F(Xv=None, Uk=None, Uk1=None, sv=None):
        XX = X[:2].copy()
        UU = U[:2].copy()
        if Xv is not None:
            XX[0] = Xv
        if Uk is not None:
            UU[0] = Uk
        if Uk1 is not None:
            UU[1] = Uk1
        ss = s[:1] if sv is None else np.array([sv])
        return oracle.discretize_rkf(model, XX, UU, ss, p, K)["xprop"][0]

    def check(fd, an):
        assert np.max(np.abs(fd - an)) <= 1e-6 * max(1.0, np.max(np.abs(an)))
    for j in rng.choice(model.nx, size=8, replace=False):
        h = 1e-6 * max(1.0, abs(X[0, j]))
        e = np.zeros(model.nx)
        e[j] = h
        check((F(Xv=X[0] + e) - F(Xv=X[0] - e)) / (2 * h), out["A"][0][:, j])
    for j in rng.choice(model.m, size=6, replace=False):
        h = 1e-6 * max(1.0, abs(U[0, j]))
        e = np.zeros(model.m)
        e[j] = h
        check((F(Uk=U[0] + e) - F(Uk=U[0] - e)) / (2 * h), out["Bm"][0][:, j])
        h = 1e-6 * max(1.0, abs(U[1, j]))
        e[j] = h
        check((F(Uk1=U[1] + e) - F(Uk1=U[1] - e)) / (2 * h), out["Bp"][0][:, j])
    h = 1e-7
    check((F(sv=s[0] + h) - F(sv=s[0] - h)) / (2 * h), out["S"][0])


def test_rkf_and_rk4_are_different_maps_with_the_same_limit():
    model, X, U, s, p = _interval("hopper", 26, airborne=True, T=0.02)
    c, a, b, _ = oracle.rkf_tableau()
    exact = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 256, c, a, b)["xf"]
    rkf = oracle.discretize_rkf(model, X[:2], U[:2], s[:1], p, 4)
    rk4 = oracle.discretize(model, X[:2], U[:2], s[:1], p, 4)
    gap = np.max(np.abs(rkf["xprop"][0] - rk4["xprop"][0]))
    assert gap > 1e-10
    assert np.max(np.abs(rk4["xprop"][0] - exact)) < 100 * gap
    assert np.max(np.abs(rkf["xprop"][0] - exact)) < 100 * gap
    # the defect is F~ - X_{k+1}, the integral-state columns of A are [0; I]
    np.testing.assert_array_equal(rkf["d"][0], rkf["xprop"][0] - X[1])
    n = model.n
    assert np.all(rkf["A"][0][:n, n:] == 0.0)
    assert np.array_equal(rkf["A"][0][n:, n:], np.eye(model.ny))


def test_discretize_rkf_is_the_pinned_tableau_interval_by_interval():
    """discretize_rkf propagates the tableau's fourth-order weights b and
    reports the largest embedded estimate (bh - b), interval by interval."""
    model, X, U, s, p = _interval("biped5", 27)
    c, a, b, bh = oracle.rkf_tableau()
    out = oracle.discretize_rkf(model, X, U, s, p, 3)
    for k in range(2):
        r = oracle.integrate_erk(model, X[k], U[k], U[k + 1], s[k], p, 3, c, a, b, bh)
        np.testing.assert_array_equal(out["xprop"][k], r["xf"])
        np.testing.assert_array_equal(out["A"][k], r["Phi"])
        np.testing.assert_array_equal(out["Bm"][k], r["Bm"])
        np.testing.assert_array_equal(out["Bp"][k], r["Bp"])
        np.testing.assert_array_equal(out["S"][k], r["S"])
        assert out["err"][k] == r["err"] > 0.0


def test_embedded_estimate_of_one_step_is_the_gap_between_the_two_solutions():
    """With one step the estimate is max |x5 - x4| over all augmented rows,
    x5 and x4 the results of propagating bh and b from the same start."""
    model, X, U, s, p = _interval("cheetah7", 31)   # largest gap entry negative
    c, a, b, bh = oracle.rkf_tableau()
    r = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 1, c, a, b, bh)
    x4 = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 1, c, a, b)["xf"]
    x5 = oracle.integrate_erk(model, X[0], U[0], U[1], s[0], p, 1, c, a, bh)["xf"]
    gap = np.max(np.abs(x5 - x4))
    assert gap > 0.0 and np.max(x5 - x4) < gap
    assert abs(r["err"] - gap) <= 1e-12 * gap + 1e-15
