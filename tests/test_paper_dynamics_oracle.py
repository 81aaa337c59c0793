"""Pins of the paper-faithful dynamics oracle (CPU only).

oracle.paper_dynamics (joint forces eliminated at the acceleration level,
controls (tau, phi_t, phi_n, gamma), four integral states per contact and one
violation state) is checked against things other than itself: the already
pinned base oracle fed the eliminated joint forces as controls, the joint
constraints and their velocity form staying satisfied along integrated
trajectories, energy and momentum conservation where the physics fixes them,
the kinematic meaning of lambda_c, closed forms of rho_c and the violation
integrand, central differences of the right-hand side and of the discrete
map, and the interval semigroup.
"""
import numpy as np
import pytest

import oracle
from oracle import paper_dynamics as pd
from paper_2604_09993_amd import synth


def _model(name, seed, **kw):
    rng = np.random.default_rng(seed)
    if name == "biped3s":
        return synth.legged_model("biped3", 2, 1, rng, terrain="sinusoid", **kw), rng
    if name == "cheetah7":
        return synth.legged_model("cheetah7", 2, 3, rng, **kw), rng
    if name == "quad13":
        return synth.legged_model("quad13", 4, 3, rng, (0.1, 0.5), (1.0, 7.0), 20.0,
                                  "horizontal", hip_x=[-0.5, -1.0 / 6.0, 1.0 / 6.0, 0.5],
                                  **kw), rng
    if name == "hopper":
        return synth.legged_model("hopper", 1, 2, rng, **kw), rng
    raise KeyError(name)


def _joint_residual(model, q):
    """h(q) and the anchors' world positions (the constraint as defined)."""
    nb = model.nb
    q = q.reshape(nb, 3)
    out = []
    for j in range(model.nj):
        p, c = int(model.joint_parent[j]), int(model.joint_child[j])
        rot = lambda th: np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        out.append(q[p, :2] + rot(q[p, 2]) @ model.anchor_parent[j]
                   - q[c, :2] - rot(q[c, 2]) @ model.anchor_child[j])
    return np.array(out).reshape(-1)


def _consistent_state(model, rng, scale=0.5):
    """Closed joints and joint-consistent velocities (v projected on the null
    space of grad h, computed by differencing h)."""
    d = synth.gen_paper_nodes(model, 1, rng)
    x = d["X"][0].copy()
    nq = 3 * model.nb
    q = x[:nq]
    G = np.zeros((2 * model.nj, nq))
    for k in range(nq):
        e = np.zeros(nq)
        e[k] = 1e-7
        G[:, k] = (_joint_residual(model, q + e) - _joint_residual(model, q - e)) / 2e-7
    v = rng.normal(0.0, scale, size=nq)
    v -= np.linalg.pinv(G) @ (G @ v)
    x[nq:2 * nq] = v
    return x, d


def _rk4(model, x, u, p, dt, steps):
    for _ in range(steps):
        k1 = pd.rhs(model, x, u, p)
        k2 = pd.rhs(model, x + 0.5 * dt * k1, u, p)
        k3 = pd.rhs(model, x + 0.5 * dt * k2, u, p)
        k4 = pd.rhs(model, x + dt * k3, u, p)
        x = x + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


@pytest.mark.parametrize("name", ["hopper", "biped3s", "cheetah7", "quad13"])
def test_accelerations_equal_the_base_model_with_the_eliminated_forces(name):
    """The base oracle takes joint forces and split friction as controls; fed
    lambda of the elimination and (lam_n, lam_t+, lam_t-) = (phi_n, phi_t, 0)
    it must produce the same accelerations."""
    model, rng = _model(name, 30)
    d = synth.gen_paper_nodes(model, 1, rng)
    x, u, p = d["X"][0], d["U"][0], d["p"]
    nb, nj, nc = model.nb, model.nj, model.nc
    lam = pd.joint_forces(model, x, u, p)
    ub = np.zeros(3 * nj + 3 * nc)
    ub[:nj] = u[:nj]
    ub[nj:3 * nj] = lam
    for i in range(nc):
        ub[3 * nj + 3 * i] = u[nj + 3 * i + 1]
        ub[3 * nj + 3 * i + 1] = u[nj + 3 * i]
    xb = np.zeros(6 * nb + nc + 1)
    xb[:6 * nb] = x[:6 * nb]
    F = oracle.rhs_jac(model, xb, ub, ub, p)[0]
    got = pd.rhs(model, x, u, p)
    np.testing.assert_allclose(got[:6 * nb], F[:6 * nb], rtol=1e-12,
                               atol=1e-12 * np.max(np.abs(F[:6 * nb])))


@pytest.mark.parametrize("name", ["hopper", "cheetah7", "quad13"])
def test_joint_constraints_stay_satisfied_along_trajectories(name):
    """From closed joints with consistent velocities, the eliminated forces keep
    h(q) = 0 and grad h v = 0 (drift only at the integration error)."""
    model, rng = _model(name, 31)
    x, d = _consistent_state(model, rng)
    u = d["U"][0]
    nq = 3 * model.nb
    h0 = _joint_residual(model, x[:nq])
    assert np.max(np.abs(h0)) < 1e-12
    xT = _rk4(model, x, u, d["p"], 2e-4, 250)
    assert np.max(np.abs(_joint_residual(model, xT[:nq]))) < 1e-9
    # velocity form, by differencing h along v
    eps = 1e-6
    hv = (_joint_residual(model, xT[:nq] + eps * xT[nq:2 * nq])
          - _joint_residual(model, xT[:nq] - eps * xT[nq:2 * nq])) / (2 * eps)
    assert np.max(np.abs(hv)) < 1e-7


def test_energy_is_conserved_without_dissipation():
    """No damping, no contact forces, no torques: kinetic + spring + gravity
    energy is constant (the joint forces do no work)."""
    model, rng = _model("cheetah7", 32, damping=0.0)
    x, d = _consistent_state(model, rng)
    u = np.zeros(model.nj + 3 * model.nc)
    p = d["p"]
    nb = model.nb
    m = p[2:]
    inertia = m * model.link_length ** 2 / 12.0

    def energy(x):
        q = x[:3 * nb].reshape(nb, 3)
        v = x[3 * nb:6 * nb].reshape(nb, 3)
        ke = 0.5 * np.sum(m * (v[:, 0] ** 2 + v[:, 1] ** 2) + inertia * v[:, 2] ** 2)
        pe = np.sum(m * model.gravity * q[:, 1])
        for j in range(model.nj):
            pe += 0.5 * model.stiffness[j] * (q[model.joint_child[j], 2] - q[model.joint_parent[j], 2]) ** 2
        return ke + pe
    E0 = energy(x)
    xT = _rk4(model, x, u, p, 2e-4, 250)
    assert abs(energy(xT) - E0) < 1e-9 * max(1.0, abs(E0))


def test_momentum_is_conserved_without_external_forces():
    model, rng = _model("quad13", 33, gravity=0.0)
    x, d = _consistent_state(model, rng)
    u = d["U"][0].copy()
    nj = model.nj
    u[nj:] = 0.0          # no contact forces; joint torques stay (internal)
    p = d["p"]
    nb = model.nb
    m = p[2:]
    inertia = m * model.link_length ** 2 / 12.0

    def momenta(x):
        q = x[:3 * nb].reshape(nb, 3)
        v = x[3 * nb:6 * nb].reshape(nb, 3)
        lin = (m[:, None] * v[:, :2]).sum(axis=0)
        ang = np.sum(inertia * v[:, 2] + m * (q[:, 0] * v[:, 1] - q[:, 1] * v[:, 0]))
        return lin, ang
    l0, a0 = momenta(x)
    xT = _rk4(model, x, u, p, 2e-4, 200)
    l1, a1 = momenta(xT)
    assert np.max(np.abs(l1 - l0)) < 1e-9 * max(1.0, np.max(np.abs(l0)))
    assert abs(a1 - a0) < 1e-9 * max(1.0, abs(a0))


def test_integrands_have_their_meaning():
    """lambda_c - gamma phi_t / sqrt(phi_t^2 + 1) is the tangential velocity of
    the contact point (central difference of its position along v on flat
    ground); rho_c at phi_t = 0 is |mu phi_n|_s; the violation integrand is 0
    at a feasible point and |phi_n|_s when only phi_n < 0."""
    model, rng = _model("hopper", 34)
    d = synth.gen_paper_nodes(model, 1, rng)
    x, u, p = d["X"][0].copy(), d["U"][0].copy(), d["p"]
    nb, nj = model.nb, model.nj
    b = int(model.contact_body[0])
    # lift the foot above the ground: sd > 0
    x[1:3 * nb:3] += 1.0
    f = pd.rhs(model, x, u, p)
    y = f[6 * nb:]
    pt, pn, gam = u[nj], u[nj + 1], u[nj + 2]

    def tip(xx):
        q = xx[:3 * nb].reshape(nb, 3)
        th = q[b, 2]
        r = model.contact_point[0]
        return q[b, :2] + np.array([np.cos(th) * r[0] - np.sin(th) * r[1],
                                    np.sin(th) * r[0] + np.cos(th) * r[1]])
    eps = 1e-6
    dx = np.zeros_like(x)
    dx[:3 * nb] = x[3 * nb:6 * nb]
    vt = (tip(x + eps * dx)[0] - tip(x - eps * dx)[0]) / (2 * eps)
    assert abs(y[1] - gam * pt / np.sqrt(pt * pt + 1.0) - vt) < 1e-8
    assert y[0] == pn and y[2] == gam
    # rho_c and the violation integrand
    u2 = u.copy()
    u2[nj] = 0.0
    y2 = pd.rhs(model, x, u2, p)[6 * nb:]
    mu = p[0]
    assert abs(y2[3] - (np.sqrt((mu * pn) ** 2 + 1.0) - 1.0)) < 1e-12
    assert y2[4] == 0.0
    u3 = u2.copy()
    u3[nj + 1] = -0.7
    y3 = pd.rhs(model, x, u3, p)[6 * nb:]
    rho3 = np.sqrt((mu * 0.7) ** 2 + 1.0) - 1.0   # |mu phi_n|_s >= 0 still
    assert rho3 >= 0.0
    assert abs(y3[4] - (np.sqrt(0.49 + 1.0) - 1.0)) < 1e-12
    # penetration: the foot 0.3 below flat ground, everything else feasible
    x4 = x.copy()
    x4[1:3 * nb:3] += -0.3 - tip(x)[1]
    y4 = pd.rhs(model, x4, u2, p)[6 * nb:]
    assert abs(y4[4] - (np.sqrt(0.09 + 1.0) - 1.0)) < 1e-12


@pytest.mark.parametrize("name", ["biped3s", "quad13"])
def test_rhs_jacobians_match_central_differences(name):
    model, rng = _model(name, 35)
    d = synth.gen_paper_nodes(model, 1, rng)
    x, u, p = d["X"][0], d["U"][0], d["p"]
    f, Jx, Ju = pd.rhs_jac(model, x, u, p)
    for j in range(x.size):
        h = 1e-6 * max(1.0, abs(x[j]))
        e = np.zeros_like(x)
        e[j] = h
        fd = (pd.rhs(model, x + e, u, p) - pd.rhs(model, x - e, u, p)) / (2 * h)
        assert np.max(np.abs(fd - Jx[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(Jx[:, j]))), j
    for j in range(u.size):
        h = 1e-6 * max(1.0, abs(u[j]))
        e = np.zeros_like(u)
        e[j] = h
        fd = (pd.rhs(model, x, u + e, p) - pd.rhs(model, x, u - e, p)) / (2 * h)
        assert np.max(np.abs(fd - Ju[:, j])) <= 1e-6 * max(1.0, np.max(np.abs(Ju[:, j]))), j
    n = 6 * model.nb
    assert np.all(Jx[:, n:] == 0.0)       # the integral states feed back into nothing


def test_discrete_sensitivities_are_central_differences_of_the_map():
    model, rng = _model("cheetah7", 36)
    d = synth.gen_paper_nodes(model, 1, rng, T=0.02)
    X, U, s, p = d["X"], d["U"], d["s"], d["p"]
    K = 2
    out = pd.discretize(model, X, U, s, p, K)

    def F(Xv=X[0], Uk=U[0], Uk1=U[1], sv=s[0]):
        return pd.integrate(model, Xv, Uk, Uk1, sv, p, K)["xf"]

    def check(fd, an):
        assert np.max(np.abs(fd - an)) <= 1e-6 * max(1.0, np.max(np.abs(an)))
    for j in rng.choice(X.shape[1], size=8, replace=False):
        h = 1e-6 * max(1.0, abs(X[0, j]))
        e = np.zeros(X.shape[1])
        e[j] = h
        check((F(Xv=X[0] + e) - F(Xv=X[0] - e)) / (2 * h), out["A"][0][:, j])
    for j in rng.choice(U.shape[1], size=6, replace=False):
        h = 1e-6 * max(1.0, abs(U[0, j]))
        e = np.zeros(U.shape[1])
        e[j] = h
        check((F(Uk=U[0] + e) - F(Uk=U[0] - e)) / (2 * h), out["Bm"][0][:, j])
        check((F(Uk1=U[1] + e) - F(Uk1=U[1] - e)) / (2 * h), out["Bp"][0][:, j])
    h = 1e-7
    check((F(sv=s[0] + h) - F(sv=s[0] - h)) / (2 * h), out["S"][0])
    np.testing.assert_array_equal(out["d"][0], out["xprop"][0] - X[1])


def test_semigroup_and_chain_rule():
    model, rng = _model("biped3s", 37)
    d = synth.gen_paper_nodes(model, 1, rng, T=0.02)
    X, U, s, p = d["X"], d["U"], d["s"], d["p"]
    full = pd.integrate(model, X[0], U[0], U[1], s[0], p, 2)
    h1 = pd.integrate(model, X[0], U[0], U[1], s[0], p, 1, tau0=0.0, tau1=0.5)
    h2 = pd.integrate(model, h1["xf"], U[0], U[1], s[0], p, 1, tau0=0.5, tau1=1.0)
    np.testing.assert_allclose(h2["xf"], full["xf"], rtol=0, atol=1e-13)
    P2 = h2["Phi"]
    for key, comp in (("Phi", P2 @ h1["Phi"]), ("Bm", P2 @ h1["Bm"] + h2["Bm"]),
                      ("Bp", P2 @ h1["Bp"] + h2["Bp"]), ("S", P2 @ h1["S"] + h2["S"])):
        scale = max(1.0, np.max(np.abs(full[key])))
        assert np.max(np.abs(comp - full[key])) <= 1e-12 * scale, key
