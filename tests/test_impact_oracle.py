"""Pins of the impact-map oracle (CPU only).

Each pin compares oracle.impact with something other than itself: the
closed-form impact of a point mass (e = 0 and e = 1), the joint velocity
constraint after the impact, linear and angular momentum balance of the
impulses, the Fischer-Burmeister zero set, structural zeros, and central
finite differences of every Jacobian (the Jacobians themselves come from
complex-step differentiation).
"""
import numpy as np
import pytest

from oracle import impact
from paper_2604_09993_amd import synth


def _point_impact(e, vx=0.3, v0=1.7, om=0.4, mass_seed=0):
    rng = np.random.default_rng(mass_seed)
    model = synth.make_point_contact(rng)
    p = model.params(mu=0.8, e=e)
    m = p[2]
    xm = np.zeros(model.nx)
    xm[0:3] = [0.1, 0.0, 0.2]            # on the ground: sd = 0
    xm[3:6] = [vx, -v0, om]
    xp = xm.copy()
    xp[3:6] = [vx, e * v0, om]           # restitution law for a point mass
    Phi = np.array([0.0, m * (1.0 + e) * v0])
    Gam = np.array([0.25])
    return model, xp, xm, Phi, Gam, p


@pytest.mark.parametrize("e", [0.0, 1.0])
def test_point_mass_impact_closed_form(e):
    model, xp, xm, Phi, Gam, p = _point_impact(e)
    delta = 1e-3
    G = impact.G_tilde(model, xp, xm, Phi, p)
    assert np.max(np.abs(G)) <= 1e-14
    th = impact.theta(model, xp, xm, Phi, Gam, p, delta)
    pn, vx, v0 = Phi[1], 0.3, 1.7
    fb0 = pn - np.sqrt(pn * pn + delta)           # FB(Phi_n, 0): sd = 0 and w = 0
    rho = np.sqrt((0.8 * pn) ** 2 + 1.0) - 1.0    # |mu Phi_n|_s - ||0||_s
    want = [fb0, fb0, pn * vx - delta, -pn * vx - delta,
            0.25 + rho - np.sqrt(0.25 ** 2 + rho * rho + delta), -pn, 0.0, 0.0, -0.25, -rho]
    np.testing.assert_allclose(th, want, rtol=1e-14, atol=1e-14)
    # restitution enters only the elasticity row: dFB(Phi_n, w)/de = dFB/db * n.J v-
    lin = impact.linearize(model, xp, xm, Phi, Gam, p, delta)
    ie = 2 * model.nx + 3 * model.nc + 1
    dfb_db = 1.0 - 0.0 / np.sqrt(pn * pn + delta)
    assert abs(lin["JT"][0, 1, ie] - dfb_db * (-v0)) <= 1e-13
    assert abs(lin["JT"][0, 7, ie] - v0) <= 1e-13          # row -w
    assert np.all(lin["JG"][0, :, ie] == 0.0)
    other = np.delete(lin["JT"][0, :, ie], [1, 7])
    assert np.all(other == 0.0)


def _rand_case(name, seed, pose_sigma=1e-3):
    rng = np.random.default_rng(seed)
    if name == "biped3s":
        model = synth.legged_model("biped3", 2, 1, rng, terrain="sinusoid")
    else:
        model = synth.MODEL_MAKERS[name](rng)
    d = synth.gen_impact_nodes(model, 2, rng, pose_sigma=pose_sigma)
    return model, d


@pytest.mark.parametrize("name", ["hopper", "biped5", "cheetah7", "quad13"])
def test_joint_velocity_constraint_after_impact(name):
    model, d = _rand_case(name, 10)
    q = d["Xp"][0, :3 * model.nb].reshape(model.nb, 3)
    vm = d["Xm"][0, 3 * model.nb:6 * model.nb]
    v = impact.post_impact_velocity(model, q, vm, d["Phi"][0], d["p"])
    Jh = impact.joint_jacobian(model, q)
    assert np.max(np.abs(Jh @ v)) <= 1e-12 * max(1.0, np.max(np.abs(v)))


@pytest.mark.parametrize("name", ["hopper", "biped5", "cheetah7", "quad13"])
def test_momentum_balance_of_the_impulses(name):
    """Joint impulses are internal: the linear momentum jumps by the sum of the
    contact impulses, and (joints closed) the angular momentum about the
    origin by the sum of their moments."""
    model, d = _rand_case(name, 11, pose_sigma=0.0)
    nb = model.nb
    q = d["Xp"][0, :3 * nb].reshape(nb, 3)
    vm = d["Xm"][0, 3 * nb:6 * nb]
    p = d["p"]
    v = impact.post_impact_velocity(model, q, vm, d["Phi"][0], p)
    dv = (v - vm).reshape(nb, 3)
    m = p[2:]
    inertia = m * model.link_length ** 2 / 12.0
    lin = (m[:, None] * dv[:, :2]).sum(axis=0)
    ang = (inertia * dv[:, 2] + m * (q[:, 0] * dv[:, 1] - q[:, 1] * dv[:, 0])).sum()
    F_sum, M_sum = np.zeros(2), 0.0
    for i in range(model.nc):
        _, P = impact.contact_jacobian(model, q, i)
        _, n, t = impact._terrain(model, P)
        F = t * d["Phi"][0, 2 * i] + n * d["Phi"][0, 2 * i + 1]
        F_sum += F
        M_sum += P[0] * F[1] - P[1] * F[0]
    scale = max(1.0, np.max(np.abs(F_sum)))
    assert np.max(np.abs(lin - F_sum)) <= 1e-12 * scale
    assert abs(ang - M_sum) <= 1e-11 * max(1.0, abs(M_sum))


def test_fischer_burmeister_zero_set():
    tiny = 1e-20
    for a, b in [(0.0, 3.0), (2.5, 0.0), (0.0, 0.0)]:
        assert abs(impact.fb(a, b, tiny)) <= 1e-9
    for a, b in [(1.0, 2.0), (0.3, 0.4)]:
        assert impact.fb(a, b, tiny) >= 0.1 * min(a, b)
    # delta > 0 is a strict relaxation of the complementarity corner
    assert impact.fb(0.0, 0.0, 1e-2) < 0.0


@pytest.mark.parametrize("name", ["hopper", "biped3s", "cheetah7"])
def test_jacobians_match_central_differences(name):
    model, d = _rand_case(name, 12)
    delta = 1e-2
    lin = impact.linearize(model, d["Xp"][:1], d["Xm"][:1], d["Phi"][:1], d["Gamma"][:1],
                           d["p"], delta)
    z0 = np.concatenate([d["Xp"][0], d["Xm"][0], d["Phi"][0], d["Gamma"][0], d["p"]])
    for j in range(z0.size):
        h = 1e-6 * max(1.0, abs(z0[j]))
        zp, zm = z0.copy(), z0.copy()
        zp[j] += h
        zm[j] -= h
        gp, tp = impact._node_residuals(model, zp, delta)
        gm, tm = impact._node_residuals(model, zm, delta)
        fdg, fdt = (gp - gm) / (2 * h), (tp - tm) / (2 * h)
        for fd, an in ((fdg, lin["JG"][0, :, j]), (fdt, lin["JT"][0, :, j])):
            err = np.abs(fd - an) / np.maximum(1.0, np.abs(an))
            assert np.max(err) <= 1e-6, (j, np.max(err))


def test_structure_of_the_node_jacobians():
    """Pose and integral-state rows of G~ are [I | -I] exactly; Theta does not
    depend on the integral states or on the pre-impact pose; G~ does not
    depend on Gamma, mu or e."""
    model, d = _rand_case("cheetah7", 13)
    lin = impact.linearize(model, d["Xp"][:1], d["Xm"][:1], d["Phi"][:1], d["Gamma"][:1],
                           d["p"], 1e-2)
    nx, n, nq, nc = model.nx, model.n, 3 * model.nb, model.nc
    JG, JT = lin["JG"][0], lin["JT"][0]
    for r in list(range(nq)) + list(range(n, nx)):
        row = np.zeros(JG.shape[1])
        row[r] = 1.0
        row[nx + r] = -1.0
        assert np.array_equal(JG[r], row), r
    assert np.all(JT[:, n:nx] == 0.0)                 # y+
    assert np.all(JT[:, nx:nx + nq] == 0.0)           # q-
    assert np.all(JT[:, nx + n:2 * nx] == 0.0)        # y-
    g0 = 2 * nx + 2 * nc
    assert np.all(JG[:, g0:g0 + nc] == 0.0)           # Gamma
    assert np.all(JG[:, g0 + nc:g0 + nc + 2] == 0.0)  # mu, e


def test_psi_interval_increments():
    rng = np.random.default_rng(14)
    model = synth.make_cheetah7(rng)
    yk = rng.uniform(0, 1, size=model.ny)
    yk1 = yk + rng.uniform(0, 0.1, size=model.ny)
    out = impact.psi(model, yk, yk1, 1e-3, 1e-4)
    np.testing.assert_allclose(out[:model.nc], (yk1 - yk)[:model.nc] - 1e-3, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[model.nc:], (yk1 - yk)[model.nc:] - 1e-4, rtol=0, atol=1e-15)


def test_terrain_frame_on_the_sinusoid():
    """Contact frame of the sinusoidal ground: a surface point has sd = 0, the
    normal is a unit vector orthogonal to the surface tangent (1, H'(x)) and
    points up, [t n] is a rotation, and sd grows like the distance along n."""
    rng = np.random.default_rng(15)
    model = synth.legged_model("biped3", 2, 1, rng, terrain="sinusoid")
    A, kap = model.terrain_amplitude, model.terrain_wavenumber
    assert A > 0.0
    for x in rng.uniform(-2.0, 2.0, size=8):
        P = np.array([x, A * np.sin(kap * x)])
        sd, n, t = impact._terrain(model, P)
        assert abs(sd) <= 1e-15
        assert abs(n @ np.array([1.0, A * kap * np.cos(kap * x)])) <= 1e-15
        assert abs(n @ n - 1.0) <= 1e-15 and n[1] > 0.0
        assert abs(t[0] * n[1] - t[1] * n[0] - 1.0) <= 1e-15
        for h in (1e-3, -1e-3):
            sd_h, _, _ = impact._terrain(model, P + h * n)
            assert abs(sd_h - h) <= 10.0 * A * kap * kap * h * h


def test_point_mass_tangential_impulse_and_friction_sign():
    """Contact at the centre of mass on flat ground: the impulse (Phi_t, Phi_n)
    changes the linear velocity by (Phi_t, Phi_n) / m and leaves the spin.
    Maximal dissipation: with the post-impact sliding velocity v_t > 0 and the
    impulse on the cone boundary opposing it (Phi_t = -mu Phi_n), the
    stationarity bracket vanishes for a positive multiplier Gamma."""
    rng = np.random.default_rng(0)
    model = synth.make_point_contact(rng)
    mu = 0.8
    p = model.params(mu=mu, e=0.0)
    m = p[2]
    vm = np.array([0.5, -1.0, 0.3])
    pn = 2.0
    Phi = np.array([-mu * pn, pn])
    q = np.array([[0.0, 0.0, 0.7]])
    v = impact.post_impact_velocity(model, q, vm, Phi, p)
    np.testing.assert_allclose(v, vm + np.array([Phi[0] / m, Phi[1] / m, 0.0]), rtol=0, atol=1e-15)
    vt = 0.5
    xm = np.zeros(model.nx)
    xm[:3], xm[3:6] = q[0], vm
    xp = xm.copy()
    xp[3:6] = [vt, 0.0, 0.3]
    gam = vt * np.sqrt(Phi[0] ** 2 + 1.0) / abs(Phi[0])
    delta = 1e-3
    th = impact.theta(model, xp, xm, Phi, np.array([gam]), p, delta)
    assert gam > 0.0
    assert abs(th[2] + delta) <= 1e-15 and abs(th[3] + delta) <= 1e-15
    assert abs(th[9]) <= 1e-15                      # rho = 0 on the cone boundary


@pytest.mark.parametrize("name", ["point1", "hopper", "biped3s", "cheetah7", "quad13"])
def test_compact_layout_holds_every_varying_entry(name):
    """The compact blocks of include/cis.h plus its constant entries rebuild the
    oracle's dense Jacobians exactly: no entry outside the blocks varies."""
    import impact_layout
    model, d = _rand_case(name, 16)
    lin = impact.linearize(model, d["Xp"], d["Xm"], d["Phi"], d["Gamma"], d["p"], 1e-2)
    JGv, JTc = impact_layout.compact_from_dense(model, lin["JG"], lin["JT"])
    JG, JT = impact_layout.dense_from_compact(model, JGv, JTc)
    assert np.array_equal(JG, lin["JG"])
    assert np.array_equal(JT, lin["JT"])
