"""CPU tests of the SCP driver (Sec. V, Alg. 1; Sec. IV-C eq. cito-problem;
Sec. VI discontinuous first-order hold) with the oracle transcription.

Pinned against things other than the driver itself: the delta update is
checked branch by branch on scripted histories; the node-doubled layout of
the discontinuous hold against the oracle's single-interval integrator; the
dense node Jacobians against the impact oracle's complex-step Jacobians;
the assembled linear model against central differences of the nonlinear
residuals (which catches misplaced columns, signs and scalings); and the
subproblem's solution against its own hard constraints.
"""
import numpy as np
import pytest

import oracle
from oracle import impact
from paper_2604_09993_amd import scp, synth
from paper_2604_09993_amd.qp import solve_qp

from impact_layout import compact_from_dense
from scp_oracle import oracle_transcriber


def _problem(N=4, K=3, seed=0):
    model = synth.make_hopper(np.random.default_rng(seed))
    xi = synth.standing_state(model, 0.0)
    xf = synth.standing_state(model, 0.3)
    pb = scp.CitoProblem(model, N, xi, xf, K=K)
    g = synth.scp_initial_guess(model, N, xi, xf, 0.05, np.random.default_rng(seed + 1))
    z = pb.pack(g["Xp"], g["Xm"], g["Phi"], g["Gamma"], g["Ua"], g["Ub"], g["S"])
    return pb, z


# ---- Alg. 1 ------------------------------------------------------------------
def test_homotopy_shrinks_when_both_terms_decrease():
    h = scp.DeltaHomotopy(delta0=1.0, alpha=0.5, n_stall=3)
    h.update(10.0, 10.0)          # j = 0: larger than J_0 = 0, so delta is held
    assert h.delta == [1.0, 1.0]
    h.update(5.0, 5.0)            # j = 1: M = 1, no increase: shrink
    h.update(4.0, 4.0)
    assert h.delta == [1.0, 1.0, 0.5, 0.25]


def test_homotopy_holds_on_an_increase_since_the_previous_iterate():
    h = scp.DeltaHomotopy(delta0=1.0, alpha=0.5, n_stall=1)
    for J in (10.0, 5.0, 4.0):
        h.update(J, J)
    # j = 3: M = max(3 - 1, 1) = 2, J_M = 5; new J_px 4.5 > J_3 = 4 but < J_M
    h.update(4.5, 1.0)
    assert h.delta[-1] == h.delta[-2]


def test_homotopy_bisects_in_log_scale_on_an_increase_since_the_stall_horizon():
    h = scp.DeltaHomotopy(delta0=1.0, alpha=0.5, n_stall=1)
    for J in (10.0, 5.0, 4.0):
        h.update(J, J)
    d = list(h.delta)             # [1, 1, 0.5, 0.25]
    h.update(1.0, 6.0)            # J_ep 6 > J_M = J_2 = 5: sqrt(delta_3 delta_2)
    assert np.isclose(h.delta[-1], np.sqrt(d[3] * d[2]), rtol=1e-15)


def test_homotopy_terminates_only_with_both_terms_small_and_delta_tight():
    h = scp.DeltaHomotopy(delta0=1.0, delta_min=0.3, eps_px=1e-3, eps_ep=1e-3, alpha=0.5)
    h.update(1e-4, 1e-4)
    assert not h.done()           # delta still 1
    h.update(1e-5, 1e-5)          # shrink to 0.5
    h.update(1e-6, 1e-6)          # shrink to 0.25
    assert h.done()
    h.update(1.0, 1e-6)
    assert not h.done()


# ---- discontinuous hold: node-doubled intervals ------------------------------
def test_doubled_layout_integrates_each_interval_with_its_own_hold_ends():
    pb, z = _problem(N=3, K=2)
    v = pb.unpack(z)
    Xd, Ud, sd = pb.doubled(v)
    out = oracle.discretize(pb.model, Xd, Ud, sd, pb.p, pb.K)
    for k in range(pb.N):
        ref = oracle.integrate(pb.model, v["Xp"][k], v["Ua"][k], v["Ub"][k], v["S"][k], pb.p,
                               pb.K)
        np.testing.assert_array_equal(out["xprop"][2 * k], ref["xf"])
        np.testing.assert_array_equal(out["A"][2 * k], ref["Phi"])
        np.testing.assert_array_equal(out["Bm"][2 * k], ref["Bm"])
        np.testing.assert_array_equal(out["Bp"][2 * k], ref["Bp"])
        np.testing.assert_array_equal(out["d"][2 * k], ref["xf"] - v["Xm"][k + 1])


def test_pack_and_unpack_are_inverse():
    pb, z = _problem()
    v = pb.unpack(z)
    np.testing.assert_array_equal(pb.pack(v["Xp"], v["Xm"], v["Phi"], v["Gamma"], v["Ua"],
                                          v["Ub"], v["S"]), z)


# ---- node Jacobians from the compact layout ----------------------------------
def test_expanded_node_jacobians_are_the_dense_ones():
    pb, z = _problem(N=2)
    v = pb.unpack(z)
    lin = impact.linearize(pb.model, v["Xp"], v["Xm"], v["Phi"], v["Gamma"], pb.p, 0.3)
    JGv, JTc = compact_from_dense(pb.model, lin["JG"], lin["JT"])
    JG, JT = scp.expand_node_jacobians(pb.model, JGv, JTc)
    np.testing.assert_array_equal(JG, lin["JG"][:, :, :pb.NB])
    np.testing.assert_array_equal(JT, lin["JT"][:, :, :pb.NB])


# ---- the assembled linear model ----------------------------------------------
def _residuals(pb, tr, z, delta):
    t = tr(pb.unpack(z), delta)
    return dict(d=t["d"], G=t["G"], Theta=t["Theta"], Psi=t["Psi"])


def test_assembled_rows_are_central_differences_of_the_residuals():
    pb, z = _problem(N=3, K=2)
    delta = 0.4
    tr = oracle_transcriber(pb)
    sub = scp.assemble(pb, z, tr(pb.unpack(z), delta), 2000.0, 5e4)
    N, nx, nth, ny, nz = pb.N, pb.nx, 10 * pb.nc, pb.ny, pb.nz
    Aeq, Gin = sub.A.toarray()[:, :nz], sub.G.toarray()[:, :nz]
    base = _residuals(pb, tr, z, delta)
    # anchoring: the constants are the residuals at the iterate
    np.testing.assert_allclose(sub.b[:N * nx], -(base["d"] / pb.xscale).ravel(), rtol=0,
                               atol=1e-15)
    np.testing.assert_allclose(sub.h[:(N + 1) * nth], -base["Theta"].ravel(), rtol=0, atol=0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal(nz)
        eps = 1e-6
        rp = _residuals(pb, tr, z + eps * pb.zscale * u, delta)
        rm = _residuals(pb, tr, z - eps * pb.zscale * u, delta)
        fd = {k: (rp[k] - rm[k]) / (2 * eps) for k in rp}
        lin_eq = Aeq @ u
        lin_in = Gin @ u
        want_dyn = (fd["d"] / pb.xscale).ravel()
        want_G = (fd["G"] / pb.xscale).ravel()
        got_dyn = lin_eq[:N * nx]
        got_G = lin_eq[N * nx:N * nx + (N + 1) * nx]
        for got, want in ((got_dyn, want_dyn), (got_G, want_G),
                          (lin_in[:(N + 1) * nth], fd["Theta"].ravel()),
                          (lin_in[(N + 1) * nth:(N + 1) * nth + N * ny], fd["Psi"].ravel())):
            assert np.max(np.abs(got - want)) <= 1e-6 * max(1.0, np.max(np.abs(want)))


def test_subproblem_solution_keeps_the_hard_constraints():
    pb, z = _problem(N=4, K=3)
    tr = oracle_transcriber(pb)
    sub = scp.assemble(pb, z, tr(pb.unpack(z), 1.0), 2000.0, 5e4)
    r = solve_qp(sub.P, sub.q, sub.A, sub.b, sub.G, sub.h, tol=1e-9)
    assert r.status == "optimal"
    zn = z + pb.zscale * r.x[:pb.nz]
    v = pb.unpack(zn)
    tol = 1e-6
    np.testing.assert_allclose(v["Xm"][0], pb.x_init, rtol=0, atol=tol)
    np.testing.assert_allclose(v["Xp"][-1][:2 * pb.nq], pb.x_final[:2 * pb.nq], rtol=0, atol=tol)
    nj, mu = pb.nj, pb.p[0]
    for U in (v["Ua"], v["Ub"]):
        assert np.abs(U[:, :nj]).max() <= pb.tau_max + tol
        lam = U[:, 3 * nj:]
        assert lam.min() >= -tol
        assert (mu * lam[:, 0::3] - lam[:, 1::3] - lam[:, 2::3]).min() >= -tol
    assert v["S"].min() >= pb.s_min - tol and v["S"].max() <= pb.s_max + tol
    assert r.x[pb.nz:].min() >= -tol     # penalty variables


def test_three_iterations_reduce_the_exact_penalty():
    """Seeded monoped problem (N = 14, K = 10, the paper's grid): the
    linearized l1 penalty of the third subproblem is well below the first's,
    and delta follows Alg. 1 (held once, then shrunk twice)."""
    pb, z = _problem(N=14, K=10, seed=0)
    drv = scp.ScpDriver(pb, oracle_transcriber(pb))
    drv.run(z, max_iter=3)
    J = [r.J_ep for r in drv.history]
    assert len(J) == 3 and J[2] < 0.1 * J[0]
    np.testing.assert_allclose(drv.hom.delta, [1.0, 1.0, 0.85, 0.85 ** 2], rtol=1e-15)
    assert all(r.qp_status in ("optimal", "stalled") for r in drv.history)
