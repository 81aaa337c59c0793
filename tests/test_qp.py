"""Pins of the interior-point QP solver of the SCP driver (CPU only).

Checked against things other than itself: SciPy's HiGHS linear-programming
solver on random LPs, the closed-form solution of equality-constrained QPs
(the KKT linear system), the projection onto a box, brute-force enumeration
of active sets on tiny QPs, and the KKT conditions.
"""
import itertools

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from paper_2604_09993_amd.qp import solve_qp

TOL = 1e-10   # tighter than the driver's default: these compare to exact optima


def _random_lp(rng, n, me, mi):
    A = rng.standard_normal((me, n))
    x0 = rng.uniform(0.1, 1.0, n)                # a strictly feasible point
    b = A @ x0
    G = np.vstack([rng.standard_normal((mi, n)), -np.eye(n), np.eye(n)])   # bounded: 0 <= x <= 5
    h = np.concatenate([G[:mi] @ x0 + rng.uniform(0.1, 1.0, mi), np.zeros(n), np.full(n, 5.0)])
    c = rng.standard_normal(n)
    return c, A, b, G, h


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_lp_matches_highs(seed):
    rng = np.random.default_rng(seed)
    c, A, b, G, h = _random_lp(rng, 30, 8, 20)
    ref = so.linprog(c, A_ub=G, b_ub=h, A_eq=A, b_eq=b, bounds=[(None, None)] * 30, method="highs")
    assert ref.status == 0
    r = solve_qp(sp.csr_matrix((30, 30)), c, A, b, G, h, tol=TOL)
    assert r.status == "optimal"
    assert abs(r.obj - ref.fun) <= 1e-7 * (1.0 + abs(ref.fun))
    assert np.abs(A @ r.x - b).max() <= 1e-7
    assert (G @ r.x - h).max() <= 1e-7


@pytest.mark.parametrize("seed", [4, 5])
def test_equality_qp_is_the_kkt_solution(seed):
    rng = np.random.default_rng(seed)
    n, me = 25, 7
    L = rng.standard_normal((n, n))
    P = L @ L.T + 0.1 * np.eye(n)
    q = rng.standard_normal(n)
    A = rng.standard_normal((me, n))
    b = rng.standard_normal(me)
    K = np.block([[P, A.T], [A, np.zeros((me, me))]])
    sol = np.linalg.solve(K, np.concatenate([-q, b]))
    r = solve_qp(P, q, A, b, tol=TOL)
    assert r.status == "optimal"
    np.testing.assert_allclose(r.x, sol[:n], rtol=0, atol=1e-9 * max(1.0, np.abs(sol).max()))
    np.testing.assert_allclose(r.y, sol[n:], rtol=0, atol=1e-8 * max(1.0, np.abs(sol).max()))


def test_box_qp_is_the_projection():
    rng = np.random.default_rng(6)
    n = 40
    c = rng.standard_normal(n) * 3.0
    lo, hi = -np.ones(n), np.ones(n)
    G = sp.vstack([sp.identity(n), -sp.identity(n)])
    r = solve_qp(sp.identity(n), -c, G=G, h=np.concatenate([hi, -lo]), tol=TOL)
    assert r.status == "optimal"
    np.testing.assert_allclose(r.x, np.clip(c, lo, hi), rtol=0, atol=1e-7)


def _brute_force_qp(P, q, G, h):
    """Enumerate active sets: the equality-constrained QP on each subset whose
    solution is feasible with nonnegative multipliers is the optimum."""
    n, mi = q.size, h.size
    best = None
    for k in range(0, n + 1):
        for act in itertools.combinations(range(mi), k):
            act = list(act)
            Ga = G[act]
            K = np.block([[P, Ga.T], [Ga, np.zeros((k, k))]])
            try:
                sol = np.linalg.solve(K, np.concatenate([-q, h[act]]))
            except np.linalg.LinAlgError:
                continue
            x, lam = sol[:n], sol[n:]
            if (G @ x - h).max() <= 1e-10 and (lam >= -1e-10).all():
                obj = 0.5 * x @ P @ x + q @ x
                if best is None or obj < best[1]:
                    best = (x, obj)
    return best


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_inequality_qp_matches_active_set_enumeration(seed):
    rng = np.random.default_rng(seed)
    n, mi = 3, 6
    L = rng.standard_normal((n, n))
    P = L @ L.T + 0.05 * np.eye(n)
    q = rng.standard_normal(n) * 2.0
    G = rng.standard_normal((mi, n))
    h = rng.uniform(0.1, 1.0, mi)                 # x = 0 strictly feasible
    x_ref, obj_ref = _brute_force_qp(P, q, G, h)
    r = solve_qp(P, q, G=G, h=h, tol=TOL)
    assert r.status == "optimal"
    np.testing.assert_allclose(r.x, x_ref, rtol=0, atol=1e-7)
    assert abs(r.obj - obj_ref) <= 1e-9 * (1.0 + abs(obj_ref))


def test_mixed_qp_satisfies_the_kkt_conditions():
    rng = np.random.default_rng(10)
    n, me, mi = 60, 10, 50
    Ls = sp.random(n, n, density=0.05, random_state=11)
    P = (Ls @ Ls.T + sp.diags(rng.uniform(0.0, 1.0, n))).tocsr()   # PSD, some zero curvature
    q = rng.standard_normal(n)
    c, A, b, G, h = _random_lp(rng, n, me, mi)
    r = solve_qp(P, q, A, b, G, h, tol=TOL)
    assert r.status == "optimal"
    stat = P @ r.x + q + A.T @ r.y + G.T @ r.z
    assert np.abs(stat).max() <= 1e-7 * (1.0 + np.abs(q).max())
    assert np.abs(A @ r.x - b).max() <= 1e-7
    assert (G @ r.x - h).max() <= 1e-7
    assert r.z.min() >= 0.0 and r.s.min() >= 0.0
    assert abs(r.z @ (h - G @ r.x)) <= 1e-6


def test_l1_penalty_in_epigraph_form_is_soft_thresholding():
    """min 1/2 (x - c)^2 + w |x| written with x = p - m, p, m >= 0: the
    minimizer is the soft threshold sign(c) max(|c| - w, 0)."""
    for c in (-3.0, -0.2, 0.0, 0.4, 2.5):
        w = 0.5
        P = sp.csr_matrix(np.array([[1.0, -1.0], [-1.0, 1.0]]))
        q = np.array([-c + w, c + w])
        r = solve_qp(P, q, G=-sp.identity(2), h=np.zeros(2), tol=TOL)
        assert r.status == "optimal"
        x = r.x[0] - r.x[1]
        assert abs(x - np.sign(c) * max(abs(c) - w, 0.0)) <= 1e-8
