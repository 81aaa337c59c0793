"""Sparse convex quadratic programs by a primal-dual interior-point method.

The convex subproblems of the sequential convex programming driver (arxiv
2604.09993, Sec. V and the canonicalization of Sec. VI) are, for the planar
models here, quadratic programs: the two-dimensional friction cone of the
controls is polyhedral, the exact l1 penalties are linear programs in
epigraph form and the proximal term is a convex quadratic.  This module
solves

    minimize 1/2 x^T P x + q^T x   subject to   A x = b,   G x <= h

with Mehrotra's predictor-corrector method on the nonnegative orthant
(slacks s = h - G x >= 0, multipliers z >= 0): each iteration factors the
reduced quasi-definite system

    [ P + G^T D G + r I   A^T  ] [dx]   [r1]
    [ A                  -r I  ] [dy] = [r2],      D = diag(z / s),

once (sparse LU of SciPy) and solves it twice (affine and corrected
directions), with a few steps of iterative refinement against the
unregularized matrix.  Rows of A and G are scaled to unit infinity norm
before the solve (the row normalization of the canonical form).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class QPResult:
    x: np.ndarray
    y: np.ndarray          # multipliers of A x = b
    z: np.ndarray          # multipliers of G x <= h (>= 0)
    s: np.ndarray          # slacks h - G x (>= 0)
    status: str            # "optimal", "stalled" (step length collapsed) or "max_iter"
    iters: int
    obj: float
    res_primal: float
    res_dual: float
    gap: float


def _row_scale(M, v):
    """Scale the rows of sparse M (and the entries of v) to unit infinity norm."""
    if M.shape[0] == 0:
        return M, v, np.ones(0)
    nrm = np.asarray(abs(M).max(axis=1).todense()).ravel()
    nrm[nrm == 0.0] = 1.0
    sc = 1.0 / nrm
    return sp.diags(sc) @ M, v * sc, sc


def _max_step(v, dv):
    """Largest a in (0, 1] with v + a dv >= 0 (v > 0)."""
    neg = dv < 0.0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-v[neg] / dv[neg])))


def solve_qp(P, q, A=None, b=None, G=None, h=None, *, tol=1e-8, max_iter=80, reg=1e-11,
             refine=2, min_step=1e-8) -> QPResult:
    """Solve the convex QP above.  P [n, n] symmetric positive semidefinite
    (sparse or dense), q [n]; A [me, n], b [me]; G [mi, n], h [mi] (either pair
    may be None).  The problem must be feasible with a bounded optimum.
    Stops when the scaled primal and dual residuals and the relative gap are
    below tol; status "stalled" reports a stop on a step shorter than min_step
    (the reduced system has lost the accuracy to go further: the last iterate
    is returned with its residuals), "max_iter" one that ran out of
    iterations."""
    q = np.asarray(q, dtype=np.float64)
    n = q.size
    P = sp.csr_matrix(P, shape=(n, n), dtype=np.float64)
    A = sp.csr_matrix((0, n)) if A is None else sp.csr_matrix(A, dtype=np.float64)
    b = np.zeros(0) if b is None else np.asarray(b, dtype=np.float64)
    G = sp.csr_matrix((0, n)) if G is None else sp.csr_matrix(G, dtype=np.float64)
    h = np.zeros(0) if h is None else np.asarray(h, dtype=np.float64)
    me, mi = A.shape[0], G.shape[0]
    if A.shape[1] != n or G.shape[1] != n or b.size != me or h.size != mi:
        raise ValueError("inconsistent QP dimensions")
    A, b, sca = _row_scale(A, b)
    G, h, scg = _row_scale(G, h)
    At, Gt = A.T.tocsr(), G.T.tocsr()
    nq, nb, nh = max(1.0, np.abs(q).max(initial=0.0)), max(1.0, np.abs(b).max(initial=0.0)), \
        max(1.0, np.abs(h).max(initial=0.0))

    def factor(D):
        H = (P + Gt @ sp.diags(D) @ G).tocsr()
        K0 = sp.bmat([[H, At], [A, sp.csr_matrix((me, me))]], format="csc")
        Kr = (K0 + sp.diags(np.concatenate([np.full(n, reg), np.full(me, -reg)]))).tocsc()
        return K0, spla.splu(Kr, permc_spec="MMD_AT_PLUS_A")

    def solve(fac, r1, r2):
        K0, lu = fac
        rhs = np.concatenate([r1, r2])
        sol = lu.solve(rhs)
        for _ in range(refine):
            sol = sol + lu.solve(rhs - K0 @ sol)
        return sol[:n], sol[n:]

    # starting point: the least-squares point of the constraints with D = I,
    # slacks and multipliers shifted into the interior
    fac = factor(np.ones(mi))
    x, y = solve(fac, -q + Gt @ h, b)
    s = h - G @ x
    z = -s.copy()
    if mi:
        a = -s.min()
        if a >= 0.0:
            s = s + 1.0 + a
        a = -z.min()
        if a >= 0.0:
            z = z + 1.0 + a

    status, it = "max_iter", 0
    rp = rd = gap = np.inf
    for it in range(1, max_iter + 1):
        r_d = P @ x + q + At @ y + Gt @ z
        r_p = A @ x - b
        r_i = G @ x + s - h
        mu = float(s @ z) / mi if mi else 0.0
        obj = 0.5 * float(x @ (P @ x)) + float(q @ x)
        rd = np.abs(r_d).max(initial=0.0) / nq
        rp = max(np.abs(r_p).max(initial=0.0) / nb, np.abs(r_i).max(initial=0.0) / nh)
        gap = (float(s @ z) / (1.0 + abs(obj))) if mi else 0.0
        if rd <= tol and rp <= tol and gap <= tol:
            status = "optimal"
            break
        D = z / s if mi else np.zeros(0)
        fac = factor(D)

        def direction(r_c):
            dx, dy = solve(fac, -r_d - Gt @ (D * r_i - r_c / s), -r_p)
            dz = D * (G @ dx + r_i) - r_c / s
            ds = -r_i - G @ dx
            return dx, dy, dz, ds

        # predictor (affine scaling) direction
        dxa, dya, dza, dsa = direction(s * z)
        if mi:
            aa = min(_max_step(s, dsa), _max_step(z, dza))
            mua = float((s + aa * dsa) @ (z + aa * dza)) / mi
            sigma = (mua / mu) ** 3 if mu > 0.0 else 0.0
            # corrector: centring plus the second-order term
            dx, dy, dz, ds = direction(s * z + dsa * dza - sigma * mu)
            a = min(1.0, 0.99 * min(_max_step(s, ds), _max_step(z, dz)))
        else:
            dx, dy, dz, ds = dxa, dya, dza, dsa
            a = 1.0
        if a < min_step:
            status = "stalled"
            break
        x, y, z, s = x + a * dx, y + a * dy, z + a * dz, s + a * ds
    obj = 0.5 * float(x @ (P @ x)) + float(q @ x)
    # undo the row scaling of the multipliers
    return QPResult(x=x, y=y * sca, z=z * scg, s=s / scg if mi else s, status=status, iters=it,
                    obj=obj, res_primal=float(rp), res_dual=float(rd), gap=float(gap))
