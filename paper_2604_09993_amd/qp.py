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

once and solves it twice (affine and corrected directions), with a few
steps of iterative refinement against the unregularized matrix.  The cost is scaled so that its largest coefficient
is 1 (multipliers are returned unscaled).  The
factorization is the native sparse LDL^T of libcis (cis_ldl_*) in a
fill-reducing symmetric order (minimum degree on the pattern, taken from
SciPy's SuperLU once per sparsity pattern); the pattern of the reduced
matrix, the order and the elimination tree are computed once per pattern and
can be kept across solves (`cache`).  Rows of A and G are scaled to unit
infinity norm before the solve (the row normalization of the canonical form).
"""
from __future__ import annotations

from dataclasses import dataclass

import ctypes
import hashlib

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import _lib


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


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data)


class _Kkt:
    """The reduced KKT matrix K(D) = [P + G^T D G + r I, A^T; A, -r I] of one
    sparsity pattern of (P, A, G): its upper triangle in a fill-reducing
    symmetric order (CSC), where every entry comes from (the constants of P,
    A and r, and the D-weighted products of pairs of entries of one row of
    G), and the native symbolic factorization.  Values are set per solve."""

    def __init__(self, P, A, G, reg):
        n, me = P.shape[0], A.shape[0]
        N = n + me
        self.n, self.me, self.N, self.reg = n, me, N, reg
        # constants: upper triangle of P, A^T above the diagonal, the diagonal
        Pc = P.tocoo()
        self.p_up = np.nonzero(Pc.row <= Pc.col)[0]
        Ac = A.tocoo()
        d = np.arange(N)
        cr = np.concatenate([Pc.row[self.p_up], Ac.col, d]).astype(np.int64)
        cc = np.concatenate([Pc.col[self.p_up], n + Ac.row, d]).astype(np.int64)
        self.regdiag = np.concatenate([np.full(n, reg), np.full(me, -reg)])
        # pairs (a <= b) of entries of each row of G, as positions in G.data
        lens = np.diff(G.indptr)
        pa, pb, pr = [], [], []
        for k in np.unique(lens):
            if k == 0:
                continue
            rows = np.nonzero(lens == k)[0]
            ia, ib = np.triu_indices(k)
            base = G.indptr[rows][:, None]
            pa.append((base + ia[None, :]).ravel())
            pb.append((base + ib[None, :]).ravel())
            pr.append(np.repeat(rows, ia.size))
        cat = lambda x: np.concatenate(x).astype(np.int64) if x else np.zeros(0, np.int64)
        self.pa, self.pb, self.gr = cat(pa), cat(pb), cat(pr)
        ga, gb = G.indices[self.pa].astype(np.int64), G.indices[self.pb].astype(np.int64)
        # fill-reducing order from the symmetric pattern (values at D = 1)
        cv = self._const_values(P, A)
        gw = G.data[self.pa] * G.data[self.pb]
        Kfull = sp.csc_matrix((np.concatenate([cv, cv, gw, gw]),
                               (np.concatenate([cr, cc, ga, gb]), np.concatenate([cc, cr, gb, ga]))),
                              shape=(N, N))
        Kfull.sum_duplicates()
        lu = spla.splu(Kfull, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        best = None
        for perm in (lu.perm_c, np.argsort(lu.perm_c)):
            st = self._structure(np.asarray(perm, np.int64), cr, cc, ga, gb)
            if best is None or st["lnz"] < best["lnz"]:
                best = st
        self.__dict__.update(best)
        self.Lp = np.zeros(N + 1, np.int32)
        self.Li = np.zeros(max(self.lnz, 1), np.int32)
        self.Lx = np.zeros(max(self.lnz, 1))
        self.Dl = np.zeros(N)
        self.iwork = np.zeros(3 * N, np.int32)
        self.y = np.zeros(N)
        # expected pivot signs in the elimination order: + on the primal block,
        # - on the multipliers of the equalities
        self.sign = np.where(self.perm < n, 1, -1).astype(np.int8)
        self.replaced = 0

    def _const_values(self, P, A):
        return np.concatenate([P.tocoo().data[self.p_up], A.tocoo().data, self.regdiag])

    def set_values(self, P, A, G):
        """Constants and pair products of this solve's matrices (same pattern)."""
        self.const = np.bincount(self.inv_c, weights=self._const_values(P, A),
                                 minlength=self.nnz)
        self.gw = G.data[self.pa] * G.data[self.pb]

    def _structure(self, perm, cr, cc, ga, gb):
        N = self.N
        pinv = np.empty(N, np.int64)
        pinv[perm] = np.arange(N)

        def key(r, c):
            pr, pc = pinv[r], pinv[c]
            return np.minimum(pr, pc) + N * np.maximum(pr, pc)
        kc, kg = key(cr, cc), key(ga, gb)
        uniq, inv = np.unique(np.concatenate([kc, kg]), return_inverse=True)
        Ai = (uniq % N).astype(np.int32)
        colk = uniq // N
        Ap = np.zeros(N + 1, np.int32)
        np.cumsum(np.bincount(colk, minlength=N), out=Ap[1:])
        parent = np.zeros(N, np.int32)
        Lnz = np.zeros(N, np.int32)
        work = np.zeros(N, np.int32)
        lnz = _lib.load().cis_ldl_symbolic(N, _vp(Ap), _vp(Ai), _vp(parent), _vp(Lnz), _vp(work))
        if lnz < 0:
            raise RuntimeError(f"cis_ldl_symbolic failed ({lnz})")
        return dict(perm=perm, Ap=Ap, Ai=Ai, nnz=uniq.size, inv_c=inv[:kc.size],
                    inv_g=inv[kc.size:], parent=parent, Lnz=Lnz, lnz=int(lnz))

    def factor(self, D):
        Ax = self.const + np.bincount(self.inv_g, weights=self.gw * D[self.gr],
                                      minlength=self.nnz)
        st = _lib.load().cis_ldl_numeric(self.N, _vp(self.Ap), _vp(self.Ai), _vp(Ax),
                                         _vp(self.parent), _vp(self.Lnz), _vp(self.sign),
                                         ctypes.c_double(1e-13), ctypes.c_double(1e-7),
                                         _vp(self.Lp), _vp(self.Li), _vp(self.Lx),
                                         _vp(self.Dl), _vp(self.iwork), _vp(self.y))
        if st < 0:
            raise RuntimeError(f"cis_ldl_numeric failed ({st})")
        self.replaced = st

    def solve(self, rhs):
        x = np.ascontiguousarray(rhs[self.perm])
        _lib.load().cis_ldl_solve(self.N, _vp(self.Lp), _vp(self.Li), _vp(self.Lx), _vp(self.Dl),
                                  _vp(x))
        out = np.empty_like(x)
        out[self.perm] = x
        return out


def _pattern_key(*mats):
    h = hashlib.sha1()
    for M in mats:
        h.update(np.asarray(M.shape, np.int64).tobytes())
        h.update(M.indptr.tobytes())
        h.update(M.indices.tobytes())
    return h.hexdigest()


D_MIN, D_MAX = 1e-24, 1e24   # bounds of the slack scaling z / s
TINY = 1e-300                # floor of slacks and multipliers after a step


def _max_step(v, dv):
    """Largest a in (0, 1] with v + a dv >= 0 (v > 0)."""
    neg = dv < 0.0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-v[neg] / dv[neg])))


def solve_qp(P, q, A=None, b=None, G=None, h=None, *, tol=1e-8, max_iter=80, reg=1e-11,
             refine=2, min_step=1e-8, cache=None) -> QPResult:
    """Solve the convex QP above.  P [n, n] symmetric positive semidefinite
    (sparse or dense), q [n]; A [me, n], b [me]; G [mi, n], h [mi] (either pair
    may be None).  The problem must be feasible with a bounded optimum.
    Stops when the scaled primal and dual residuals and the relative gap are
    below tol; status "stalled" reports a stop on a step shorter than min_step
    (the reduced system has lost the accuracy to go further: the last iterate
    is returned with its residuals), "max_iter" one that ran out of
    iterations.  `cache` (a dict) keeps the ordering and symbolic
    factorization for the next solve with the same sparsity pattern."""
    q = np.asarray(q, dtype=np.float64)
    n = q.size
    P = sp.csr_matrix(P, shape=(n, n), dtype=np.float64)
    P.sum_duplicates()
    A = sp.csr_matrix((0, n)) if A is None else sp.csr_matrix(A, dtype=np.float64)
    b = np.zeros(0) if b is None else np.asarray(b, dtype=np.float64)
    G = sp.csr_matrix((0, n)) if G is None else sp.csr_matrix(G, dtype=np.float64)
    h = np.zeros(0) if h is None else np.asarray(h, dtype=np.float64)
    me, mi = A.shape[0], G.shape[0]
    if A.shape[1] != n or G.shape[1] != n or b.size != me or h.size != mi:
        raise ValueError("inconsistent QP dimensions")
    A, b, sca = _row_scale(A, b)
    G, h, scg = _row_scale(G, h)
    # cost scaling: the largest entry of P and q becomes 1, so that the
    # multipliers (and the slack scaling z / s) stay near unit size
    cs = max(np.abs(q).max(initial=0.0), np.abs(P.data).max(initial=0.0))
    cs = 1.0 / cs if cs > 0.0 else 1.0
    P, q = P * cs, q * cs
    At, Gt = A.T.tocsr(), G.T.tocsr()
    nq, nb, nh = max(1.0, np.abs(q).max(initial=0.0)), max(1.0, np.abs(b).max(initial=0.0)), \
        max(1.0, np.abs(h).max(initial=0.0))

    for M in (P, A, G):
        M.sum_duplicates()
        M.sort_indices()
    key = _pattern_key(P, A, G) + repr(reg)
    kkt = cache.get(key) if cache is not None else None
    if kkt is None:
        kkt = _Kkt(P, A, G, reg)
        if cache is not None:
            cache.clear()
            cache[key] = kkt
    kkt.set_values(P, A, G)

    def factor(D):
        kkt.factor(D)
        return D

    def solve(D, r1, r2):
        # K(D) without the regularization, applied for the refinement steps
        def K0(v):
            v1, v2 = v[:n], v[n:]
            return np.concatenate([P @ v1 + Gt @ (D * (G @ v1)) + At @ v2, A @ v1])
        rhs = np.concatenate([r1, r2])
        sol = kkt.solve(rhs)
        for _ in range(refine):
            sol = sol + kkt.solve(rhs - K0(sol))
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
        # scaling of the slacks, bounded so that the reduced matrix stays
        # finite when a slack or multiplier has reached the rounding level
        D = np.clip(z / s, D_MIN, D_MAX) if mi else np.zeros(0)
        try:
            fac = factor(D)
        except RuntimeError:
            status = "stalled"
            break

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
        if mi:
            np.maximum(z, TINY, out=z)
            np.maximum(s, TINY, out=s)
    obj = (0.5 * float(x @ (P @ x)) + float(q @ x)) / cs
    # undo the cost scaling and the row scaling of the multipliers
    return QPResult(x=x, y=y * sca / cs, z=z * scg / cs, s=s / scg if mi else s, status=status,
                    iters=it, obj=obj, res_primal=float(rp), res_dual=float(rd), gap=float(gap))
