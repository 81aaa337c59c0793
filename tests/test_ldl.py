"""Pins of the native sparse LDL^T (cis_ldl_*) used by the QP solver (CPU):
random quasi-definite matrices against dense NumPy solves, the symbolic
column counts against the dense factor's pattern, and the dynamic
regularization of pivots of the wrong sign."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2604_09993_amd import _lib


def _vp(a):
    return ctypes.c_void_p(a.ctypes.data)


def _quasi_definite(rng, n1, n2, density):
    H = sp.random(n1, n1, density=density, random_state=rng.integers(1 << 30)).toarray()
    H = H @ H.T + np.eye(n1)
    B = sp.random(n2, n1, density=density, random_state=rng.integers(1 << 30)).toarray()
    C = -np.eye(n2) * rng.uniform(0.5, 2.0, n2)
    return np.block([[H, B.T], [B, C]])


def _factor(K, sign=None, eps=0.0, delta=0.0):
    lib = _lib.load()
    n = K.shape[0]
    U = sp.csc_matrix(np.triu(K))
    U.sort_indices()
    Ap, Ai, Ax = U.indptr.astype(np.int32), U.indices.astype(np.int32), U.data.copy()
    parent, Lnz, work = (np.zeros(n, np.int32) for _ in range(3))
    lnz = lib.cis_ldl_symbolic(n, _vp(Ap), _vp(Ai), _vp(parent), _vp(Lnz), _vp(work))
    assert lnz >= 0
    Lp, Li, Lx = np.zeros(n + 1, np.int32), np.zeros(max(lnz, 1), np.int32), np.zeros(max(lnz, 1))
    D, iw, y = np.zeros(n), np.zeros(3 * n, np.int32), np.zeros(n)
    sg = None if sign is None else np.asarray(sign, np.int8)
    st = lib.cis_ldl_numeric(n, _vp(Ap), _vp(Ai), _vp(Ax), _vp(parent), _vp(Lnz),
                             None if sg is None else _vp(sg), ctypes.c_double(eps),
                             ctypes.c_double(delta), _vp(Lp), _vp(Li), _vp(Lx), _vp(D), _vp(iw),
                             _vp(y))
    return st, lnz, Lnz, (Lp, Li, Lx, D)


def _solve(n, fac, b):
    Lp, Li, Lx, D = fac
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    _lib.load().cis_ldl_solve(n, _vp(Lp), _vp(Li), _vp(Lx), _vp(D), _vp(x))
    return x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ldl_solves_quasi_definite_systems(seed):
    rng = np.random.default_rng(seed)
    K = _quasi_definite(rng, 40, 15, 0.08)
    n = K.shape[0]
    st, _, _, fac = _factor(K)
    assert st == 0
    b = rng.standard_normal(n)
    x = _solve(n, fac, b)
    np.testing.assert_allclose(x, np.linalg.solve(K, b), rtol=0, atol=1e-10)
    Lp, Li, Lx, D = fac
    L = np.eye(n) + sp.csc_matrix((Lx[:Lp[-1]], Li[:Lp[-1]], Lp), shape=(n, n)).toarray()
    np.testing.assert_allclose(L @ np.diag(D) @ L.T, K, rtol=0, atol=1e-11)
    assert (D[:40] > 0).all() and (D[40:] < 0).all()     # inertia of a quasi-definite matrix


def test_symbolic_counts_match_the_dense_factor_pattern():
    rng = np.random.default_rng(3)
    K = _quasi_definite(rng, 30, 10, 0.1)
    n = K.shape[0]
    _, lnz, Lnz, fac = _factor(K)
    Lp, Li, Lx, _ = fac
    L = sp.csc_matrix((Lx[:Lp[-1]], Li[:Lp[-1]], Lp), shape=(n, n)).toarray()
    # structural counts bound the numerical nonzeros and equal them for generic values
    assert np.array_equal(np.count_nonzero(np.abs(L) > 0, axis=0), Lnz)
    assert lnz == Lnz.sum()


def test_pivot_of_the_wrong_sign_is_replaced():
    K = np.array([[1.0, 1.0], [1.0, 0.5]])          # second pivot 0.5 - 1 = -0.5
    st, _, _, fac = _factor(K, sign=[1, 1], eps=1e-12, delta=1e-3)
    assert st == 1 and fac[3][1] == 1e-3
    st, _, _, fac = _factor(K, sign=[1, -1], eps=1e-12, delta=1e-3)
    assert st == 0 and fac[3][1] == -0.5


def test_entries_below_the_diagonal_are_rejected():
    lib = _lib.load()
    Ap = np.array([0, 2, 3], np.int32)
    Ai = np.array([0, 1, 1], np.int32)                # row 1 in column 0
    parent, Lnz, work = (np.zeros(2, np.int32) for _ in range(3))
    assert lib.cis_ldl_symbolic(2, _vp(Ap), _vp(Ai), _vp(parent), _vp(Lnz), _vp(work)) == -2


def test_zero_pivot_without_signs_is_an_error_and_null_pointers_are_refused():
    K = np.array([[1.0, 1.0], [1.0, 1.0]])          # singular: second pivot exactly 0
    st, _, _, _ = _factor(K)
    assert st == -2
    lib = _lib.load()
    assert lib.cis_ldl_symbolic(2, None, None, None, None, None) == -1
    assert lib.cis_ldl_numeric(2, None, None, None, None, None, None, ctypes.c_double(0.0),
                               ctypes.c_double(0.0), None, None, None, None, None, None) == -1
    assert lib.cis_ldl_symbolic(0, _vp(np.zeros(1, np.int32)), None, None, None, None) == 0
