"""CPU FP64 oracle for the interval linearize-and-discretize step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  The oracle shares no code
with the HIP path and never calls it.  It is plain, dense and slow on purpose;
see ``cis_oracle.c`` for what each function follows in the paper
(arxiv 2604.09993: Sec. II dynamics, Sec. III integral cross-complementarity,
Sec. IV-B time-dilated augmented system with FOH controls, Sec. VI IND).

Arrays here are node-major numpy float64: X[N+1, nx], U[N+1, m], s[N].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cis_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, IEEE arithmetic, OpenMP over intervals)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OModel(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("nj", ctypes.c_int), ("nc", ctypes.c_int),
                ("len", ctypes.c_void_p), ("jp", ctypes.c_void_p), ("jc", ctypes.c_void_p),
                ("rp", ctypes.c_void_p), ("rc", ctypes.c_void_p),
                ("kst", ctypes.c_void_p), ("dmp", ctypes.c_void_p),
                ("cb", ctypes.c_void_p), ("cr", ctypes.c_void_p),
                ("g", ctypes.c_double), ("A", ctypes.c_double), ("kappa", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        _lib.oracle_rhs_jac.argtypes = [P] * 10
        _lib.oracle_integrate.argtypes = [P, P, P, P, ctypes.c_double, P, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, P, P, P, P, P, P]
        _lib.oracle_discretize.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P,
                                           P, P, P, P, P, P, P, ctypes.c_int]
        _lib.oracle_defects.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                        ctypes.c_int]
        _lib.oracle_adjoint.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P,
                                        P, P, P, P, ctypes.c_int]
        _lib.oracle_rkf_tableau.argtypes = [P, P, P, P]
        _lib.oracle_integrate_erk.argtypes = ([P, P, P, P, ctypes.c_double, P, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int]
                                              + [P] * 10)
        _lib.oracle_discretize_rkf.argtypes = [P, ctypes.c_int, ctypes.c_int] + [P] * 11 + [
            ctypes.c_int]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleModel:
    """Holds contiguous copies of a model description for the C oracle."""

    def __init__(self, model):
        self._keep = [
            np.ascontiguousarray(model.link_length, dtype=np.float64),
            np.ascontiguousarray(model.joint_parent, dtype=np.int32),
            np.ascontiguousarray(model.joint_child, dtype=np.int32),
            np.ascontiguousarray(model.anchor_parent, dtype=np.float64).reshape(-1),
            np.ascontiguousarray(model.anchor_child, dtype=np.float64).reshape(-1),
            np.ascontiguousarray(model.stiffness, dtype=np.float64),
            np.ascontiguousarray(model.damping, dtype=np.float64),
            np.ascontiguousarray(model.contact_body, dtype=np.int32),
            np.ascontiguousarray(model.contact_point, dtype=np.float64).reshape(-1),
        ]
        # empty arrays still need a valid pointer
        self._keep = [k if k.size else np.zeros(1, dtype=k.dtype) for k in self._keep]
        k = self._keep
        self.s = _OModel(model.nb, model.nj, model.nc, *[a.ctypes.data for a in k],
                         model.gravity, model.terrain_amplitude, model.terrain_wavenumber)
        self.nb, self.nj, self.nc = model.nb, model.nj, model.nc
        self.nx = 6 * model.nb + model.nc + 1
        self.n = 6 * model.nb
        self.m = 3 * model.nj + 3 * model.nc
        self.np = model.nb + 2

    @property
    def ref(self):
        return ctypes.byref(self.s)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def rhs_jac(model, x, u, ubar, p):
    """F~ and the dense Jacobians (Jx, Ju, Jubar, Jp) at one point."""
    om = OracleModel(model)
    lib = _load()
    x, u, ubar, p = _f64(x), _f64(u), _f64(ubar), _f64(p)
    F = np.zeros(om.nx)
    Jx = np.zeros((om.nx, om.nx))
    Ju = np.zeros((om.nx, max(om.m, 1)))
    Jub = np.zeros((om.nx, max(om.m, 1)))
    Jp = np.zeros((om.nx, om.np))
    if u.size == 0:
        u = np.zeros(1); ubar = np.zeros(1)
    lib.oracle_rhs_jac(om.ref, _ptr(x), _ptr(u), _ptr(ubar), _ptr(p), _ptr(F), _ptr(Jx),
                       _ptr(Ju), _ptr(Jub), _ptr(Jp))
    return F, Jx, Ju[:, :om.m], Jub[:, :om.m], Jp


def integrate(model, x0, Uk, Uk1, s, p, K, tau0=0.0, tau1=1.0):
    """One interval (or sub-interval) with variational equations.

    Returns dict xf, Phi [nx,nx], Bm, Bp [nx,m], S [nx], Pi [nx,np].
    """
    om = OracleModel(model)
    lib = _load()
    nx, m, npar = om.nx, om.m, om.np
    x0, p = _f64(x0), _f64(p)
    Uk = _f64(Uk) if m else np.zeros(1)
    Uk1 = _f64(Uk1) if m else np.zeros(1)
    out = dict(xf=np.zeros(nx), Phi=np.zeros((nx, nx)), Bm=np.zeros((nx, max(m, 1))),
               Bp=np.zeros((nx, max(m, 1))), S=np.zeros(nx), Pi=np.zeros((nx, npar)))
    lib.oracle_integrate(om.ref, _ptr(x0), _ptr(Uk), _ptr(Uk1), float(s), _ptr(p),
                         float(tau0), float(tau1), int(K), _ptr(out["xf"]), _ptr(out["Phi"]),
                         _ptr(out["Bm"]), _ptr(out["Bp"]), _ptr(out["S"]), _ptr(out["Pi"]))
    out["Bm"] = out["Bm"][:, :m]
    out["Bp"] = out["Bp"][:, :m]
    return out


def discretize(model, X, U, s, p, K, nthreads=0, param_sens=False):
    """All intervals: A[N,nx,nx], Bm/Bp[N,nx,m], S[N,nx], d[N,nx], xprop[N,nx] (+Pi)."""
    om = OracleModel(model)
    lib = _load()
    X, s, p = _f64(X), _f64(s), _f64(p)
    N = X.shape[0] - 1
    nx, m, npar = om.nx, om.m, om.np
    U = _f64(U) if m else np.zeros((N + 1, 1))
    mm = max(m, 1)
    out = dict(A=np.zeros((N, nx, nx)), Bm=np.zeros((N, nx, mm)), Bp=np.zeros((N, nx, mm)),
               S=np.zeros((N, nx)), d=np.zeros((N, nx)), xprop=np.zeros((N, nx)))
    Pi = np.zeros((N, nx, npar)) if param_sens else None
    if m == 0:
        # the C code indexes U with stride m = 0: pass a dummy array
        U = np.zeros((N + 1, 1))
    lib.oracle_discretize(om.ref, N, int(K), _ptr(X), _ptr(U), _ptr(s), _ptr(p),
                          _ptr(out["A"]), _ptr(out["Bm"]) if m else None,
                          _ptr(out["Bp"]) if m else None, _ptr(out["S"]), _ptr(out["d"]),
                          _ptr(out["xprop"]), _ptr(Pi), int(nthreads))
    out["Bm"] = out["Bm"][:, :, :m]
    out["Bp"] = out["Bp"][:, :, :m]
    if param_sens:
        out["Pi"] = Pi
    return out


def defects(model, X, U, s, p, K, nthreads=0):
    om = OracleModel(model)
    lib = _load()
    X, s, p = _f64(X), _f64(s), _f64(p)
    N = X.shape[0] - 1
    U = _f64(U) if om.m else np.zeros((N + 1, 1))
    d = np.zeros((N, om.nx))
    xp = np.zeros((N, om.nx))
    lib.oracle_defects(om.ref, N, int(K), _ptr(X), _ptr(U), _ptr(s), _ptr(p), _ptr(d),
                       _ptr(xp), int(nthreads))
    return dict(d=d, xprop=xp)


def adjoint(model, X, U, s, p, K, lam, nthreads=0):
    """VJP of (X, U, s, p) -> F~ with seed lam[N, nx]: gX[N+1,nx], gU[N+1,m], gs[N], gp[P]."""
    om = OracleModel(model)
    lib = _load()
    X, s, p, lam = _f64(X), _f64(s), _f64(p), _f64(lam)
    N = X.shape[0] - 1
    m = om.m
    U = _f64(U) if m else np.zeros((N + 1, 1))
    gX = np.zeros((N + 1, om.nx))
    gU = np.zeros((N + 1, max(m, 1)))
    gs = np.zeros(N)
    gp = np.zeros(om.np)
    lib.oracle_adjoint(om.ref, N, int(K), _ptr(X), _ptr(U), _ptr(s), _ptr(p), _ptr(lam),
                       _ptr(gX), _ptr(gU), _ptr(gs), _ptr(gp), int(nthreads))
    return dict(gX=gX, gU=gU[:, :m], gs=gs, gp=gp)


def rkf_tableau():
    """The Fehlberg 4(5) tableau the oracle integrates with: c[6], a[6, 6], b[6]
    (propagated, fourth order), bh[6] (embedded, fifth order)."""
    lib = _load()
    c, a, b, bh = np.zeros(6), np.zeros((6, 6)), np.zeros(6), np.zeros(6)
    lib.oracle_rkf_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bh))
    return c, a, b, bh


def integrate_erk(model, x0, Uk, Uk1, s, p, K, c, a, b, bh=None, tau0=0.0, tau1=1.0):
    """One interval with K steps of an explicit Runge-Kutta tableau and the
    variational equations: dict xf, Phi, Bm, Bp, S, err."""
    om = OracleModel(model)
    lib = _load()
    nx, m = om.nx, om.m
    c, a, b = _f64(c), _f64(a), _f64(b)
    bh = None if bh is None else _f64(bh)
    x0, p = _f64(x0), _f64(p)
    Uk = _f64(Uk) if m else np.zeros(1)
    Uk1 = _f64(Uk1) if m else np.zeros(1)
    out = dict(xf=np.zeros(nx), Phi=np.zeros((nx, nx)), Bm=np.zeros((nx, max(m, 1))),
               Bp=np.zeros((nx, max(m, 1))), S=np.zeros(nx))
    err = np.zeros(1)
    lib.oracle_integrate_erk(om.ref, _ptr(x0), _ptr(Uk), _ptr(Uk1), float(s), _ptr(p),
                             float(tau0), float(tau1), int(K), int(c.size), _ptr(c), _ptr(a),
                             _ptr(b), _ptr(bh), _ptr(out["xf"]), _ptr(out["Phi"]),
                             _ptr(out["Bm"]), _ptr(out["Bp"]), _ptr(out["S"]), _ptr(err))
    out["Bm"] = out["Bm"][:, :m]
    out["Bp"] = out["Bp"][:, :m]
    out["err"] = float(err[0])
    return out


def discretize_rkf(model, X, U, s, p, K, nthreads=0):
    """All intervals with K Fehlberg steps each: A, Bm, Bp, S, d, xprop as in
    discretize, and err[N] (largest embedded estimate over the steps)."""
    om = OracleModel(model)
    lib = _load()
    X, s, p = _f64(X), _f64(s), _f64(p)
    N = X.shape[0] - 1
    nx, m = om.nx, om.m
    U = _f64(U) if m else np.zeros((N + 1, 1))
    mm = max(m, 1)
    out = dict(A=np.zeros((N, nx, nx)), Bm=np.zeros((N, nx, mm)), Bp=np.zeros((N, nx, mm)),
               S=np.zeros((N, nx)), d=np.zeros((N, nx)), xprop=np.zeros((N, nx)),
               err=np.zeros(N))
    lib.oracle_discretize_rkf(om.ref, N, int(K), _ptr(X), _ptr(U), _ptr(s), _ptr(p),
                              _ptr(out["A"]), _ptr(out["Bm"]) if m else None,
                              _ptr(out["Bp"]) if m else None, _ptr(out["S"]), _ptr(out["d"]),
                              _ptr(out["xprop"]), _ptr(out["err"]), int(nthreads))
    out["Bm"] = out["Bm"][:, :, :m]
    out["Bp"] = out["Bp"][:, :, :m]
    return out
