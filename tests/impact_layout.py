"""Compact impact-Jacobian layout of include/cis.h, expanded to the dense
Jacobians of the oracle (test helper; no arithmetic of the method)."""
import numpy as np

from paper_2604_09993_amd import api


def compact_from_dense(model, JG, JT):
    """JGv [n, 3 nb, 7 nb + 2 nc] and JTc [n, 10 nc, 14] taken from dense
    JG [n, nx, nz], JT [n, 10 nc, nz]."""
    jgv, jtc = api.impact_columns(model)
    nq = 3 * model.nb
    JGv = JG[:, nq:2 * nq][:, :, jgv]
    JTc = np.zeros((JT.shape[0], 10 * model.nc, 14))
    for i in range(model.nc):
        JTc[:, 10 * i:10 * i + 10] = JT[:, 10 * i:10 * i + 10][:, :, jtc[i]]
    return JGv, JTc


def dense_from_compact(model, JGv, JTc):
    """The dense node Jacobians: the compact blocks plus the entries that are
    the same for every node (+I / -I on pose and integral rows, I on v+)."""
    jgv, jtc = api.impact_columns(model)
    n, nx, nq, nc = JGv.shape[0], model.nx, 3 * model.nb, model.nc
    nz = 2 * nx + 3 * nc + model.n_params
    JG = np.zeros((n, nx, nz))
    for r in list(range(nq)) + list(range(2 * nq, nx)):
        JG[:, r, r] = 1.0
        JG[:, r, nx + r] = -1.0
    for r in range(nq):
        JG[:, nq + r, nq + r] = 1.0
    JG[:, nq:2 * nq, jgv] += JGv
    JT = np.zeros((n, 10 * nc, nz))
    for i in range(nc):
        JT[:, 10 * i:10 * i + 10, jtc[i]] = JTc[:, 10 * i:10 * i + 10]
    return JG, JT
