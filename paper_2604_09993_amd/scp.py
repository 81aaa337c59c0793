"""Sequential convex programming driver of the contact-implicit problem.

arxiv 2604.09993: the transcribed problem eq. cito-problem (Sec. IV-C), solved
by the prox-linear method with exact l1 penalization of the nonconvex
constraints (Sec. V), with the tightness parameter delta of eq. FB-relax
driven by the embedded delta-homotopy with backtracking (Sec. V, Alg. 1), and
controls parameterized by a first-order hold that may jump at the nodes
(Sec. VI).

Decision variables (per node k = 0..N: post- and pre-impact augmented states
x~+_k, x~-_k, impulses Phi_k, multipliers Gamma_k; per interval k = 0..N-1:
the hold's end values Ua_k, Ub_k and the dilation S_k).  Each iteration

  1. transcribes the iterate on the GPU: one discretize call over the
     intervals (dynamics eq. cito-augdyn and its sensitivities; the
     discontinuous hold is laid out as 2N intervals over the node sequence
     x~+_0, x~-_1, x~+_1, ..., x~-_N, x~+_N whose odd intervals are not
     used) and one impact-map call over the nodes (G~, Theta^delta,
     Psi^{delta,eps} and their Jacobians, eq. cito-impulse);
  2. assembles the convex subproblem: quadratic cost (squared joint torques
     along the hold), proximal term w_px/2 ||dz||^2 on scaled variables,
     linearized dynamics and node equalities with l1-penalized virtual
     controls, linearized Theta and Psi with l1-penalized positive parts,
     the convex control set (torque bounds, nonnegative contact forces inside
     the planar friction cone), dilation bounds and boundary states;
  3. solves it with the interior-point QP solver of this package (the
     planar cones are polyhedral) and takes the solution as the next
     iterate;
  4. updates delta by Alg. 1 from the proximal and penalty terms.

The GPU transcriber is the product path; any object with the same call
(returning the same arrays) can stand in for it.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .qp import solve_qp

N_THETA = 10   # Theta rows per contact


# ---------------------------------------------------------------------------
# Problem layout
# ---------------------------------------------------------------------------
@dataclass
class CitoProblem:
    """A contact-implicit trajectory problem of a planar model: N intervals,
    boundary states, bounds, weights and the transcription settings."""
    model: object
    N: int
    x_init: np.ndarray                 # [nx] pre-impact state at node 0 (q, v, y = 0)
    x_final: np.ndarray                # [nx] post-impact pose and velocity at node N
    K: int = 10                        # integration steps per interval (Sec. VI)
    tau_max: float = 50.0              # joint torque bound
    s_min: float = 0.02                # dilation bounds (interval length, s)
    s_max: float = 0.10
    eps_ctcs: float = 1e-4             # bound of the violation-state increment
    w_cost: float = 1.0                # weight of the squared scaled torques
    mu: float = 1.0                    # friction coefficient (the experiments' value, Sec. VI)
    e: float = 0.0                     # restitution (the experiments' value, Sec. VI)
    scales: dict = field(default_factory=dict)

    def __post_init__(self):
        m = self.model
        self.nx, self.m, self.nc, self.nb, self.nj = m.nx, m.m, m.nc, m.nb, m.nj
        self.ny = m.ny
        self.nq = 3 * m.nb
        self.NB = 2 * self.nx + 3 * self.nc          # node block
        self.IB = 2 * self.m + 1                      # interval block
        self.nz = (self.N + 1) * self.NB + self.N * self.IB
        self.p = m.params(mu=self.mu, e=self.e)
        sc = dict(q=1.0, v=2.0, y=1.0, phi=1.0, gam=1.0, tau=self.tau_max / 2.0,
                  jf=20.0, cf=20.0, s=0.05)
        sc.update(self.scales)
        self.scales = sc
        xs = np.concatenate([np.full(self.nq, sc["q"]), np.full(self.nq, sc["v"]),
                             np.full(self.ny, sc["y"])])
        us = np.concatenate([np.full(self.nj, sc["tau"]), np.full(2 * self.nj, sc["jf"]),
                             np.full(3 * self.nc, sc["cf"])])
        self.xscale = xs
        node = np.concatenate([xs, xs, np.full(2 * self.nc, sc["phi"]), np.full(self.nc, sc["gam"])])
        ivl = np.concatenate([us, us, [sc["s"]]])
        self.zscale = np.concatenate([np.tile(node, self.N + 1), np.tile(ivl, self.N)])

    # index maps of the decision vector
    def node(self, k):
        return k * self.NB

    def ivl(self, k):
        return (self.N + 1) * self.NB + k * self.IB

    def unpack(self, z):
        N, nx, nc, m = self.N, self.nx, self.nc, self.m
        nodes = z[:(N + 1) * self.NB].reshape(N + 1, self.NB)
        ivls = z[(N + 1) * self.NB:].reshape(N, self.IB)
        return dict(Xp=nodes[:, :nx], Xm=nodes[:, nx:2 * nx],
                    Phi=nodes[:, 2 * nx:2 * nx + 2 * nc], Gamma=nodes[:, 2 * nx + 2 * nc:],
                    Ua=ivls[:, :m], Ub=ivls[:, m:2 * m], S=ivls[:, 2 * m])

    def pack(self, Xp, Xm, Phi, Gamma, Ua, Ub, S):
        N = self.N
        nodes = np.concatenate([Xp, Xm, Phi, Gamma], axis=1)
        ivls = np.concatenate([Ua, Ub, np.asarray(S).reshape(N, 1)], axis=1)
        return np.concatenate([nodes.reshape(-1), ivls.reshape(-1)])

    def doubled(self, v):
        """Node-doubled arrays of the discontinuous hold: states
        [x~+_0, x~-_1, x~+_1, ..., x~-_N, x~+_N] [2N+1, nx], controls
        [Ua_0, Ub_0, Ua_1, ..., Ub_{N-1}, Ub_{N-1}] [2N+1, m], dilations
        [S_0, S_0, S_1, ...] [2N]; interval 2k is interval k of the problem."""
        N = self.N
        Xd = np.empty((2 * N + 1, self.nx))
        Xd[0::2] = v["Xp"]
        Xd[1::2] = v["Xm"][1:]
        Ud = np.empty((2 * N + 1, self.m))
        Ud[0:2 * N:2] = v["Ua"]
        Ud[1::2] = v["Ub"]
        Ud[2 * N] = v["Ub"][-1]
        sd = np.repeat(np.asarray(v["S"], dtype=np.float64), 2)
        return Xd, Ud, sd


# ---------------------------------------------------------------------------
# GPU transcription
# ---------------------------------------------------------------------------
def expand_node_jacobians(model, JGv, JTc):
    """Dense node Jacobians over (x~+, x~-, Phi, Gamma) from the compact
    impact-map outputs (the layout of cis_impact_linearize: constant blocks
    +-I on the pose and integral rows, I on v+, JGv over (q+, v-, Phi,
    masses) on the velocity rows, JTc over (q+_b, v+_b, v-_b, Phi_t_i,
    Phi_n_i, Gamma_i, mu, e) on the rows of contact i)."""
    nb, nc, nx = model.nb, model.nc, model.nx
    nq = 3 * nb
    nn = JGv.shape[0]
    NB = 2 * nx + 3 * nc
    phi0, gam0 = 2 * nx, 2 * nx + 2 * nc
    JG = np.zeros((nn, nx, NB))
    r = np.arange(nq)
    JG[:, r, r] = 1.0
    JG[:, r, nx + r] = -1.0
    ry = 2 * nq + np.arange(nx - 2 * nq)
    JG[:, ry, ry] = 1.0
    JG[:, ry, nx + ry] = -1.0
    rv = nq + np.arange(nq)
    JG[:, rv, rv] = 1.0
    JG[:, nq:2 * nq, 0:nq] += JGv[:, :, 0:nq]
    JG[:, nq:2 * nq, nx + nq:nx + 2 * nq] += JGv[:, :, nq:2 * nq]
    JG[:, nq:2 * nq, phi0:phi0 + 2 * nc] += JGv[:, :, 2 * nq:2 * nq + 2 * nc]
    JT = np.zeros((nn, N_THETA * nc, NB))
    for i in range(nc):
        b = int(model.contact_body[i])
        rows = slice(N_THETA * i, N_THETA * (i + 1))
        cols = np.concatenate([3 * b + np.arange(3), nq + 3 * b + np.arange(3),
                               nx + nq + 3 * b + np.arange(3),
                               [phi0 + 2 * i, phi0 + 2 * i + 1, gam0 + i]])
        JT[:, rows, cols] = JTc[:, rows, :12]
    return JG, JT


class GpuTranscriber:
    """Transcription of an iterate with the HIP kernels: cis_discretize (or
    cis_discretize_rkf) over the node-doubled intervals and
    cis_impact_linearize over the nodes, FP64 on `device`."""

    def __init__(self, problem: CitoProblem, integrator="rk4", device="cuda"):
        import torch
        from . import api
        self._torch, self._api = torch, api
        self.pb = problem
        self.integrator = integrator
        self.device = device
        self.cm = api.CisModel(problem.model)
        self.p = torch.from_numpy(problem.p).to(device)
        self.ws = None
        if integrator == "rkf":
            nbytes = api.rkf_workspace_bytes(self.cm, 2 * problem.N, problem.K)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        elif integrator != "rk4":
            raise ValueError("integrator must be 'rk4' or 'rkf'")

    def __call__(self, v, delta):
        torch, api, pb = self._torch, self._api, self.pb
        N = pb.N
        Xd, Ud, sd = pb.doubled(v)
        dev = self.device
        X = api.to_device_soa(Xd, dev)
        U = api.to_device_soa(Ud, dev)
        s = torch.from_numpy(sd).to(dev)
        if self.integrator == "rk4":
            out = api.discretize(self.cm, X, U, s, self.p, pb.K, with_xprop=False)
        else:
            out = api.discretize_rkf(self.cm, X, U, s, self.p, pb.K, with_xprop=False, ws=self.ws)
        Xp = api.to_device_soa(v["Xp"], dev)
        Xm = api.to_device_soa(v["Xm"], dev)
        Phi = api.to_device_soa(v["Phi"], dev)
        Gam = api.to_device_soa(v["Gamma"], dev)
        imp = api.impact_linearize(self.cm, Xp, Xm, Phi, Gam, self.p, delta, pb.eps_ctcs)
        host = {k: t[..., 0::2].cpu().numpy() for k, t in out.items()
                if t is not None and k in ("A", "Bm", "Bp", "S", "d")}
        res = dict(A=np.moveaxis(host["A"], 2, 0), Bm=np.moveaxis(host["Bm"], 2, 0),
                   Bp=np.moveaxis(host["Bp"], 2, 0), S=host["S"].T, d=host["d"].T)
        assert res["A"].shape[0] == N
        JG, JT = expand_node_jacobians(pb.model, imp["JGv"].cpu().numpy(),
                                       imp["JTc"].cpu().numpy())
        res.update(G=imp["G"].cpu().numpy(), Theta=imp["Theta"].cpu().numpy(), JG=JG, JT=JT,
                   Psi=imp["Psi"].cpu().numpy())
        return res


# ---------------------------------------------------------------------------
# Subproblem assembly (Sec. V: prox-linear with exact l1 penalties)
# ---------------------------------------------------------------------------
class _Triplets:
    def __init__(self):
        self.r, self.c, self.v = [], [], []

    def add(self, rows, cols, vals):
        rows, cols, vals = np.broadcast_arrays(np.asarray(rows), np.asarray(cols),
                                               np.asarray(vals, dtype=np.float64))
        self.r.append(rows.ravel())
        self.c.append(cols.ravel())
        self.v.append(vals.ravel())

    def matrix(self, nrows, ncols):
        if not self.r:
            return sp.csr_matrix((nrows, ncols))
        return sp.csr_matrix((np.concatenate(self.v), (np.concatenate(self.r),
                                                       np.concatenate(self.c))),
                             shape=(nrows, ncols))


def _dense_block(T, rows, cols, block):
    """Add the nonzeros of a dense block at (rows, cols)."""
    nz = np.nonzero(block)
    T.add(rows[nz[0]], cols[nz[1]], block[nz])


@dataclass
class Subproblem:
    P: sp.csr_matrix
    q: np.ndarray
    A: sp.csr_matrix
    b: np.ndarray
    G: sp.csr_matrix
    h: np.ndarray
    n_z: int
    n_pen: int          # penalty variables after the scaled step


def assemble(pb: CitoProblem, z, tr, w_px, w_ep):
    """The convex subproblem at iterate z from transcription tr, in the
    scaled step dzh (dz = zscale * dzh) followed by the penalty variables
    [nu_dyn+, nu_dyn-, nu_G+, nu_G-, t_Theta, t_Psi] (all >= 0)."""
    N, nx, m, nc, nq, ny = pb.N, pb.nx, pb.m, pb.nc, pb.nq, pb.ny
    NB, nz = pb.NB, pb.nz
    D = pb.zscale
    nth = N_THETA * nc
    o_nd = nz
    o_ng = o_nd + 2 * N * nx
    o_tt = o_ng + 2 * (N + 1) * nx
    o_tp = o_tt + (N + 1) * nth
    nw = o_tp + N * ny
    v = pb.unpack(z)

    # ---- equalities -------------------------------------------------------
    Te, be = _Triplets(), []
    row = 0
    xs = pb.xscale
    for k in range(N):   # linearized dynamics (eq. cito-augdyn), rows scaled by the state scales
        rows = row + np.arange(nx)
        n0, i0, n1 = pb.node(k), pb.ivl(k), pb.node(k + 1)
        blk = np.concatenate([tr["A"][k], tr["Bm"][k], tr["Bp"][k], tr["S"][k][:, None]], axis=1)
        cols = np.concatenate([n0 + np.arange(nx), i0 + np.arange(2 * m + 1)])
        _dense_block(Te, rows, cols, blk * D[cols][None, :] / xs[:, None])
        Te.add(rows, n1 + nx + np.arange(nx), -D[n1 + nx + np.arange(nx)] / xs)
        Te.add(rows, o_nd + k * nx + np.arange(nx), -1.0)
        Te.add(rows, o_nd + N * nx + k * nx + np.arange(nx), 1.0)
        be.append(-tr["d"][k] / xs)
        row += nx
    for k in range(N + 1):   # node equalities G~ (eq. cito-impulse)
        rows = row + np.arange(nx)
        cols = pb.node(k) + np.arange(NB)
        _dense_block(Te, rows, cols, tr["JG"][k] * D[cols][None, :] / xs[:, None])
        Te.add(rows, o_ng + k * nx + np.arange(nx), -1.0)
        Te.add(rows, o_ng + (N + 1) * nx + k * nx + np.arange(nx), 1.0)
        be.append(-tr["G"][k] / xs)
        row += nx
    # boundary states: x~-_0 = x_init (pose, velocity, integral states zero),
    # pose and velocity of x~+_N = x_final
    c0 = pb.node(0) + nx + np.arange(nx)
    Te.add(row + np.arange(nx), c0, D[c0])
    be.append(pb.x_init - v["Xm"][0])
    row += nx
    cN = pb.node(N) + np.arange(2 * nq)
    Te.add(row + np.arange(2 * nq), cN, D[cN])
    be.append(pb.x_final[:2 * nq] - v["Xp"][N][:2 * nq])
    row += 2 * nq
    A = Te.matrix(row, nw)
    b = np.concatenate(be)

    # ---- inequalities -----------------------------------------------------
    Ti, hi = _Triplets(), []
    row = 0
    for k in range(N + 1):   # Theta^delta <= t (eq. cito-problem, node conditions)
        if nth == 0:
            break
        rows = row + np.arange(nth)
        cols = pb.node(k) + np.arange(NB)
        _dense_block(Ti, rows, cols, tr["JT"][k] * D[cols][None, :])
        Ti.add(rows, o_tt + k * nth + np.arange(nth), -1.0)
        hi.append(-tr["Theta"][k])
        row += nth
    for k in range(N):       # Psi^{delta,eps} <= t (increments of the integral states)
        rows = row + np.arange(ny)
        cy1 = pb.node(k + 1) + nx + 2 * nq + np.arange(ny)     # y-_{k+1}
        cy0 = pb.node(k) + 2 * nq + np.arange(ny)              # y+_k
        Ti.add(rows, cy1, D[cy1])
        Ti.add(rows, cy0, -D[cy0])
        Ti.add(rows, o_tp + k * ny + np.arange(ny), -1.0)
        hi.append(-tr["Psi"][k])
        row += ny
    npen = nw - nz           # penalty variables are nonnegative
    Ti.add(row + np.arange(npen), nz + np.arange(npen), -1.0)
    hi.append(np.zeros(npen))
    row += npen
    # convex control set: |tau| <= tau_max, contact forces >= 0 and inside the
    # planar friction cone mu lam_n - lam_t+ - lam_t- >= 0; dilation bounds
    mu = pb.p[0]
    nj = pb.nj
    for k in range(N):
        for side, U in ((0, v["Ua"][k]), (1, v["Ub"][k])):
            c = pb.ivl(k) + side * m
            for j in range(nj):
                Ti.add([row, row + 1], [c + j, c + j], [D[c + j], -D[c + j]])
                hi.append([pb.tau_max - U[j], pb.tau_max + U[j]])
                row += 2
            for i in range(nc):
                cn, cp, cm_ = c + 3 * nj + 3 * i, c + 3 * nj + 3 * i + 1, c + 3 * nj + 3 * i + 2
                Ti.add([row, row + 1, row + 2], [cn, cp, cm_], [-D[cn], -D[cp], -D[cm_]])
                hi.append([U[3 * nj + 3 * i], U[3 * nj + 3 * i + 1], U[3 * nj + 3 * i + 2]])
                Ti.add([row + 3] * 3, [cn, cp, cm_], [-mu * D[cn], D[cp], D[cm_]])
                hi.append([mu * U[3 * nj + 3 * i] - U[3 * nj + 3 * i + 1] - U[3 * nj + 3 * i + 2]])
                row += 4
        cs = pb.ivl(k) + 2 * m
        Ti.add([row, row + 1], [cs, cs], [D[cs], -D[cs]])
        hi.append([pb.s_max - v["S"][k], v["S"][k] - pb.s_min])
        row += 2
    G = Ti.matrix(row, nw)
    h = np.concatenate([np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in hi])

    # ---- objective ----------------------------------------------------------
    # w_px/2 ||dzh||^2 + w_cost sum_k int_0^1 ||tau(t)/tau_scale||^2 dt (the hold
    # of interval k: (a^2 + a b + b^2) / 3 per joint) + w_ep (sum nu + sum t)
    Pd = np.concatenate([np.full(nz, w_px), np.zeros(nw - nz)])
    q = np.concatenate([np.zeros(nz), np.full(nw - nz, w_ep)])
    Tp = _Triplets()
    Tp.add(np.arange(nw), np.arange(nw), Pd)
    ts = pb.scales["tau"]
    for k in range(N):
        ca = pb.ivl(k) + np.arange(nj)
        cb = ca + m
        ua, ub = v["Ua"][k][:nj] / ts, v["Ub"][k][:nj] / ts
        da, db = D[ca] / ts, D[cb] / ts
        wq = pb.w_cost / 3.0
        # 1/2 x^T (2 wq [[1, 1/2], [1/2, 1]]) x over (a, b), x = u + d dzh
        Tp.add(ca, ca, 2.0 * wq * da * da)
        Tp.add(cb, cb, 2.0 * wq * db * db)
        Tp.add(ca, cb, wq * da * db)
        Tp.add(cb, ca, wq * da * db)
        q[ca] += wq * (2.0 * ua + ub) * da
        q[cb] += wq * (ua + 2.0 * ub) * db
    P = Tp.matrix(nw, nw)
    return Subproblem(P=P, q=q, A=A, b=b, G=G, h=h, n_z=nz, n_pen=nw - nz)


def control_cost(pb: CitoProblem, z):
    """sum_k int_0^1 ||tau(t) / tau_scale||^2 dt over the holds, times w_cost."""
    v = pb.unpack(z)
    ts = pb.scales["tau"]
    a, b = v["Ua"][:, :pb.nj] / ts, v["Ub"][:, :pb.nj] / ts
    return pb.w_cost * float(np.sum(a * a + a * b + b * b) / 3.0)


# ---------------------------------------------------------------------------
# Embedded delta-homotopy with backtracking (Sec. V, Alg. 1)
# ---------------------------------------------------------------------------
class DeltaHomotopy:
    """The tightness update of Alg. 1.  Histories are indexed by SCP iterate
    j: J_px[0] = J_ep[0] = 0 and delta[0] = delta0.  After the subproblem at
    iterate j returns J_px[j+1], J_ep[j+1], with M = max(j - N_stall, 1):
    if either term exceeds its value at M, delta[j+1] is the geometric mean
    of delta[j] and delta[M] (log-scale bisection); else if either exceeds
    its value at j, delta[j+1] = delta[j]; else delta[j+1] = alpha delta[j]."""

    def __init__(self, delta0=1.0, delta_min=1e-3, eps_px=1e-6, eps_ep=1e-6, alpha=0.85,
                 n_stall=10):
        if not 0.0 < alpha < 1.0 or not 0.0 < delta_min < delta0:
            raise ValueError("need 0 < alpha < 1 and 0 < delta_min < delta0")
        self.delta_min, self.eps_px, self.eps_ep = delta_min, eps_px, eps_ep
        self.alpha, self.n_stall = alpha, int(n_stall)
        self.J_px, self.J_ep, self.delta = [0.0], [0.0], [float(delta0)]

    @property
    def j(self):
        return len(self.delta) - 1

    def done(self):
        """Loop condition of Alg. 1 negated: both terms within tolerance and
        delta at or below delta_min."""
        j = self.j
        return (self.J_px[j] <= self.eps_px and self.J_ep[j] <= self.eps_ep
                and self.delta[j] <= self.delta_min)

    def update(self, J_px_new, J_ep_new):
        j = self.j
        self.J_px.append(float(J_px_new))
        self.J_ep.append(float(J_ep_new))
        M = max(j - self.n_stall, 1)
        Jp, Je, d = self.J_px, self.J_ep, self.delta
        if Jp[j + 1] > Jp[M] or Je[j + 1] > Je[M]:
            new = float(np.exp(0.5 * np.log(d[j] * d[M])))
        elif Jp[j + 1] > Jp[j] or Je[j + 1] > Je[j]:
            new = d[j]
        else:
            new = self.alpha * d[j]
        d.append(new)
        return new


# ---------------------------------------------------------------------------
# Driver
# ---------------------------------------------------------------------------
@dataclass
class ScpIteration:
    j: int
    delta: float
    J_px: float
    J_ep: float
    cost: float
    qp_status: str
    qp_iters: int
    t_transcribe: float
    t_assemble: float
    t_solve: float


class ScpDriver:
    """Prox-linear SCP with exact penalties and Alg. 1 on a CitoProblem."""

    def __init__(self, problem: CitoProblem, transcriber, *, w_px=2000.0, w_ep=5.0e4,
                 homotopy: DeltaHomotopy | None = None, qp_tol=1e-8):
        self.pb = problem
        self.tr = transcriber
        self.w_px, self.w_ep = float(w_px), float(w_ep)
        self.hom = homotopy if homotopy is not None else DeltaHomotopy()
        self.qp_tol = qp_tol
        self.qp_cache = {}     # ordering and symbolic factorization of the KKT pattern
        self.history: list[ScpIteration] = []

    def subproblem(self, z, delta):
        """One SCP step from z: (z_next, J_px, J_ep, iteration record)."""
        pb = self.pb
        t0 = time.perf_counter()
        tr = self.tr(pb.unpack(z), delta)
        t1 = time.perf_counter()
        sub = assemble(pb, z, tr, self.w_px, self.w_ep)
        t2 = time.perf_counter()
        r = solve_qp(sub.P, sub.q, sub.A, sub.b, sub.G, sub.h, tol=self.qp_tol,
                     cache=self.qp_cache)
        t3 = time.perf_counter()
        dzh = r.x[:sub.n_z]
        z_next = z + pb.zscale * dzh
        J_px = 0.5 * float(dzh @ dzh)
        J_ep = float(np.sum(r.x[sub.n_z:]))
        rec = ScpIteration(j=len(self.history), delta=delta, J_px=J_px, J_ep=J_ep,
                           cost=control_cost(pb, z_next), qp_status=r.status, qp_iters=r.iters,
                           t_transcribe=t1 - t0, t_assemble=t2 - t1, t_solve=t3 - t2)
        return z_next, J_px, J_ep, rec

    def run(self, z0, max_iter=100, callback=None):
        """Alg. 1 from z0 until its termination test or max_iter iterations."""
        z = np.asarray(z0, dtype=np.float64).copy()
        for _ in range(max_iter):
            delta = self.hom.delta[-1]
            z, J_px, J_ep, rec = self.subproblem(z, delta)
            self.hom.update(J_px, J_ep)
            self.history.append(rec)
            if callback is not None:
                callback(rec, z)
            if self.hom.done():
                break
        return z
