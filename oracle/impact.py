"""CPU FP64 oracle of the node-level impact map and its linearization.

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing else; it shares
no code with the HIP path.  Plain, dense numpy, written to be checked against
the paper by eye (arxiv 2604.09993):

* velocity jump with the joint impulse eliminated (Sec. II-B,
  eq. impulse-dynamics:velocity-change, with the joint constraint imposed
  after the impact at the velocity level, grad h(q) v+ = 0) and the
  continuity of pose and integral states: the node equality G~(x~+, x~-, Phi)
  of eq. cito-impulse;
* the impact conditions eq. impulse-dynamics:no-penetration,
  eq. elasticity-impact, eq. max-diss-impulse-KKT:stationarity and
  eq. impulse-friction-cone, relaxed with the Fischer-Burmeister function
  of eq. FB-relax and collected into Theta^delta(x+, x-, Phi, Gamma) <= 0;
* Psi^{delta, eps}: the interval increments of the integral states
  (relaxed cross-complementarity and continuous-time violation, eq. ctcs-relax).

Jacobians are taken by complex-step differentiation of the same residual
functions (f'(z) e_j = Im f(z + i h e_j) / h with h = 1e-30: exact up to the
rounding of f, no subtraction), a library-level step independent of any
hand-derived formula.  Readings where the paper is silent are listed in the
functions that take them.

Arrays are node-major: X[n_nodes, nx]; Phi[n_nodes, 2 nc] ordered
(Phi_t_1, Phi_n_1, Phi_t_2, ...); Gamma[n_nodes, nc]; p = (mu, e, masses).
"""
from __future__ import annotations

import numpy as np

N_THETA_PER_CONTACT = 10


def sabs(a):
    """Pseudo-Huber absolute value with unit steepness, sqrt(a^2 + 1) - 1 (Sec. II
    notation; in the plane the smooth norm of a scalar is the same function)."""
    return np.sqrt(a * a + 1.0) - 1.0


def fb(a, b, delta):
    """Fischer-Burmeister relaxation FB^delta(a, b) = a + b - sqrt(a^2 + b^2 + delta)
    (eq. FB-relax)."""
    return a + b - np.sqrt(a * a + b * b + delta)


def _rot(th):
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s], [s, c]])


def _cross(a, f):
    return a[0] * f[1] - a[1] * f[0]


def _terrain(model, P):
    """Contact frame at world point P: signed distance sd = H / |grad H| with
    H = P_y - A sin(kappa P_x) (Sec. VI-B), normal n = grad H / |grad H|,
    tangent t = (n_y, -n_x) (right-handed [t n])."""
    A, kap = model.terrain_amplitude, model.terrain_wavenumber
    H = P[1] - A * np.sin(kap * P[0])
    Hx = -A * kap * np.cos(kap * P[0])
    G = np.sqrt(1.0 + Hx * Hx)
    n = np.array([Hx / G, 1.0 / G])
    t = np.array([n[1], -n[0]])
    return H / G, n, t


def _split(model, x):
    nb = model.nb
    q = x[:3 * nb].reshape(nb, 3)
    v = x[3 * nb:6 * nb].reshape(nb, 3)
    y = x[6 * nb:]
    return q, v, y


def joint_jacobian(model, q):
    """grad h(q) [2 nj, 3 nb]: h_j = p_p + R(th_p) r_p - p_c - R(th_c) r_c (Sec. II-A)."""
    nb, nj = model.nb, model.nj
    Jh = np.zeros((2 * nj, 3 * nb), dtype=q.dtype)
    E = np.array([[0.0, -1.0], [1.0, 0.0]])
    for j in range(nj):
        p, c = int(model.joint_parent[j]), int(model.joint_child[j])
        ap = _rot(q[p, 2]) @ model.anchor_parent[j]
        ac = _rot(q[c, 2]) @ model.anchor_child[j]
        Jh[2 * j:2 * j + 2, 3 * p:3 * p + 2] = np.eye(2)
        Jh[2 * j:2 * j + 2, 3 * p + 2] = E @ ap
        Jh[2 * j:2 * j + 2, 3 * c:3 * c + 2] = -np.eye(2)
        Jh[2 * j:2 * j + 2, 3 * c + 2] = -(E @ ac)
    return Jh


def contact_jacobian(model, q, i):
    """J_i(q) = d P_i / d q [2, 3 nb] of contact point P_i = p_b + R(th_b) r_i."""
    b = int(model.contact_body[i])
    a = _rot(q[b, 2]) @ model.contact_point[i]
    J = np.zeros((2, 3 * model.nb), dtype=q.dtype)
    J[:, 3 * b:3 * b + 2] = np.eye(2)
    J[:, 3 * b + 2] = np.array([-a[1], a[0]])
    return J, q[b, :2] + a


def mass_inverse(model, p):
    """Diagonal of M^-1 [3 nb]: M = diag(m, m, I) per body, I = m L^2 / 12 (R10)."""
    m = p[2:]
    inertia = m * model.link_length ** 2 / 12.0
    return np.stack([1.0 / m, 1.0 / m, 1.0 / inertia], axis=1).reshape(-1)


def post_impact_velocity(model, q, vm, Phi, p):
    """v* solving M (v* - v-) = J^T R Phi + grad h^T Lambda together with
    grad h(q) v* = 0 (Sec. II-B: the joint impulse Lambda eliminated).
    Reading: every geometric term is evaluated at the post-impact pose q
    (the velocity constraint is stated there; the pose is continuous)."""
    nb, nc = model.nb, model.nc
    Minv = mass_inverse(model, p)
    gen = np.zeros(3 * nb, dtype=np.result_type(q, vm, Phi, p))
    for i in range(nc):
        J, P = contact_jacobian(model, q, i)
        _, n, t = _terrain(model, P)
        F = t * Phi[2 * i] + n * Phi[2 * i + 1]   # R Phi, world frame
        gen = gen + J.T @ F
    f = vm.reshape(-1) + Minv * gen
    if model.nj == 0:
        return f
    Jh = joint_jacobian(model, q)
    A = Jh @ (Minv[:, None] * Jh.T)
    lam = -np.linalg.solve(A, Jh @ f)
    return f + Minv * (Jh.T @ lam)


def G_tilde(model, xp, xm, Phi, p):
    """Node equality G~(x~+, x~-, Phi) of eq. cito-impulse: pose and integral
    states continuous, velocities jump by the impact map."""
    qp, vp, yp = _split(model, xp)
    qm, vm, ym = _split(model, xm)
    vstar = post_impact_velocity(model, qp, vm, Phi, p)
    return np.concatenate([(qp - qm).reshape(-1), vp.reshape(-1) - vstar, yp - ym])


def theta(model, xp, xm, Phi, Gam, p, delta):
    """Impact conditions relaxed with FB^delta, per contact (10 rows each):

      FB(Phi_n, sd), FB(Phi_n, w), Phi_n lam - delta, -Phi_n lam - delta, FB(Gamma, rho),
      -Phi_n, -sd, -w, -Gamma, -rho,

    with w = n^T J (v+ + e v-) (eq. elasticity-impact as a complementarity of
    the normal impulse and the restitution-weighted normal velocity), lam = the
    post-impact tangential velocity + Gamma dsmoothnorm(Phi_t) (the bracket of
    eq. max-diss-impulse-KKT:stationarity, whose product with Phi_n must vanish:
    relaxed as |Phi_n lam| <= delta), rho = |mu Phi_n|_s - ||Phi_t||_s
    (eq. impulse-friction-cone).  Readings: geometry at the post-impact pose;
    the stationarity product relaxed by delta in both signs."""
    qp, vp, _ = _split(model, xp)
    _, vm, _ = _split(model, xm)
    mu, e = p[0], p[1]
    rows = []
    for i in range(model.nc):
        J, P = contact_jacobian(model, qp, i)
        sd, n, t = _terrain(model, P)
        pn, pt, gam = Phi[2 * i + 1], Phi[2 * i], Gam[i]
        w = n @ (J @ (vp.reshape(-1) + e * vm.reshape(-1)))
        vt = t @ (J @ vp.reshape(-1))
        lam = vt + gam * pt / np.sqrt(pt * pt + 1.0)
        rho = sabs(mu * pn) - sabs(pt)
        rows += [fb(pn, sd, delta), fb(pn, w, delta), pn * lam - delta, -pn * lam - delta,
                 fb(gam, rho, delta), -pn, -sd, -w, -gam, -rho]
    return np.array(rows)


def psi(model, y_plus_k, y_minus_k1, delta, eps):
    """Psi^{delta, eps}(y-_{k+1}, y+_k) <= 0 for the integral states of this
    build (one cross-complementarity state per contact and one violation state):
    the increment of each cross-complementarity state (a sum of products of
    nonnegative integrals) at most delta, the violation increment at most eps
    (eq. ctcs-relax)."""
    dy = np.asarray(y_minus_k1) - np.asarray(y_plus_k)
    nc = model.nc
    return np.concatenate([dy[:nc] - delta, dy[nc:] - eps])


def n_dirs(model):
    """Directions of the node linearization: z = (x~+, x~-, Phi, Gamma, p)."""
    return 2 * model.nx + 3 * model.nc + model.n_params


def _node_residuals(model, z, delta):
    nx, nc = model.nx, model.nc
    xp, xm = z[:nx], z[nx:2 * nx]
    Phi = z[2 * nx:2 * nx + 2 * nc]
    Gam = z[2 * nx + 2 * nc:2 * nx + 3 * nc]
    p = z[2 * nx + 3 * nc:]
    return G_tilde(model, xp, xm, Phi, p), theta(model, xp, xm, Phi, Gam, p, delta)


def linearize(model, Xp, Xm, Phi, Gam, p, delta):
    """Per node: G~ [nx], Theta [10 nc] and their Jacobians with respect to
    z = (x~+, x~-, Phi, Gamma, p): JG [nx, nz], JT [10 nc, nz].  Node-major
    arrays in, dict of arrays [n_nodes, ...] out."""
    Xp, Xm = np.atleast_2d(Xp), np.atleast_2d(Xm)
    Phi, Gam = np.atleast_2d(Phi), np.atleast_2d(Gam)
    nn = Xp.shape[0]
    nz = n_dirs(model)
    nt = N_THETA_PER_CONTACT * model.nc
    out = {"G": np.zeros((nn, model.nx)), "Theta": np.zeros((nn, nt)),
           "JG": np.zeros((nn, model.nx, nz)), "JT": np.zeros((nn, nt, nz))}
    h = 1e-30
    for k in range(nn):
        z = np.concatenate([Xp[k], Xm[k], Phi[k], Gam[k], p]).astype(np.float64)
        g, th = _node_residuals(model, z, delta)
        out["G"][k], out["Theta"][k] = g, th
        for j in range(nz):
            zc = z.astype(np.complex128)
            zc[j] += 1j * h
            gc, tc = _node_residuals(model, zc, delta)
            out["JG"][k, :, j] = np.imag(gc) / h
            out["JT"][k, :, j] = np.imag(tc) / h
    return out
