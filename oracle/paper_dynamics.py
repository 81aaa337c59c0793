"""CPU FP64 oracle of the paper-faithful dynamics variant and its discretization.

TEST INFRASTRUCTURE ONLY: used by the test-suite and nothing else; it shares
no code with the HIP path.  Plain numpy, written to be checked against the
paper by eye (arxiv 2604.09993):

* joint reaction forces eliminated at the acceleration level: with
  grad h(q) v' + c(q, v) = 0, c_j = v^T grad^2 h_j v, and the equations of
  motion M v' = W + J^T R phi + grad h^T lambda, lambda solves
  (grad h M^-1 grad h^T) lambda = -(grad h M^-1 (W + J^T R phi) + c)
  (Sec. II-A, eq. ct-dynamics, eq. joint-cnstr-pos-vel, eq. joint-cnstr-acc);
* control u = (tau, (phi_t, phi_n, gamma) per contact) (Sec. II-A state-space
  form), contact force R phi = t phi_t + n phi_n in the world frame;
* auxiliary system with four states per contact, integrating phi_n,
  lambda_c = t^T J v + gamma dsmoothnorm(phi_t), gamma and
  rho_c = |mu phi_n|_s - ||phi_t||_s (eq. max-diss-tangent-contact-force-KKT-
  reformulate and the definitions after it; eq. aux-dynamics), and N^g = 1
  continuous-time violation state M^g ramp_s(g) with M^g = (1, .., 1) over
  g = (-phi_n, -sd, -gamma, -rho_c) per contact (the nonnegativity path
  constraints listed with the state-space form);
* time-dilated augmented system s (f, Omega) with first-order-hold controls,
  classical RK4 with K substeps and the variational equations through the
  same stages (Sec. IV-B, eq. aug-dynamics, eq. intg-aug-sys-param; Sec. VI).

Readings where the paper is silent: M^g (one state summing every smoothed
violation); the planar smooth norm of the scalar phi_t is |phi_t|_s; the
printed list of four auxiliary integrands per contact is taken as printed
(it carries no integral of sd).  Jacobians come from complex-step
differentiation of the right-hand side (exact to rounding; no hand-derived
formula), evaluated on all directions at once.

Layouts: x~ = (q [3 nb], v [3 nb], y [4 nc + 1]); per contact the y block is
(int phi_n, int lambda_c, int gamma, int rho_c); u = (tau [nj], (phi_t, phi_n,
gamma) per contact); p = (mu, e, masses).  Node-major arrays as in oracle.
"""
from __future__ import annotations

import numpy as np


def dims(model):
    """(n, ny, nx, m) of the variant."""
    n = 6 * model.nb
    ny = 4 * model.nc + 1
    return n, ny, n + ny, model.nj + 3 * model.nc


def sabs(a):
    """|a|_s = sqrt(a^2 + 1) - 1, written a^2 / (sqrt(a^2 + 1) + 1)."""
    return a * a / (np.sqrt(a * a + 1.0) + 1.0)


def sramp(a):
    """Smooth ramp: |a|_s for a > 0, else 0 (the branch on the real part, so
    that complex steps see the branch of their base point)."""
    return np.where(np.real(a) > 0.0, sabs(a), 0.0 * a)


def _terrain(model, Px, Py):
    """sd = H / ||grad H||, n = grad H / ||grad H||, t = (n_y, -n_x) for
    H = P_y - A sin(kappa P_x) (Sec. II contact frame, Sec. VI-B)."""
    A, kap = model.terrain_amplitude, model.terrain_wavenumber
    H = Py - A * np.sin(kap * Px)
    Hx = -A * kap * np.cos(kap * Px)
    G = np.sqrt(1.0 + Hx * Hx)
    nx, ny = Hx / G, 1.0 / G
    return H / G, (nx, ny), (ny, -nx)


def _parts(model, x, u, p):
    """Everything the right-hand side is made of, batched over leading axes."""
    nb, nj, nc = model.nb, model.nj, model.nc
    dt = np.result_type(x, u, p, np.float64)
    lead = np.broadcast_shapes(x.shape[:-1], u.shape[:-1])
    q = np.broadcast_to(x[..., :3 * nb], lead + (3 * nb,)).reshape(lead + (nb, 3))
    v = np.broadcast_to(x[..., 3 * nb:6 * nb], lead + (3 * nb,)).reshape(lead + (nb, 3))
    u = np.broadcast_to(u, lead + (u.shape[-1],))
    mu, masses = p[0], p[2:]
    inertia = masses * model.link_length ** 2 / 12.0
    minv = np.stack([1.0 / masses, 1.0 / masses, 1.0 / inertia], axis=1).reshape(3 * nb)
    c, s = np.cos(q[..., 2]), np.sin(q[..., 2])
    W = np.zeros(lead + (nb, 3), dtype=dt)
    W[..., :, 1] -= masses * model.gravity
    arms = []
    for j in range(nj):
        pb, cb = int(model.joint_parent[j]), int(model.joint_child[j])
        rp, rc = model.anchor_parent[j], model.anchor_child[j]
        ap = (c[..., pb] * rp[0] - s[..., pb] * rp[1], s[..., pb] * rp[0] + c[..., pb] * rp[1])
        ac = (c[..., cb] * rc[0] - s[..., cb] * rc[1], s[..., cb] * rc[0] + c[..., cb] * rc[1])
        arms.append((pb, cb, ap, ac))
        tsd = (-model.stiffness[j] * (q[..., cb, 2] - q[..., pb, 2])
               - model.damping[j] * (v[..., cb, 2] - v[..., pb, 2]))
        tt = u[..., j] + tsd
        W[..., pb, 2] -= tt
        W[..., cb, 2] += tt
    contacts = []
    for i in range(nc):
        b = int(model.contact_body[i])
        r = model.contact_point[i]
        ax, ay = c[..., b] * r[0] - s[..., b] * r[1], s[..., b] * r[0] + c[..., b] * r[1]
        sd, n, t = _terrain(model, q[..., b, 0] + ax, q[..., b, 1] + ay)
        pt, pn, gam = u[..., nj + 3 * i], u[..., nj + 3 * i + 1], u[..., nj + 3 * i + 2]
        Fx, Fy = t[0] * pt + n[0] * pn, t[1] * pt + n[1] * pn
        W[..., b, 0] += Fx
        W[..., b, 1] += Fy
        W[..., b, 2] += ax * Fy - ay * Fx
        # tangential velocity of the contact point, t^T J v with J v = v_b + w_b E a
        vt = t[0] * (v[..., b, 0] - v[..., b, 2] * ay) + t[1] * (v[..., b, 1] + v[..., b, 2] * ax)
        lam_c = vt + gam * pt / np.sqrt(pt * pt + 1.0)
        rho_c = sabs(mu * pn) - sabs(pt)
        contacts.append(dict(sd=sd, pt=pt, pn=pn, gam=gam, vt=vt, lam_c=lam_c, rho_c=rho_c))
    return dict(q=q, v=v, W=W.reshape(lead + (3 * nb,)), minv=minv, arms=arms,
                contacts=contacts, lead=lead, dt=dt)


def joint_jacobian(model, parts):
    """grad h [.., 2 nj, 3 nb] and c [.., 2 nj] with c_j = v^T grad^2 h_j v =
    -w_p^2 a_p + w_c^2 a_c (h_j = p_p + R(th_p) r_p - p_c - R(th_c) r_c)."""
    nb, nj = model.nb, model.nj
    lead, v = parts["lead"], parts["v"]
    Jh = np.zeros(lead + (2 * nj, 3 * nb), dtype=parts["dt"])
    cv = np.zeros(lead + (2 * nj,), dtype=parts["dt"])
    for j, (pb, cb, ap, ac) in enumerate(parts["arms"]):
        for k in range(2):
            Jh[..., 2 * j + k, 3 * pb + k] = 1.0
            Jh[..., 2 * j + k, 3 * cb + k] = -1.0
        Jh[..., 2 * j, 3 * pb + 2] = -ap[1]
        Jh[..., 2 * j + 1, 3 * pb + 2] = ap[0]
        Jh[..., 2 * j, 3 * cb + 2] = ac[1]
        Jh[..., 2 * j + 1, 3 * cb + 2] = -ac[0]
        wp, wc = v[..., pb, 2], v[..., cb, 2]
        cv[..., 2 * j] = -wp * wp * ap[0] + wc * wc * ac[0]
        cv[..., 2 * j + 1] = -wp * wp * ap[1] + wc * wc * ac[1]
    return Jh, cv


def joint_forces(model, x, u, p):
    """lambda [.., 2 nj] of the acceleration-level elimination."""
    parts = _parts(model, x, u, p)
    return _solve_lambda(model, parts)[0]


def _solve_lambda(model, parts):
    Jh, cv = joint_jacobian(model, parts)
    minv, W = parts["minv"], parts["W"]
    if model.nj == 0:
        return np.zeros(parts["lead"] + (0,), dtype=parts["dt"]), Jh
    A = Jh @ (minv[:, None] * np.swapaxes(Jh, -1, -2))
    rhs = -(np.einsum("...ij,...j->...i", Jh, minv * W) + cv)
    lam = np.linalg.solve(A, rhs[..., None])[..., 0]
    return lam, Jh


def rhs(model, x, u, p):
    """f~(x~, u) = (v, v', Omega) (the dilation s multiplies it), batched."""
    x, u, p = np.asarray(x), np.asarray(u), np.asarray(p)
    parts = _parts(model, x, u, p)
    lam, Jh = _solve_lambda(model, parts)
    minv, W = parts["minv"], parts["W"]
    gen = W + np.einsum("...ji,...j->...i", Jh, lam) if model.nj else W
    vdot = minv * gen
    lead = parts["lead"]
    nb = model.nb
    ys, ctcs = [], 0.0
    for ci in parts["contacts"]:
        ys += [ci["pn"], ci["lam_c"], ci["gam"], ci["rho_c"]]
        ctcs = ctcs + sramp(-ci["pn"]) + sramp(-ci["sd"]) + sramp(-ci["gam"]) + sramp(-ci["rho_c"])
    ys.append(ctcs + 0.0 * vdot[..., 0])
    y = np.stack([np.broadcast_to(a, lead) for a in ys], axis=-1)
    vflat = parts["v"].reshape(lead + (3 * nb,))
    return np.concatenate([vflat, vdot, y], axis=-1)


def rhs_jac(model, x, u, p, h=1e-30):
    """f~ and its Jacobians Jx [nx, nx], Ju [nx, m] at one point, all complex
    steps in one batched evaluation."""
    n, ny, nx, m = dims(model)
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    nd = nx + m
    X = np.tile(x.astype(np.complex128), (nd, 1))
    U = np.tile(u.astype(np.complex128), (nd, 1))
    X[np.arange(nx), np.arange(nx)] += 1j * h
    U[nx + np.arange(m), np.arange(m)] += 1j * h
    F = rhs(model, X, U, np.asarray(p, dtype=np.float64))
    f0 = rhs(model, x, u, np.asarray(p, dtype=np.float64))
    J = np.imag(F).T / h
    return np.real(f0), J[:, :nx], J[:, nx:]


def integrate(model, x0, Uk, Uk1, s, p, K, tau0=0.0, tau1=1.0):
    """One interval: classical RK4 with K substeps and the variational
    equations Z = [Phi | Bm | Bp | S] (Phi(tau0) = I; Bm' = s (Jx Bm + Ju (1 - tau));
    Bp' = s (Jx Bp + Ju tau); S' = s Jx S + f~).  Returns xf, Phi, Bm, Bp, S."""
    n, ny, nx, m = dims(model)
    nz = nx + 2 * m + 1
    h = (tau1 - tau0) / K
    x = np.array(x0, dtype=np.float64)
    Z = np.zeros((nx, nz))
    Z[:, :nx] = np.eye(nx)
    Uk, Uk1 = np.asarray(Uk, dtype=np.float64), np.asarray(Uk1, dtype=np.float64)
    cst = (0.0, 0.5, 0.5, 1.0)
    wts = (1.0, 2.0, 2.0, 1.0)
    for j in range(K):
        kx_prev = KZ_prev = None
        xacc = np.zeros(nx)
        Zacc = np.zeros_like(Z)
        for st in range(4):
            tau = tau0 + (j + cst[st]) * h
            if st == 0:
                xs, Zs = x, Z
            else:
                xs = x + h * cst[st] * kx_prev
                Zs = Z + h * cst[st] * KZ_prev
            u = (1.0 - tau) * Uk + tau * Uk1
            f, Jx, Ju = rhs_jac(model, xs, u, p)
            KZ = s * (Jx @ Zs)
            KZ[:, nx:nx + m] += s * Ju * (1.0 - tau)
            KZ[:, nx + m:nx + 2 * m] += s * Ju * tau
            KZ[:, nx + 2 * m] += f
            kx = s * f
            xacc += wts[st] * kx
            Zacc += wts[st] * KZ
            kx_prev, KZ_prev = kx, KZ
        x = x + h / 6.0 * xacc
        Z = Z + h / 6.0 * Zacc
    return dict(xf=x, Phi=Z[:, :nx], Bm=Z[:, nx:nx + m], Bp=Z[:, nx + m:nx + 2 * m],
                S=Z[:, nx + 2 * m])


def discretize(model, X, U, s, p, K):
    """All intervals: A [N, nx, nx], Bm/Bp [N, nx, m], S, d, xprop [N, nx]."""
    X, U, s = np.asarray(X), np.asarray(U), np.asarray(s)
    N = s.shape[0]
    out = {k: [] for k in ("A", "Bm", "Bp", "S", "d", "xprop")}
    for k in range(N):
        r = integrate(model, X[k], U[k], U[k + 1], s[k], p, K)
        out["A"].append(r["Phi"])
        out["Bm"].append(r["Bm"])
        out["Bp"].append(r["Bp"])
        out["S"].append(r["S"])
        out["xprop"].append(r["xf"])
        out["d"].append(r["xf"] - X[k + 1])
    return {k: np.array(v) for k, v in out.items()}
