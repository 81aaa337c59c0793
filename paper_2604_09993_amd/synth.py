"""Seeded synthetic models and node data for the interval discretization.

This module only builds *inputs*: planar multibody model descriptions and
random node states, FOH control coefficients, dilations and parameters with
the shapes and value ranges of the legged-locomotion workloads of the paper
(Sec. VI: monoped, five-link biped on a sinusoid, HalfCheetah; plus a 13-body
quadruped-shaped chain).  It holds none of the method's arithmetic: no
dynamics, no Jacobians, no integration.  Both the HIP path (through the C-ABI)
and the CPU oracle consume what it returns.

Conventions (shared by every consumer, stated once here):

* bodies b = 0..nb-1 in maximal coordinates, pose q_b = (x_b, y_b, theta_b),
  velocity v_b = (xdot_b, ydot_b, omega_b) (Sec. II, maximal coordinates);
* augmented state x~ = (q_0..q_{nb-1}, v_0..v_{nb-1}, y_cc_0..y_cc_{nc-1},
  y_ctcs): n = 6 nb body states, n_y = nc + 1 integral states;
* control u = (tau_0..tau_{nj-1}, lam_0x, lam_0y, ..., [lam_n_i, lam_t+_i,
  lam_t-_i]_i): m = 3 nj + 3 nc (joint torques, world-frame joint forces,
  normal and split-friction contact forces);
* parameters p = (mu, e, m_0..m_{nb-1});
* node arrays are node-major here: X[N+1, n~], U[N+1, m], s[N].

Topology family: every model is a torso (body 0) carrying ``legs`` legs of
``depth`` links each; leg l, link d is body 1 + l*depth + d; joint index
equals child body - 1; the contact of leg l sits at the distal tip of its
last link (for depth 0 the contacts sit on the torso itself).
"""
from __future__ import annotations

import dataclasses
import numpy as np

GRAVITY = 9.81
STIFFNESS = 1.0      # N m / rad, joint stiffness (value not given in the paper)
DAMPING = 0.1        # N m s / rad, joint damping (value not given in the paper)
SIN_AMPLITUDE = 0.05  # m, sinusoidal terrain amplitude (value not given)
SIN_WAVENUMBER = 2.0 * np.pi  # rad / m
MU = 0.8
RESTITUTION = 0.2


@dataclasses.dataclass
class Model:
    """Planar maximal-coordinate model description (host data only)."""
    name: str
    legs: int
    depth: int
    link_length: np.ndarray          # [nb]
    joint_parent: np.ndarray         # [nj] int32
    joint_child: np.ndarray          # [nj] int32
    anchor_parent: np.ndarray        # [nj, 2] body frame of the parent
    anchor_child: np.ndarray         # [nj, 2] body frame of the child
    stiffness: np.ndarray            # [nj]
    damping: np.ndarray              # [nj]
    contact_body: np.ndarray         # [nc] int32
    contact_point: np.ndarray        # [nc, 2] body frame
    gravity: float
    terrain_amplitude: float         # 0 => flat ground
    terrain_wavenumber: float
    masses: np.ndarray               # [nb] default mass parameters
    torque_sigma: float

    @property
    def nb(self) -> int:
        return int(self.link_length.shape[0])

    @property
    def nj(self) -> int:
        return int(self.joint_parent.shape[0])

    @property
    def nc(self) -> int:
        return int(self.contact_body.shape[0])

    @property
    def n(self) -> int:
        return 6 * self.nb

    @property
    def ny(self) -> int:
        return self.nc + 1

    @property
    def nx(self) -> int:
        """Augmented state size n~ = n + n_y."""
        return self.n + self.ny

    @property
    def m(self) -> int:
        return 3 * self.nj + 3 * self.nc

    @property
    def n_params(self) -> int:
        return self.nb + 2

    def params(self, mu: float = MU, e: float = RESTITUTION) -> np.ndarray:
        return np.concatenate([[mu, e], self.masses]).astype(np.float64)


def _rod_y(length: float) -> tuple:
    """Proximal and distal anchors of a rod along the body y axis."""
    return np.array([0.0, 0.5 * length]), np.array([0.0, -0.5 * length])


def legged_model(name: str, legs: int, depth: int, rng: np.random.Generator,
                 length_range=(0.3, 0.5), mass_range=(1.0, 5.0),
                 torque_sigma: float = 5.0, torso: str = "vertical",
                 terrain: str = "flat", hip_x=None,
                 stiffness: float = STIFFNESS, damping: float = DAMPING,
                 gravity: float = GRAVITY) -> Model:
    """Torso + ``legs`` legs of ``depth`` rod links, seeded sizes and masses."""
    nb = 1 + legs * depth
    L = rng.uniform(*length_range, size=nb)
    masses = rng.uniform(*mass_range, size=nb)
    jp, jc, ap, ac = [], [], [], []
    for leg in range(legs):
        for d in range(depth):
            child = 1 + leg * depth + d
            if d == 0:
                parent = 0
                if torso == "vertical":
                    anchor_p = np.array([0.0, -0.5 * L[0]])
                else:
                    xs = hip_x if hip_x is not None else np.linspace(-0.5, 0.5, legs)
                    anchor_p = np.array([xs[leg] * L[0], 0.0])
            else:
                parent = child - 1
                anchor_p = _rod_y(L[parent])[1]
            jp.append(parent)
            jc.append(child)
            ap.append(anchor_p)
            ac.append(_rod_y(L[child])[0])
    cb, cp = [], []
    for leg in range(legs):
        if depth == 0:
            cb.append(0)
            cp.append(np.zeros(2))
        else:
            body = 1 + leg * depth + depth - 1
            cb.append(body)
            cp.append(_rod_y(L[body])[1])
    nj = len(jp)
    nc = len(cb)
    A = SIN_AMPLITUDE if terrain == "sinusoid" else 0.0
    return Model(
        name=name, legs=legs, depth=depth,
        link_length=L.astype(np.float64),
        joint_parent=np.asarray(jp, dtype=np.int32).reshape(nj),
        joint_child=np.asarray(jc, dtype=np.int32).reshape(nj),
        anchor_parent=np.asarray(ap, dtype=np.float64).reshape(nj, 2),
        anchor_child=np.asarray(ac, dtype=np.float64).reshape(nj, 2),
        stiffness=np.full(nj, stiffness, dtype=np.float64),
        damping=np.full(nj, damping, dtype=np.float64),
        contact_body=np.asarray(cb, dtype=np.int32).reshape(nc),
        contact_point=np.asarray(cp, dtype=np.float64).reshape(nc, 2),
        gravity=float(gravity), terrain_amplitude=float(A),
        terrain_wavenumber=float(SIN_WAVENUMBER if A != 0.0 else 0.0),
        masses=masses.astype(np.float64), torque_sigma=float(torque_sigma))


def make_hopper(rng):
    """2-body hopper (torso + one leg link), one foot contact, flat ground."""
    return legged_model("hopper", 1, 1, rng, (0.3, 0.5), (1.0, 5.0), 5.0, "vertical")


def make_biped5(rng):
    """5-body planar biped (torso + two 2-link legs) on the sinusoidal surface."""
    return legged_model("biped5", 2, 2, rng, (0.3, 0.5), (1.0, 5.0), 5.0, "vertical",
                        terrain="sinusoid")


def make_cheetah7(rng):
    """HalfCheetah-shaped chain: horizontal torso + two 3-link legs, 2 feet."""
    return legged_model("cheetah7", 2, 3, rng, (0.1, 0.5), (1.0, 7.0), 20.0,
                        "horizontal", hip_x=[-0.5, 0.5])


def make_quad13(rng):
    """Quadruped-shaped chain: horizontal torso + four 3-link legs, 4 feet."""
    return legged_model("quad13", 4, 3, rng, (0.1, 0.5), (1.0, 7.0), 20.0,
                        "horizontal", hip_x=[-0.5, -1.0 / 6.0, 1.0 / 6.0, 0.5])


def make_free_body(rng, gravity=GRAVITY):
    """Single free body, no joints, no contacts (ballistic case)."""
    return legged_model("free1", 0, 0, rng, (0.3, 0.5), (1.0, 5.0), 5.0,
                        gravity=gravity)


def make_point_contact(rng, terrain="flat", gravity=GRAVITY):
    """Single body with one contact at its centre of mass."""
    return legged_model("point1", 1, 0, rng, (0.3, 0.5), (1.0, 5.0), 5.0,
                        terrain=terrain, gravity=gravity)


MODEL_MAKERS = {
    "hopper": make_hopper,
    "biped5": make_biped5,
    "cheetah7": make_cheetah7,
    "quad13": make_quad13,
    "free1": make_free_body,
    "point1": make_point_contact,
}


def _rot(th):
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s], [s, c]])


def _place(model: Model, x0: float, y0: float, th0: float, joint_angles: np.ndarray):
    """Body poses for given torso pose and relative joint angles (joints closed)."""
    nb = model.nb
    pos = np.zeros((nb, 2))
    th = np.zeros(nb)
    pos[0] = (x0, y0)
    th[0] = th0
    for j in range(model.nj):  # parents always precede children in this family
        p, c = int(model.joint_parent[j]), int(model.joint_child[j])
        th[c] = th[p] + joint_angles[j]
        hinge = pos[p] + _rot(th[p]) @ model.anchor_parent[j]
        pos[c] = hinge - _rot(th[c]) @ model.anchor_child[j]
    return pos, th


def _lowest_clearance(model: Model, pos, th):
    """Smallest vertical gap between a contact point and the terrain."""
    gaps = []
    for i in range(model.nc):
        b = int(model.contact_body[i])
        P = pos[b] + _rot(th[b]) @ model.contact_point[i]
        ground = model.terrain_amplitude * np.sin(model.terrain_wavenumber * P[0])
        gaps.append(P[1] - ground)
    return min(gaps) if gaps else None


def gen_nodes(model: Model, N: int, rng: np.random.Generator,
              vel_sigma: float = 0.5, joint_force_sigma: float = 10.0,
              contact_range=(0.0, 30.0), T: float = 1.0):
    """Seeded node data for one trajectory with N intervals (N+1 nodes).

    Returns a dict with X[N+1, n~], U[N+1, m], s[N], p[P] (float64, node-major).
    Poses come from forward placement of random joint angles U(-0.5, 0.5), so
    joints are closed at the nodes; the torso height is shifted so the lowest
    contact sits U(-0.02, 0.10) m above the terrain; every velocity component
    is N(0, vel_sigma); integral states are zero.
    """
    nb, nj, nc = model.nb, model.nj, model.nc
    X = np.zeros((N + 1, model.nx))
    for k in range(N + 1):
        x0 = rng.uniform(-0.5, 0.5)
        th0 = rng.uniform(-0.2, 0.2)
        ja = rng.uniform(-0.5, 0.5, size=nj)
        pos, th = _place(model, x0, 0.0, th0, ja)
        gap = _lowest_clearance(model, pos, th)
        target = rng.uniform(-0.02, 0.10)
        if gap is None:
            shift = 1.0
        else:
            shift = target - gap
        pos[:, 1] += shift
        q = np.column_stack([pos[:, 0], pos[:, 1], th]).reshape(-1)
        v = rng.normal(0.0, vel_sigma, size=3 * nb)
        X[k, :3 * nb] = q
        X[k, 3 * nb:6 * nb] = v
    U = np.zeros((N + 1, model.m))
    U[:, :nj] = rng.normal(0.0, model.torque_sigma, size=(N + 1, nj))
    U[:, nj:3 * nj] = rng.normal(0.0, joint_force_sigma, size=(N + 1, 2 * nj))
    U[:, 3 * nj:] = rng.uniform(*contact_range, size=(N + 1, 3 * nc))
    s = rng.uniform(0.5, 2.0, size=N) * T / N
    return {"X": X, "U": U, "s": s, "p": model.params()}


def gen_impact_nodes(model: Model, n_nodes: int, rng: np.random.Generator,
                     pose_sigma: float = 1e-3, impulse_range=(0.0, 5.0)):
    """Seeded node variables of the impact map at an SCP iterate (not feasible in
    general): pre-impact augmented states x~- as in gen_nodes (closed joints,
    integral states U(0, 0.1)); post-impact states with the pose perturbed by
    N(0, pose_sigma), velocities x- + N(0, 0.5) and integral states x- + U(0, 0.1);
    per contact impulses Phi_n ~ U(impulse_range), Phi_t ~ U(-mu Phi_n, mu Phi_n)
    (inside the friction cone), multipliers Gamma ~ U(0, 1).

    Returns a dict with Xm, Xp [n_nodes, n~], Phi [n_nodes, 2 nc] (t, n per
    contact), Gamma [n_nodes, nc], p [P] (float64, node-major).
    """
    nb, nc = model.nb, model.nc
    Xm = gen_nodes(model, max(n_nodes - 1, 1), rng)["X"][:n_nodes].copy()
    Xm[:, 6 * nb:] = rng.uniform(0.0, 0.1, size=(n_nodes, model.ny))
    Xp = Xm.copy()
    Xp[:, :3 * nb] += rng.normal(0.0, pose_sigma, size=(n_nodes, 3 * nb))
    Xp[:, 3 * nb:6 * nb] += rng.normal(0.0, 0.5, size=(n_nodes, 3 * nb))
    Xp[:, 6 * nb:] += rng.uniform(0.0, 0.1, size=(n_nodes, model.ny))
    p = model.params()
    pn = rng.uniform(*impulse_range, size=(n_nodes, nc))
    pt = rng.uniform(-1.0, 1.0, size=(n_nodes, nc)) * p[0] * pn
    Phi = np.stack([pt, pn], axis=2).reshape(n_nodes, 2 * nc)
    Gam = rng.uniform(0.0, 1.0, size=(n_nodes, nc))
    return {"Xm": Xm, "Xp": Xp, "Phi": Phi, "Gamma": Gam, "p": p}


def gen_paper_nodes(model: Model, N: int, rng: np.random.Generator, T: float = 1.0,
                    vel_sigma: float = 0.5, contact_range=(0.0, 30.0)):
    """Seeded node data of the paper-faithful dynamics variant (joint forces
    eliminated, n_y = 4 nc + 1): poses and velocities as gen_nodes, integral
    states zero; u = (tau ~ N(0, torque_sigma), per contact phi_t, phi_n, gamma)
    with phi_n ~ U(contact_range), phi_t ~ U(-mu phi_n, mu phi_n) (inside the
    friction cone), gamma ~ U(0, 1).

    Returns a dict with X[N+1, 6 nb + 4 nc + 1], U[N+1, nj + 3 nc], s[N], p[P].
    """
    base = gen_nodes(model, N, rng, vel_sigma=vel_sigma, T=T)
    nb, nj, nc = model.nb, model.nj, model.nc
    X = np.zeros((N + 1, 6 * nb + 4 * nc + 1))
    X[:, :6 * nb] = base["X"][:, :6 * nb]
    U = np.zeros((N + 1, nj + 3 * nc))
    U[:, :nj] = rng.normal(0.0, model.torque_sigma, size=(N + 1, nj))
    p = model.params()
    pn = rng.uniform(*contact_range, size=(N + 1, nc))
    U[:, nj::3] = rng.uniform(-1.0, 1.0, size=(N + 1, nc)) * p[0] * pn
    U[:, nj + 1::3] = pn
    U[:, nj + 2::3] = rng.uniform(0.0, 1.0, size=(N + 1, nc))
    return {"X": X, "U": U, "s": base["s"], "p": p}


# Workload recipes (model, N, substeps) of the benchmark configurations.
# The benchmark workloads by name: model, intervals N, substeps K, and the
# seed of their node data (batch: trajectories; ckpt: substeps between the
# checkpoints of the reverse sweep).
WORKLOADS = {
    "hopper_N20_K10": dict(model="hopper", N=20, K=10, seed=1),
    "cheetah7_N50_K20": dict(model="cheetah7", N=50, K=20, seed=2),
    "cheetah7_N50_K20_ckpt5": dict(model="cheetah7", N=50, K=20, ckpt=5, seed=3),
    "quad13_N200_K20_x64": dict(model="quad13", N=200, K=20, batch=64, seed=5),
    # the 64 x 200 intervals of the batch as one trajectory (same interval
    # lengths: T scaled with N)
    "quad13_N12800_K20": dict(model="quad13", N=12800, K=20, T=64.0, seed=7),
}


def make_workload(name: str, traj_id: int = 0):
    """Model and node data of a named workload, seeded by (its seed, traj_id)."""
    cfg = WORKLOADS[name]
    rng = np.random.default_rng([cfg["seed"], traj_id])
    model = MODEL_MAKERS[cfg["model"]](rng)
    data = gen_nodes(model, cfg["N"], rng, T=cfg.get("T", 1.0))
    return model, data, cfg["K"]


# Node batches of the impact map: the nodes of a batched workload (every node
# of every trajectory, (N + 1) x batch), drawn by gen_impact_nodes with `seed`.
IMPACT_WORKLOADS = {
    "quad13_x64": dict(workload="quad13_N200_K20_x64", seed=6),
}


def impact_workload(name: str):
    """Model and node variables of a named impact-map batch."""
    cfg = IMPACT_WORKLOADS[name]
    w = WORKLOADS[cfg["workload"]]
    model, _, _ = make_workload(cfg["workload"], 0)
    n = (w["N"] + 1) * w.get("batch", 1)
    return model, gen_impact_nodes(model, n, np.random.default_rng(cfg["seed"]))


# Model mix of the uneven multi-trajectory batch (trajectories per 256).
BATCH_MIX = (("hopper", 128), ("cheetah7", 77), ("biped5", 51))


def mixed_batch(n_traj: int = 256, seed: int = 4, N_range=(20, 100), K_range=(10, 30)):
    """Uneven batch over three models: hopper / cheetah7 / biped5 trajectories
    in the ratio 128 : 77 : 51, N ~ U{N_range}, K ~ U{K_range}.

    One model per kind (seeded by (seed, 0, kind index)); the order of the
    kinds is shuffled with (seed, 0); trajectory t draws N, K and its nodes
    from (seed, t + 1).  Returns a list of (model, data, K).
    """
    total = sum(c for _, c in BATCH_MIX)
    counts = [int(round(n_traj * c / total)) for _, c in BATCH_MIX]
    counts[-1] = n_traj - sum(counts[:-1])
    models = {kind: MODEL_MAKERS[kind](np.random.default_rng([seed, 0, i]))
              for i, (kind, _) in enumerate(BATCH_MIX)}
    kinds = [kind for (kind, _), c in zip(BATCH_MIX, counts) for _ in range(c)]
    np.random.default_rng([seed, 0]).shuffle(kinds)
    out = []
    for t, kind in enumerate(kinds):
        r = np.random.default_rng([seed, t + 1])
        N = int(r.integers(N_range[0], N_range[1] + 1))
        K = int(r.integers(K_range[0], K_range[1] + 1))
        model = models[kind]
        out.append((model, gen_nodes(model, N, r), K))
    return out


def workload_batch(name: str, n_traj=None):
    """The trajectories of a batched workload, all of one model.

    Trajectory 0 is make_workload(name, 0); trajectory t > 0 takes the same
    model and draws its nodes from (the workload's seed, t).
    """
    cfg = WORKLOADS[name]
    n_traj = cfg.get("batch", 1) if n_traj is None else n_traj
    model, data, K = make_workload(name, 0)
    out = [(model, data, K)]
    for t in range(1, n_traj):
        r = np.random.default_rng([cfg["seed"], t])
        MODEL_MAKERS[cfg["model"]](r)   # same stream position as make_workload
        out.append((model, gen_nodes(model, cfg["N"], r), K))
    return out


def standing_state(model: Model, x0: float, th0: float = 0.0, joint_angles=None,
                   clearance: float = 0.0):
    """Augmented state of the model at rest with its lowest contact `clearance`
    above the terrain: torso at horizontal position x0 and angle th0, relative
    joint angles (default zero), velocities and integral states zero."""
    ja = np.zeros(model.nj) if joint_angles is None else np.asarray(joint_angles, float)
    pos, th = _place(model, x0, 0.0, th0, ja)
    gap = _lowest_clearance(model, pos, th)
    pos[:, 1] += (clearance - gap) if gap is not None else 1.0
    x = np.zeros(model.nx)
    x[:3 * model.nb] = np.column_stack([pos[:, 0], pos[:, 1], th]).reshape(-1)
    return x


def scp_initial_guess(model: Model, N: int, x_init, x_final, s0: float,
                      rng: np.random.Generator, force_range=(0.0, 20.0),
                      impulse_range=(0.0, 1.0), mu: float = 1.0):
    """Naive starting point of the contact-implicit SCP (the initialization of
    the paper's experiments, Sec. VI): node poses interpolated linearly between
    the boundary states, velocities, integral states, joint torques and joint
    forces zero, contact forces and impulses drawn inside the friction cone of
    coefficient mu (lambda_n ~ U(force_range), lambda_t+ + lambda_t- <= mu lambda_n;
    Phi_n ~ U(impulse_range), |Phi_t| <= mu Phi_n), multipliers Gamma ~ U(0, 1).

    Returns node-major Xp, Xm [N+1, nx], Phi [N+1, 2 nc], Gamma [N+1, nc],
    interval controls Ua, Ub [N, m] (discontinuous first-order hold) and S [N].
    """
    nb, nj, nc, nx, m = model.nb, model.nj, model.nc, model.nx, model.m
    w = np.linspace(0.0, 1.0, N + 1)[:, None]
    X = np.zeros((N + 1, nx))
    X[:, :3 * nb] = (1.0 - w) * np.asarray(x_init)[:3 * nb] + w * np.asarray(x_final)[:3 * nb]
    Xm, Xp = X.copy(), X.copy()

    def controls():
        U = np.zeros((N, m))
        ln = rng.uniform(*force_range, size=(N, nc))
        frac = rng.uniform(0.0, 1.0, size=(N, nc, 2))
        frac /= np.maximum(1.0, frac.sum(axis=2, keepdims=True))
        U[:, 3 * nj::3] = ln
        U[:, 3 * nj + 1::3] = frac[:, :, 0] * mu * ln
        U[:, 3 * nj + 2::3] = frac[:, :, 1] * mu * ln
        return U

    Ua, Ub = controls(), controls()
    pn = rng.uniform(*impulse_range, size=(N + 1, nc))
    pt = rng.uniform(-1.0, 1.0, size=(N + 1, nc)) * mu * pn
    Phi = np.stack([pt, pn], axis=2).reshape(N + 1, 2 * nc)
    Gam = rng.uniform(0.0, 1.0, size=(N + 1, nc))
    return {"Xp": Xp, "Xm": Xm, "Phi": Phi, "Gamma": Gam, "Ua": Ua, "Ub": Ub,
            "S": np.full(N, float(s0))}
