"""Torch-facing calls of the HIP discretization library.

Tensors live on the GPU in the library's layout (interval or node index
contiguous, see include/cis.h): X[nx, ld_node], U[m, ld_node], s[N],
params[P]; outputs come back as A[nx, nx, N], Bm/Bp[nx, m, N], S/d/F~[nx, N].
``as_interval_major`` gives [N, ...] views.  PyTorch only provides device
memory and the current stream; every arithmetic step runs in the kernels.
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _alloc_on(stream):
    """Allocate outputs and workspaces on the stream the kernels run on, so the
    caching allocator does not hand their memory to other work before the
    kernels have finished with it."""
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


class CisModel:
    """A model description registered with the library (host object)."""

    def __init__(self, model):
        lib = _lib.load()
        self.model = model
        keep = [
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
        ptrs = [k.ctypes.data if k.size else None for k in keep]
        desc = _lib.ModelDesc(model.nb, model.nj, model.nc, *ptrs, model.gravity,
                              model.terrain_amplitude, model.terrain_wavenumber)
        h = ctypes.c_void_p()
        _lib.check(lib.cis_model_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        dims = [ctypes.c_int32() for _ in range(4)]
        _lib.check(lib.cis_model_dims(h, *[ctypes.byref(d) for d in dims]))
        self.n, self.ny, self.m, self.np = [d.value for d in dims]
        self.nx = self.n + self.ny

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and lib is not None:
            lib.cis_model_destroy(h)
            self._h = None


def _dtype_code(dtype):
    if dtype == torch.float64:
        return _lib.CIS_F64
    if dtype == torch.float32:
        return _lib.CIS_F32
    raise TypeError(f"unsupported dtype {dtype}")


LAYOUTS = {"rule": 0, "latency": 1, "latency_s": 2, "narrow": 3, "throughput": 4}


def _shape(X, s, K, ld_int=None, layout="rule"):
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be [nx, ld_node] with unit stride along nodes")
    N = s.shape[0]
    return _lib.Shape(N, int(K), _dtype_code(X.dtype), LAYOUTS[layout], X.stride(0),
                      N if ld_int is None else int(ld_int))


def _check_inputs(cm, X, U, s, params):
    dev = X.device
    if dev.type != "cuda":
        raise ValueError("inputs must be GPU tensors")
    for t in (U, s, params):
        if t is not None and (t.device != dev or t.dtype != X.dtype):
            raise ValueError("all inputs must share device and dtype")
    if X.shape[0] != cm.nx or s.dim() != 1 or X.shape[1] < s.shape[0] + 1:
        raise ValueError("X must be [nx, >= N+1] and s [N]")
    if cm.m and (U is None or U.shape[0] != cm.m or U.stride(1) != 1 or U.stride(0) != X.stride(0)
                 or U.shape[1] < s.shape[0] + 1):
        raise ValueError("U must be [m, >= N+1] with the same ld_node as X")
    if params.numel() != cm.np or not params.is_contiguous() or not s.is_contiguous():
        raise ValueError("params must hold P contiguous values and s must be contiguous")


def discretize(cm: CisModel, X, U, s, params, K, *, with_xprop=True, layout="rule",
               stream=None):
    """A, Bm, Bp, S, defect (and F~) of every interval, written by one kernel launch.
    layout: one of LAYOUTS ("rule": chosen from N and the device's CU count)."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
    sh = _shape(X, s, K, layout=layout)
    lib = _lib.load()
    _lib.check(lib.cis_discretize(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                  _ptr(params), _ptr(out["A"]), _ptr(out["Bm"] if m else None),
                                  _ptr(out["Bp"] if m else None), _ptr(out["S"]), _ptr(out["d"]),
                                  _ptr(out["xprop"]), _stream(stream)))
    return out


def discretize_into(cm, X, U, s, params, K, out, stream=None):
    """Same as discretize, writing into preallocated outputs (no allocation).

    out holds A[nx, nx, ld], Bm/Bp[nx, m, ld], S/d[nx, ld] and optionally
    xprop[nx, ld], all contiguous with the same ld >= N.
    """
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    ld = out["S"].shape[-1]
    for key, lead in (("A", (nx, nx)), ("Bm", (nx, m)), ("Bp", (nx, m)), ("S", (nx,)),
                      ("d", (nx,)), ("xprop", (nx,))):
        t = out.get(key)
        if t is None and key in ("xprop",):
            continue
        if (t is None or not t.is_contiguous() or tuple(t.shape[:-1]) != lead or t.shape[-1] != ld
                or ld < N or t.dtype != X.dtype or t.device != X.device):
            raise ValueError(f"output {key} must be a contiguous {lead + (ld,)} tensor, ld >= N")
    sh = _shape(X, s, K, ld_int=ld)
    lib = _lib.load()
    _lib.check(lib.cis_discretize(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                  _ptr(params), _ptr(out["A"]), _ptr(out["Bm"] if cm.m else None),
                                  _ptr(out["Bp"] if cm.m else None), _ptr(out["S"]), _ptr(out["d"]),
                                  _ptr(out.get("xprop")), _stream(stream)))
    return out


def blocked_workspace_bytes(cm: CisModel, N, K, blocks, ld_int=None):
    sh = _lib.Shape(N, int(K), _lib.CIS_F64, 0, N + 1, N if ld_int is None else int(ld_int))
    nbytes = ctypes.c_size_t()
    _lib.check(_lib.load().cis_blocked_workspace_size(cm.handle, ctypes.byref(sh), int(blocks),
                                                      ctypes.byref(nbytes)))
    return nbytes.value


def discretize_blocked(cm: CisModel, X, U, s, params, K, blocks, compose="valu", *,
                       with_xprop=True, ws=None, stream=None):
    """Same outputs as :func:`discretize` (FP64) with the substeps split into
    `blocks` blocks integrated in parallel and chained by dense products
    (compose = "valu" or "mfma").  ws: optional preallocated uint8 workspace."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    nbytes = blocked_workspace_bytes(cm, N, K, blocks)
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty((nbytes,), device=X.device, dtype=torch.uint8)
    sh = _shape(X, s, K)
    mode = {"valu": _lib.CIS_COMPOSE_VALU, "mfma": _lib.CIS_COMPOSE_MFMA}[compose]
    lib = _lib.load()
    _lib.check(lib.cis_discretize_blocked(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                          _ptr(params), int(blocks), mode, _ptr(out["A"]),
                                          _ptr(out["Bm"] if m else None),
                                          _ptr(out["Bp"] if m else None), _ptr(out["S"]),
                                          _ptr(out["d"]), _ptr(out["xprop"]), _ptr(ws),
                                          ws.numel(), _stream(stream)))
    return out


FORMS = {_lib.CIS_FORM_ONE_LAUNCH: "one_launch", _lib.CIS_FORM_SPLIT: "split",
         _lib.CIS_FORM_BLOCKED: "blocked"}


def single_tune(cm: CisModel, X, U, s, params, K, *, with_xprop=True, stream=None):
    """Tuner of the discretize step for one trajectory shape: the fastest of
    the one-launch layouts, the split form (1 or 2 waves) and the FP64 blocked
    forms on these inputs.  Returns (outputs of the chosen configuration, a
    dict describing it: form, layout, waves, blocks, compose, from_cache, ms)."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
    sh = _shape(X, s, K)
    ch = _lib.SingleChoice()
    _lib.check(_lib.load().cis_single_tune(
        cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s), _ptr(params), _ptr(out["A"]),
        _ptr(out["Bm"] if m else None), _ptr(out["Bp"] if m else None), _ptr(out["S"]),
        _ptr(out["d"]), _ptr(out["xprop"]), ctypes.byref(ch), _stream(stream)))
    names = {v: k for k, v in LAYOUTS.items()}
    choice = dict(form=FORMS[ch.form], layout=names.get(ch.layout, "rule"), waves=ch.waves,
                  blocks=ch.blocks,
                  compose="mfma" if ch.compose == _lib.CIS_COMPOSE_MFMA else "valu",
                  from_cache=bool(ch.from_cache), ms=float(ch.ms))
    return out, choice


def split_workspace_bytes(cm: CisModel, N, K, dtype=torch.float64):
    sh = _lib.Shape(N, int(K), _dtype_code(dtype), 0, N + 1, N)
    nbytes = ctypes.c_size_t()
    _lib.check(_lib.load().cis_split_workspace_size(cm.handle, ctypes.byref(sh),
                                                    ctypes.byref(nbytes)))
    return nbytes.value


def discretize_split(cm: CisModel, X, U, s, params, K, *, waves=1, with_xprop=True, ws=None,
                     stream=None):
    """Same outputs as :func:`discretize`, computed by the two-launch split
    form (stage coefficient records, then one wave per leg over 64 tangent
    columns).  ws: optional preallocated uint8 workspace."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    nbytes = split_workspace_bytes(cm, N, K, X.dtype)
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty((nbytes,), device=X.device, dtype=torch.uint8)
    sh = _shape(X, s, K)
    lib = _lib.load()
    _lib.check(lib.cis_discretize_split(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                        _ptr(params), int(waves), _ptr(out["A"]),
                                        _ptr(out["Bm"] if m else None),
                                        _ptr(out["Bp"] if m else None), _ptr(out["S"]),
                                        _ptr(out["d"]), _ptr(out["xprop"]), _ptr(ws),
                                        ws.numel(), _stream(stream)))
    return out


def rkf_workspace_bytes(cm: CisModel, N, K, dtype=torch.float64):
    sh = _lib.Shape(N, int(K), _dtype_code(dtype), 0, N + 1, N)
    nb = ctypes.c_size_t()
    _lib.check(_lib.load().cis_rkf_workspace_size(cm.handle, ctypes.byref(sh), ctypes.byref(nb)))
    return nb.value


def discretize_rkf(cm: CisModel, X, U, s, params, K, *, waves=1, with_xprop=True, ws=None,
                   stream=None):
    """The discretize outputs with K Runge-Kutta-Fehlberg steps per interval
    (fourth-order solution propagated) and err[N], the embedded estimate."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    nbytes = rkf_workspace_bytes(cm, N, K, X.dtype)
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw), err=torch.empty((N,), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty((nbytes,), device=X.device, dtype=torch.uint8)
    sh = _shape(X, s, K)
    lib = _lib.load()
    _lib.check(lib.cis_discretize_rkf(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                      _ptr(params), int(waves), _ptr(out["A"]),
                                      _ptr(out["Bm"] if m else None),
                                      _ptr(out["Bp"] if m else None), _ptr(out["S"]),
                                      _ptr(out["d"]), _ptr(out["xprop"]), _ptr(out["err"]),
                                      _ptr(ws), ws.numel(), _stream(stream)))
    return out


def paper_dims(cm: CisModel):
    """(nx, m) of the paper-faithful dynamics variant of a model."""
    nx, m = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().cis_paper_dims(cm.handle, ctypes.byref(nx), ctypes.byref(m)))
    return nx.value, m.value


def discretize_paper(cm: CisModel, X, U, s, params, K, *, with_xprop=True, stream=None):
    """The discretize outputs of the paper-faithful dynamics variant (joint
    forces eliminated, controls (tau, phi_t, phi_n, gamma), nx = 6 nb + 4 nc + 1),
    FP64: X [nx, ld_node], U [m, ld_node]."""
    nx, m = paper_dims(cm)
    if X.dtype != torch.float64 or X.device.type != "cuda":
        raise ValueError("inputs must be float64 GPU tensors")
    N = s.shape[0]
    if (X.shape[0] != nx or U.shape[0] != m or X.stride(1) != 1 or U.stride(1) != 1
            or U.stride(0) != X.stride(0) or X.shape[1] < N + 1 or U.shape[1] < N + 1):
        raise ValueError("X must be [nx, >= N+1] and U [m, >= N+1] with one ld_node")
    kw = dict(device=X.device, dtype=X.dtype)
    sh = _lib.Shape(N, int(K), _lib.CIS_F64, 0, X.stride(0), N)
    nb_ = ctypes.c_size_t()
    lib = _lib.load()
    _lib.check(lib.cis_paper_workspace_size(cm.handle, ctypes.byref(sh), ctypes.byref(nb_)))
    with _alloc_on(stream):
        out = dict(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                   Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw),
                   d=torch.empty((nx, N), **kw))
        out["xprop"] = torch.empty((nx, N), **kw) if with_xprop else None
        ws = torch.empty((nb_.value,), device=X.device, dtype=torch.uint8)
    _lib.check(lib.cis_discretize_paper(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                        _ptr(params), _ptr(out["A"]), _ptr(out["Bm"]),
                                        _ptr(out["Bp"]), _ptr(out["S"]), _ptr(out["d"]),
                                        _ptr(out["xprop"]), _ptr(ws), ws.numel(),
                                        _stream(stream)))
    return out


def defects(cm: CisModel, X, U, s, params, K, *, ckpt_every=None, stream=None):
    """F~ and defects only; optional substep checkpoints [K/C, n, N] for the adjoint."""
    _check_inputs(cm, X, U, s, params)
    N, nx = s.shape[0], cm.nx
    kw = dict(device=X.device, dtype=X.dtype)
    C = 0
    if ckpt_every is not None:
        C = int(ckpt_every)
        if C < 1 or K % C:
            raise ValueError("ckpt_every must divide K")
    with _alloc_on(stream):
        out = dict(d=torch.empty((nx, N), **kw), xprop=torch.empty((nx, N), **kw), ckpt=None)
        if C:
            out["ckpt"] = torch.empty((K // C, cm.n, N), **kw)
    sh = _shape(X, s, K)
    lib = _lib.load()
    _lib.check(lib.cis_defects(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                               _ptr(params), _ptr(out["d"]), _ptr(out["xprop"]), _ptr(out["ckpt"]),
                               C, _stream(stream)))
    return out


def adjoint_workspace_bytes(cm: CisModel, N, K, dtype=torch.float64):
    sh = _lib.Shape(N, int(K), _dtype_code(dtype), 0, N + 1, N)
    nbytes = ctypes.c_size_t()
    _lib.check(_lib.load().cis_adjoint_workspace_size(cm.handle, ctypes.byref(sh),
                                                      ctypes.byref(nbytes)))
    return nbytes.value


def adjoint(cm: CisModel, X, U, s, params, K, ckpt, ckpt_every, seed, *, stream=None):
    """gX[nx, N+1], gU[m, N+1], gs[N], gp[P] for the cotangent seed[nx, N] of F~."""
    _check_inputs(cm, X, U, s, params)
    N, nx, m = s.shape[0], cm.nx, cm.m
    kw = dict(device=X.device, dtype=X.dtype)
    if seed.shape != (nx, N) or not seed.is_contiguous():
        raise ValueError("seed must be a contiguous [nx, N] tensor")
    if ckpt is None or ckpt.shape != (K // ckpt_every, cm.n, N) or not ckpt.is_contiguous():
        raise ValueError("ckpt must come from defects(..., ckpt_every=C) with the same K, C")
    ld = X.stride(0)
    nbytes = adjoint_workspace_bytes(cm, N, K, X.dtype)
    with _alloc_on(stream):
        gX = torch.empty((nx, ld), **kw)
        gU = torch.empty((max(m, 1), ld), **kw)
        gs = torch.empty((N,), **kw)
        gp = torch.empty((cm.np,), **kw)
        ws = torch.empty((max(nbytes, 1),), device=X.device, dtype=torch.uint8)
    sh = _shape(X, s, K)
    lib = _lib.load()
    _lib.check(lib.cis_discretize_adjoint(cm.handle, ctypes.byref(sh), _ptr(X), _ptr(U), _ptr(s),
                                          _ptr(params), _ptr(ckpt), int(ckpt_every), _ptr(seed),
                                          _ptr(gX), _ptr(gU if m else None), _ptr(gs), _ptr(gp),
                                          _ptr(ws), nbytes, _stream(stream)))
    return dict(gX=gX[:, :N + 1], gU=gU[:m, :N + 1], gs=gs, gp=gp)


class CisDefects(torch.autograd.Function):
    """F~ = F~(X, U, s, p) of every interval; backward is the reverse-mode kernel.

    forward(X, U, s, params, cm, K, C) -> F~[nx, N]; substep checkpoints every C
    substeps are saved and recomputed from in the backward pass.
    """

    @staticmethod
    def forward(ctx, X, U, s, params, cm, K, C):
        out = defects(cm, X.detach(), U.detach(), s.detach(), params.detach(), K, ckpt_every=C)
        ctx.save_for_backward(X, U, s, params, out["ckpt"])
        ctx.cm, ctx.K, ctx.C = cm, K, C
        return out["xprop"]

    @staticmethod
    def backward(ctx, gF):
        X, U, s, params, ckpt = ctx.saved_tensors
        g = adjoint(ctx.cm, X.detach(), U.detach(), s.detach(), params.detach(), ctx.K, ckpt,
                    ctx.C, gF.contiguous())
        N = s.shape[0]
        gX = torch.zeros_like(X)
        gX[:, :N + 1] = g["gX"]
        gU = torch.zeros_like(U)
        if ctx.cm.m:
            gU[:, :N + 1] = g["gU"]
        return gX, gU, g["gs"], g["gp"], None, None, None


def impact_dims(cm: CisModel):
    """(rows of Theta, columns of JGv, columns of JTc) of a model."""
    d = [ctypes.c_int32() for _ in range(3)]
    _lib.check(_lib.load().cis_impact_dims(cm.handle, *[ctypes.byref(v) for v in d]))
    return tuple(v.value for v in d)


def impact_columns(model):
    """Where the columns of the compact impact Jacobians sit in the node vector
    z = (x~+ [nx], x~- [nx], Phi [2 nc], Gamma [nc], p [P]): an index array
    [7 nb + 2 nc] for JGv and [nc, 14] for JTc (layout of include/cis.h)."""
    nb, nc, nx = model.nb, model.nc, model.nx
    nq = 3 * nb
    phi0, gam0, p0 = 2 * nx, 2 * nx + 2 * nc, 2 * nx + 3 * nc
    jgv = np.concatenate([np.arange(nq), nx + nq + np.arange(nq), phi0 + np.arange(2 * nc),
                          p0 + 2 + np.arange(nb)])
    jtc = np.zeros((nc, 14), dtype=np.int64)
    for i in range(nc):
        b = int(model.contact_body[i])
        jtc[i] = np.concatenate([3 * b + np.arange(3), nq + 3 * b + np.arange(3),
                                 nx + nq + 3 * b + np.arange(3),
                                 [phi0 + 2 * i, phi0 + 2 * i + 1, gam0 + i, p0, p0 + 1]])
    return jgv, jtc


def impact_linearize(cm: CisModel, Xp, Xm, Phi, Gamma, params, delta, eps=0.0, *, n_nodes=None,
                     with_psi=True, stream=None):
    """Node residuals G~, Theta (and Psi) with the compact Jacobians JGv, JTc of
    n_nodes nodes (FP64).  Xp, Xm [nx, ld], Phi [2 nc, ld], Gamma [nc, ld] share
    one row stride ld; outputs are node-major (include/cis.h)."""
    if Xp.device.type != "cuda" or Xp.dtype != torch.float64:
        raise ValueError("inputs must be float64 GPU tensors")
    n = Xp.shape[1] if n_nodes is None else int(n_nodes)
    ld = Xp.stride(0)
    nth, ncv, nct = impact_dims(cm)
    nc = nth // 10
    for t, rows in ((Xp, cm.nx), (Xm, cm.nx), (Phi, 2 * nc), (Gamma, nc)):
        if nc == 0 and rows == 0:
            continue
        if (t.device != Xp.device or t.dtype != torch.float64 or t.dim() != 2 or t.shape[0] != rows
                or t.stride(1) != 1 or t.stride(0) != ld or t.shape[1] < n):
            raise ValueError("Xp, Xm, Phi, Gamma must be float64 [rows, >= n_nodes] with one stride")
    if params.numel() != cm.np or not params.is_contiguous() or params.dtype != torch.float64:
        raise ValueError("params must hold P contiguous float64 values")
    nq = cm.n // 2
    kw = dict(device=Xp.device, dtype=torch.float64)
    with _alloc_on(stream):
        out = dict(G=torch.empty((n, cm.nx), **kw), Theta=torch.empty((n, nth), **kw),
                   JGv=torch.empty((n, nq, ncv), **kw), JTc=torch.empty((n, nth, nct), **kw),
                   Psi=torch.empty((max(n - 1, 0), cm.ny), **kw) if with_psi else None)
    lib = _lib.load()
    _lib.check(lib.cis_impact_linearize(
        cm.handle, n, max(ld, 1), _ptr(Xp), _ptr(Xm), _ptr(Phi if nc else None),
        _ptr(Gamma if nc else None), _ptr(params), float(delta), float(eps), _ptr(out["G"]),
        _ptr(out["Theta"] if nc else None), _ptr(out["JGv"]), _ptr(out["JTc"] if nc else None),
        _ptr(out["Psi"]), _stream(stream)))
    return out


def as_interval_major(out):
    """[N, ...] views of the outputs (A[N,nx,nx], Bm/Bp[N,nx,m], S/d/F~[N,nx])."""
    v = {}
    for key, t in out.items():
        if t is None:
            v[key] = None
        elif t.dim() == 3 and key != "ckpt":
            v[key] = t.permute(2, 0, 1)
        elif t.dim() == 2:
            v[key] = t.t()
        else:
            v[key] = t
    return v


def to_device_soa(arr, device="cuda", dtype=torch.float64, ld=None):
    """Node-major numpy [N+1, c] -> device tensor [c, ld] (node index contiguous)."""
    arr = np.asarray(arr, dtype=np.float64)
    t = torch.from_numpy(np.ascontiguousarray(arr.T))
    if ld is not None and ld > t.shape[1]:
        pad = torch.zeros((t.shape[0], ld - t.shape[1]), dtype=t.dtype)
        t = torch.cat([t, pad], dim=1)
    return t.to(device=device, dtype=dtype).contiguous()


_SCHED = {"grid": _lib.CIS_SCHED_GRID, "persistent": _lib.CIS_SCHED_PERSISTENT,
          "tune": _lib.CIS_SCHED_TUNE}
_OPS = {"discretize": _lib.CIS_BATCH_DISCRETIZE, "adjoint": _lib.CIS_BATCH_ADJOINT}


class BatchPlan:
    """Many trajectories (of one or several models) discretized together.

    ``trajs`` is a list of dicts with keys cm, X, U, s, params, K (inputs laid
    out as for :func:`discretize`).  The plan allocates, per trajectory, the
    outputs of the requested operations: A, Bm, Bp, S, d, xprop
    ("discretize"); d, xprop, seed (zeros, to be filled in place by the
    caller), gX, gU, gs, gp ("adjoint").  They are in ``self.out[i]`` and stay
    bound to the plan: each run overwrites them.
    """

    def __init__(self, trajs, ops=("discretize",), *, sched="tune", ckpt_every=0, graph=True,
                 adjoint_waves=None, waves_per_simd=None, defects_waves=None, form=None,
                 stream=None):
        lib = _lib.load()
        if not trajs:
            raise ValueError("a batch needs at least one trajectory")
        self.ops = 0
        for o in ops:
            self.ops |= _OPS[o]
        dtype = trajs[0]["X"].dtype
        self.out = []
        arr = (_lib.Traj * len(trajs))()
        for i, t in enumerate(trajs):
            cm, X, U, s, params = t["cm"], t["X"], t.get("U"), t["s"], t["params"]
            _check_inputs(cm, X, U, s, params)
            if X.dtype != dtype:
                raise ValueError("all trajectories of a batch share one dtype")
            N, nx, m = s.shape[0], cm.nx, cm.m
            kw = dict(device=X.device, dtype=dtype)
            o = dict(d=torch.empty((nx, N), **kw), xprop=torch.empty((nx, N), **kw))
            if self.ops & _lib.CIS_BATCH_DISCRETIZE:
                o.update(A=torch.empty((nx, nx, N), **kw), Bm=torch.empty((nx, m, N), **kw),
                         Bp=torch.empty((nx, m, N), **kw), S=torch.empty((nx, N), **kw))
            if self.ops & _lib.CIS_BATCH_ADJOINT:
                ld = X.stride(0)
                o.update(seed=torch.zeros((nx, N), **kw), gX=torch.empty((nx, ld), **kw),
                         gU=torch.empty((max(m, 1), ld), **kw), gs=torch.empty((N,), **kw),
                         gp=torch.empty((cm.np,), **kw))
            o["_in"] = (cm, X, U, s, params)   # keep the inputs alive with the plan
            self.out.append(o)
            tr = arr[i]
            tr.model = cm.handle.value
            tr.N, tr.substeps = N, int(t["K"])
            tr.ld_node, tr.ld_int = X.stride(0), N
            for name, ten in (("X", X), ("U", U if m else None), ("s", s), ("params", params)):
                setattr(tr, name, None if ten is None else ten.data_ptr())
            for name, key in (("A", "A"), ("Bm", "Bm"), ("Bp", "Bp"), ("S", "S"),
                              ("defect", "d"), ("xprop", "xprop"), ("seed", "seed"),
                              ("gX", "gX"), ("gU", "gU"), ("gs", "gs"), ("gparams", "gp")):
                ten = o.get(key)
                if key in ("Bm", "Bp", "gU") and m == 0:
                    ten = None
                setattr(tr, name, None if ten is None else ten.data_ptr())
        self._arr = arr
        h = ctypes.c_void_p()
        sched_code = _SCHED[sched]
        if adjoint_waves is not None:
            sched_code |= {1: _lib.CIS_SCHED_ADJ_1, 2: _lib.CIS_SCHED_ADJ_2,
                           3: _lib.CIS_SCHED_ADJ_3, 4: _lib.CIS_SCHED_ADJ_4}[int(adjoint_waves)]
        if waves_per_simd is not None:
            sched_code |= {1: _lib.CIS_SCHED_WAVES_1,
                           2: _lib.CIS_SCHED_WAVES_2}[int(waves_per_simd)]
        if defects_waves is not None:
            sched_code |= {2: _lib.CIS_SCHED_DEF_BODY,
                           1: _lib.CIS_SCHED_DEF_LANE}[int(defects_waves)]
        if form is not None:
            sched_code |= {"split": _lib.CIS_SCHED_SPLIT, "fused": _lib.CIS_SCHED_FUSED}[form]
        _lib.check(lib.cis_batch_plan_create(arr, len(trajs), _dtype_code(dtype), self.ops,
                                             sched_code, int(ckpt_every), int(bool(graph)),
                                             _stream(stream), ctypes.byref(h)))
        self._h = h
        self.graph = bool(graph)

    def run(self, op="discretize", *, graph=False, stream=None):
        """Enqueue one operation over the whole batch (graph replay if graph=True)."""
        lib = _lib.load()
        fn = lib.cis_batch_graph_run if graph else lib.cis_batch_run
        _lib.check(fn(self._h, _OPS[op], _stream(stream)))

    def run_part(self, op="discretize", part=0, *, stream=None):
        """Enqueue one launch of the operation for every model group (for timing
        the kernels one by one; parts of one run in order on one stream)."""
        lib = _lib.load()
        _lib.check(lib.cis_batch_run_part(self._h, _OPS[op], int(part), _stream(stream)))

    def groups(self):
        """Per model group: trajectories, items, units per item, persistent grid (0 = grid),
        waves of the reverse sweep, register budget of the discretize kernel, waves of the
        defects pass, and the discretize form (split: 1 for the two-launch form)."""
        lib = _lib.load()
        ng = ctypes.c_int32()
        _lib.check(lib.cis_batch_plan_info(self._h, -1, ctypes.byref(ng), None, None, None, None,
                                           None, None, None))
        res = []
        for g in range(ng.value):
            v = [ctypes.c_int32() for _ in range(7)]
            _lib.check(lib.cis_batch_plan_info(self._h, g, None, *[ctypes.byref(x) for x in v]))
            sp, tw, fc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _lib.check(lib.cis_batch_plan_discretize_form(self._h, g, ctypes.byref(sp),
                                                          ctypes.byref(tw)))
            _lib.check(lib.cis_batch_plan_tuned_from_cache(self._h, g, ctypes.byref(fc)))
            res.append(dict(n_traj=v[0].value, n_items=v[1].value, units_per_item=v[2].value,
                            persist_blocks=v[3].value, adjoint_waves=v[4].value,
                            waves_per_simd=v[5].value, defects_waves=v[6].value,
                            split=sp.value, from_cache=fc.value))
        return res

    def close(self):
        h = getattr(self, "_h", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.cis_batch_plan_destroy(h)
        self._h = None

    def __del__(self):
        self.close()
