"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects malformed arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2604_09993_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "cis.h")).read()
    return sorted(set(re.findall(r"\b(cis_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_symbols() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.cis_version()


def _desc(model):
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
    d = _lib.ModelDesc(model.nb, model.nj, model.nc, *ptrs, model.gravity,
                       model.terrain_amplitude, model.terrain_wavenumber)
    return d, keep


def _create(model):
    lib = _lib.load()
    d, keep = _desc(model)
    h = ctypes.c_void_p()
    st = lib.cis_model_create(ctypes.byref(d), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("name", ["free1", "point1", "hopper", "biped5", "cheetah7", "quad13"])
def test_model_create_and_dims(name):
    lib = _lib.load()
    model = synth.MODEL_MAKERS[name](np.random.default_rng(0))
    st, h = _create(model)
    assert st == _lib.CIS_OK, lib.cis_last_error()
    dims = [ctypes.c_int32() for _ in range(4)]
    assert lib.cis_model_dims(h, *[ctypes.byref(x) for x in dims]) == 0
    assert [x.value for x in dims] == [model.n, model.ny, model.m, model.n_params]
    lib.cis_model_destroy(h)


def test_model_create_rejects_bad_descriptions():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.cis_model_create(None, ctypes.byref(h)) == _lib.CIS_ERR_NULL
    model = synth.make_cheetah7(np.random.default_rng(0))
    bad = synth.make_cheetah7(np.random.default_rng(0))
    bad.link_length = bad.link_length.copy()
    bad.link_length[2] = -1.0
    assert _create(bad)[0] == _lib.CIS_ERR_MODEL
    bad = synth.make_cheetah7(np.random.default_rng(0))
    bad.joint_parent = bad.joint_parent.copy()
    bad.joint_parent[3] = 99
    assert _create(bad)[0] == _lib.CIS_ERR_MODEL
    bad = synth.make_cheetah7(np.random.default_rng(0))
    bad.contact_body = bad.contact_body.copy()
    bad.contact_body[0] = 1              # not a leg tip
    assert _create(bad)[0] == _lib.CIS_ERR_UNSUPPORTED
    bad = synth.legged_model("tri", 3, 2, np.random.default_rng(0))   # 3 legs not compiled
    assert _create(bad)[0] == _lib.CIS_ERR_UNSUPPORTED
    assert b"legs" in lib.cis_last_error()
    bad = synth.make_cheetah7(np.random.default_rng(0))
    bad.gravity = float("nan")
    assert _create(bad)[0] == _lib.CIS_ERR_MODEL
    assert _create(model)[0] == _lib.CIS_OK


def _call_discretize(h, shape, X=8, U=8, s=8, p=8, outs=(8, 8, 8, 8, 8, 0)):
    lib = _lib.load()
    ptr = lambda v: None if v == 0 else ctypes.c_void_p(v)
    return lib.cis_discretize(h, ctypes.byref(shape) if shape is not None else None, ptr(X), ptr(U),
                              ptr(s), ptr(p), *[ptr(o) for o in outs], None)


def _gpu_visible():
    import torch
    return torch.cuda.device_count() > 0


@pytest.mark.skipif("_gpu_visible()", reason="uses fake addresses; run only where no GPU exists")
def test_debug_mode_keeps_validation_before_launch(monkeypatch):
    """With CIS_DEBUG_FINITE set, invalid arguments are still refused before
    any launch and before the non-finite scan (fake addresses, never read)."""
    monkeypatch.setenv("CIS_DEBUG_FINITE", "1")
    model = synth.make_hopper(np.random.default_rng(0))
    st, h = _create(model)
    assert st == 0
    good = _lib.Shape(5, 4, _lib.CIS_F64, 0, 6, 5)
    assert _call_discretize(h, _lib.Shape(5, 4, 0, 0, 5, 5)) == _lib.CIS_ERR_DIM
    assert _call_discretize(h, good, X=0) == _lib.CIS_ERR_NULL
    assert _call_discretize(h, good, X=12) == _lib.CIS_ERR_LAYOUT
    lib = _lib.load()
    P = lambda v: ctypes.c_void_p(v)
    assert lib.cis_defects(h, ctypes.byref(good), P(8), P(8), P(8), P(8), None, None, None, 0,
                           None) == _lib.CIS_ERR_NULL
    lib.cis_model_destroy(h)


@pytest.mark.skipif("_gpu_visible()", reason="uses fake addresses; run only where no GPU exists")
def test_entry_points_validate_before_launch():
    """Every rejection returns before any HIP call (fake, never-dereferenced addresses)."""
    lib = _lib.load()
    model = synth.make_hopper(np.random.default_rng(0))
    st, h = _create(model)
    assert st == 0
    good = _lib.Shape(5, 4, _lib.CIS_F64, 0, 6, 5)
    assert _call_discretize(h, None) == _lib.CIS_ERR_NULL
    assert _call_discretize(None, good) == _lib.CIS_ERR_NULL
    assert _call_discretize(h, _lib.Shape(0, 4, 0, 0, 6, 5)) == _lib.CIS_ERR_DIM
    assert _call_discretize(h, _lib.Shape(5, 0, 0, 0, 6, 5)) == _lib.CIS_ERR_DIM
    assert _call_discretize(h, _lib.Shape(5, 5000, 0, 0, 6, 5)) == _lib.CIS_ERR_DIM
    assert _call_discretize(h, _lib.Shape(5, 4, 0, 0, 5, 5)) == _lib.CIS_ERR_DIM   # ld_node < N+1
    assert _call_discretize(h, _lib.Shape(5, 4, 0, 0, 6, 4)) == _lib.CIS_ERR_DIM   # ld_int < N
    assert _call_discretize(h, _lib.Shape(5, 4, 7, 0, 6, 5)) == _lib.CIS_ERR_DTYPE
    assert _call_discretize(h, _lib.Shape(5, 4, 0, 5, 6, 5)) == _lib.CIS_ERR_DIM   # layout > 4
    assert _call_discretize(h, _lib.Shape(5, 4, 0, -1, 6, 5)) == _lib.CIS_ERR_DIM
    assert _call_discretize(h, good, X=0) == _lib.CIS_ERR_NULL
    assert _call_discretize(h, good, U=0) == _lib.CIS_ERR_NULL                      # m > 0
    assert _call_discretize(h, good, X=12) == _lib.CIS_ERR_LAYOUT                   # misaligned
    assert _call_discretize(h, good, outs=(8, 0, 8, 8, 8, 0)) == _lib.CIS_ERR_NULL  # Bm missing
    assert _call_discretize(h, good, outs=(8, 8, 8, 8, 12, 0)) == _lib.CIS_ERR_LAYOUT
    # defects: ckpt stride must divide K
    P = lambda v: ctypes.c_void_p(v)
    assert lib.cis_defects(h, ctypes.byref(good), P(8), P(8), P(8), P(8), P(8), None, P(8), 3,
                           None) == _lib.CIS_ERR_DIM
    assert lib.cis_defects(h, ctypes.byref(good), P(8), P(8), P(8), P(8), None, None, None, 0,
                           None) == _lib.CIS_ERR_NULL
    assert lib.cis_status_string(_lib.CIS_ERR_DIM) == b"dimension out of range"
    assert lib.cis_status_string(_lib.CIS_ERR_NONFINITE) == b"non-finite values (debug mode)"
    # workspaces: missing or short workspaces are refused before any launch
    need = ctypes.c_size_t(0)
    assert lib.cis_adjoint_workspace_size(h, ctypes.byref(good), ctypes.byref(need)) == 0
    assert need.value == (2 * model.m + model.n_params) * 5 * 8
    adj = lambda ws, nb: lib.cis_discretize_adjoint(h, ctypes.byref(good), P(8), P(8), P(8), P(8),
                                                     P(8), 2, P(8), P(8), P(8), P(8), P(8), ws,
                                                     nb, None)
    assert adj(None, need.value) == _lib.CIS_ERR_WORKSPACE
    assert adj(P(8), need.value - 8) == _lib.CIS_ERR_WORKSPACE
    sh4 = _lib.Shape(5, 4, _lib.CIS_F64, 0, 6, 5)
    assert lib.cis_blocked_workspace_size(h, ctypes.byref(sh4), 2, ctypes.byref(need)) == 0
    blk = lambda ws, nb: lib.cis_discretize_blocked(h, ctypes.byref(sh4), P(8), P(8), P(8), P(8),
                                                    2, _lib.CIS_COMPOSE_VALU, P(8), P(8), P(8),
                                                    P(8), P(8), None, ws, nb, None)
    assert blk(None, need.value) == _lib.CIS_ERR_WORKSPACE
    assert blk(P(8), need.value - 8) == _lib.CIS_ERR_WORKSPACE
    # the single-trajectory tuner: the choice output is required, the shape
    # names no layout (the tuner picks it)
    ch = _lib.SingleChoice()
    tune = lambda sh, c: lib.cis_single_tune(h, ctypes.byref(sh), P(8), P(8), P(8), P(8), P(8),
                                             P(8), P(8), P(8), P(8), None, c, None)
    assert tune(sh4, None) == _lib.CIS_ERR_NULL
    assert tune(_lib.Shape(5, 4, _lib.CIS_F64, 3, 6, 5), ctypes.byref(ch)) == _lib.CIS_ERR_DIM
    assert tune(_lib.Shape(5, 4, 7, 0, 6, 5), ctypes.byref(ch)) == _lib.CIS_ERR_DTYPE
    # the allocation-free reverse sweep holds (2 m + P) N <= 2^20 doubles
    big = (1 << 20) // (2 * model.m + model.n_params) + 1
    shb = _lib.Shape(big, 4, _lib.CIS_F64, 0, big + 1, big)
    assert lib.cis_discretize_adjoint_noalloc(h, ctypes.byref(shb), P(8), P(8), P(8), P(8), P(8),
                                              2, P(8), P(8), P(8), P(8), P(8),
                                              None) == _lib.CIS_ERR_WORKSPACE
    assert b"cis_discretize_adjoint_noalloc" in lib.cis_last_error()
    assert lib.cis_discretize_adjoint_noalloc(h, None, P(8), P(8), P(8), P(8), P(8), 2, P(8),
                                              P(8), P(8), P(8), P(8), None) == _lib.CIS_ERR_NULL
    # impact map: sizes, delta, required pointers, alignment; n_nodes = 0 is a no-op
    imp = lambda n, ld, dl=1e-3, eps=0.0, ptrs=(8,) * 10: lib.cis_impact_linearize(
        h, n, ld, *[P(v) if v else None for v in ptrs[:5]], dl, eps,
        *[P(v) if v else None for v in ptrs[5:]], None)
    assert imp(4, 3) == _lib.CIS_ERR_DIM                       # ld_node < n_nodes
    assert imp(-1, 3) == _lib.CIS_ERR_DIM
    assert imp(4, 4, dl=0.0) == _lib.CIS_ERR_DIM
    assert imp(4, 4, dl=float("nan")) == _lib.CIS_ERR_DIM
    assert imp(4, 4, eps=float("inf")) == _lib.CIS_ERR_DIM
    assert imp(4, 4, ptrs=(8, 8, 0, 8, 8, 8, 8, 8, 8, 8)) == _lib.CIS_ERR_NULL   # Phi, nc > 0
    assert imp(4, 4, ptrs=(8, 8, 8, 8, 8, 8, 8, 0, 8, 8)) == _lib.CIS_ERR_NULL   # JGv
    assert imp(4, 4, ptrs=(8, 8, 8, 8, 8, 8, 8, 8, 12, 8)) == _lib.CIS_ERR_LAYOUT
    assert imp(0, 1, ptrs=(0,) * 10) == 0
    assert lib.cis_impact_linearize(None, 4, 4, *[P(8)] * 5, 1e-3, 0.0, *[P(8)] * 5,
                                    None) == _lib.CIS_ERR_NULL
    # paper-dynamics form: FP64 only, workspace checked
    need = ctypes.c_size_t(0)
    assert lib.cis_paper_workspace_size(h, ctypes.byref(good), ctypes.byref(need)) == 0
    sh32 = _lib.Shape(5, 4, _lib.CIS_F32, 0, 6, 5)
    pap = lambda sh, ws, nb: lib.cis_discretize_paper(h, ctypes.byref(sh), P(8), P(8), P(8), P(8),
                                                      P(8), P(8), P(8), P(8), P(8), None, ws, nb,
                                                      None)
    assert pap(sh32, P(8), need.value) == _lib.CIS_ERR_DTYPE
    assert pap(good, None, need.value) == _lib.CIS_ERR_WORKSPACE
    assert pap(good, P(8), need.value - 8) == _lib.CIS_ERR_WORKSPACE
    pd = [ctypes.c_int32() for _ in range(2)]
    assert lib.cis_paper_dims(h, *[ctypes.byref(d) for d in pd]) == 0
    assert [d.value for d in pd] == [6 * model.nb + 4 * model.nc + 1, model.nj + 3 * model.nc]
    # RKF form: workspace checked
    assert lib.cis_rkf_workspace_size(h, ctypes.byref(good), ctypes.byref(need)) == 0
    rkf = lambda ws, nb: lib.cis_discretize_rkf(h, ctypes.byref(good), P(8), P(8), P(8), P(8), 1,
                                                P(8), P(8), P(8), P(8), P(8), None, None, ws, nb,
                                                None)
    assert rkf(None, need.value) == _lib.CIS_ERR_WORKSPACE
    assert rkf(P(8), need.value - 8) == _lib.CIS_ERR_WORKSPACE
    dims = [ctypes.c_int32() for _ in range(3)]
    assert lib.cis_impact_dims(h, *[ctypes.byref(d) for d in dims]) == 0
    assert [d.value for d in dims] == [10 * model.nc, 7 * model.nb + 2 * model.nc, 14]
    lib.cis_model_destroy(h)


_LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "cis.h"
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("cis_shape size %zu\n", sizeof(cis_shape));
  F(cis_shape, N) F(cis_shape, substeps) F(cis_shape, dtype) F(cis_shape, ld_node) F(cis_shape, ld_int)
  printf("cis_model_desc size %zu\n", sizeof(cis_model_desc));
  F(cis_model_desc, link_length) F(cis_model_desc, contact_point) F(cis_model_desc, gravity)
  F(cis_model_desc, terrain_wavenumber)
  printf("cis_traj size %zu\n", sizeof(cis_traj));
  F(cis_traj, N) F(cis_traj, ld_node) F(cis_traj, X) F(cis_traj, A) F(cis_traj, xprop)
  F(cis_traj, seed) F(cis_traj, gparams)
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of cis_shape, cis_model_desc and cis_traj have the C layout."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        t, f, v = line.split()
        got[(t, f)] = int(v)
    mirrors = {"cis_shape": _lib.Shape, "cis_model_desc": _lib.ModelDesc, "cis_traj": _lib.Traj}
    for (t, f), v in got.items():
        cls = mirrors[t]
        if f == "size":
            assert ctypes.sizeof(cls) == v, t
        else:
            assert getattr(cls, f).offset == v, (t, f)


def _traj(h, **kw):
    t = _lib.Traj()
    t.model = h.value
    t.N, t.substeps, t.ld_node, t.ld_int = 5, 4, 6, 5
    for name in ("X", "U", "s", "params", "A", "Bm", "Bp", "S", "defect", "xprop", "seed",
                 "gX", "gU", "gs", "gparams"):
        setattr(t, name, 8)
    for k, v in kw.items():
        setattr(t, k, v)
    return t


@pytest.mark.skipif("_gpu_visible()", reason="uses fake addresses; run only where no GPU exists")
def test_batch_plan_validates_before_any_device_call():
    lib = _lib.load()
    st, h = _create(synth.make_hopper(np.random.default_rng(0)))
    assert st == 0
    plan = ctypes.c_void_p()

    def create(trajs, n=None, dtype=_lib.CIS_F64, ops=_lib.CIS_BATCH_DISCRETIZE,
               sched=_lib.CIS_SCHED_GRID, ckpt=0):
        arr = (_lib.Traj * len(trajs))(*trajs)
        return lib.cis_batch_plan_create(arr, len(trajs) if n is None else n, dtype, ops, sched,
                                         ckpt, 0, None, ctypes.byref(plan))

    good = _traj(h)
    assert lib.cis_batch_plan_create(None, 1, 0, 1, 1, 0, 0, None, ctypes.byref(plan)) == _lib.CIS_ERR_NULL
    assert create([good], n=0) == _lib.CIS_ERR_DIM
    assert create([good], dtype=9) == _lib.CIS_ERR_DTYPE
    assert create([good], ops=0) == _lib.CIS_ERR_DIM
    assert create([good], ops=4) == _lib.CIS_ERR_DIM
    assert create([good], sched=0) == _lib.CIS_ERR_DIM
    assert create([good], sched=_lib.CIS_SCHED_GRID | 0x2000) == _lib.CIS_ERR_DIM   # unknown bit
    assert create([good], sched=_lib.CIS_SCHED_TUNE | _lib.CIS_SCHED_SPLIT
                  | _lib.CIS_SCHED_FUSED) == _lib.CIS_ERR_DIM
    two_def = _lib.CIS_SCHED_DEF_BODY | _lib.CIS_SCHED_DEF_LANE
    assert create([good], sched=_lib.CIS_SCHED_GRID | two_def) == _lib.CIS_ERR_DIM
    assert create([good], sched=_lib.CIS_SCHED_GRID | _lib.CIS_SCHED_ADJ_4
                  | _lib.CIS_SCHED_ADJ_1) == _lib.CIS_ERR_DIM                     # two forms
    both = _lib.CIS_SCHED_WAVES_1 | _lib.CIS_SCHED_WAVES_2
    assert create([good], sched=_lib.CIS_SCHED_GRID | both) == _lib.CIS_ERR_DIM
    assert create([_traj(h)], dtype=_lib.CIS_F32,
                  sched=_lib.CIS_SCHED_GRID | _lib.CIS_SCHED_WAVES_2) == _lib.CIS_ERR_DTYPE
    assert create([good], ops=_lib.CIS_BATCH_ADJOINT, dtype=_lib.CIS_F32) == _lib.CIS_ERR_DTYPE
    assert create([good, _traj(h, N=0)]) == _lib.CIS_ERR_DIM
    assert b"trajectory 1" in lib.cis_last_error()
    assert create([good, _traj(h, A=None)]) == _lib.CIS_ERR_NULL
    assert create([_traj(h, xprop=12)]) == _lib.CIS_ERR_LAYOUT
    assert create([_traj(h, seed=None)], ops=_lib.CIS_BATCH_ADJOINT) == _lib.CIS_ERR_NULL
    assert create([good], ops=_lib.CIS_BATCH_ADJOINT, ckpt=3) == _lib.CIS_ERR_DIM   # 3 does not divide 4
    assert create([good], ckpt=-1) == _lib.CIS_ERR_DIM
    assert not plan.value
    assert lib.cis_batch_run(None, 1, None) == _lib.CIS_ERR_NULL
    assert lib.cis_batch_graph_run(None, 1, None) == _lib.CIS_ERR_NULL
    lib.cis_batch_plan_destroy(None)
    lib.cis_model_destroy(h)
