"""Tuning cache (CIS_TUNE_CACHE) of the batch plans (GPU).

A tuned plan writes its per-group choices to the cache file; a second plan
over the same work reads them back without timing and makes the same
choices; a damaged file is treated as empty and rewritten.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2604_09993_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("split", "waves_per_simd", "persist_blocks", "defects_waves", "adjoint_waves")


def _trajs(api, dev):
    rng = np.random.default_rng(700)
    out = []
    for name, n in (("cheetah7", 3), ("hopper", 2)):
        model = synth.MODEL_MAKERS[name](rng)
        cm = api.CisModel(model)
        for _ in range(n):
            d = synth.gen_nodes(model, 10, rng, T=0.2)
            out.append(dict(cm=cm, K=4, X=api.to_device_soa(d["X"], dev),
                            U=api.to_device_soa(d["U"], dev), s=torch.tensor(d["s"], device=dev),
                            params=torch.tensor(d["p"], device=dev)))
    return out


def test_tuned_choices_are_cached_and_reproduced(tmp_path, monkeypatch):
    from paper_2604_09993_amd import api
    print("[gpu] tune cache: 3 cheetah7 + 2 hopper trajectories N=10 K=4", flush=True)
    sys.stdout.flush()
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CIS_TUNE_CACHE", str(path))
    dev = torch.device("cuda:0")
    trajs = _trajs(api, dev)
    p1 = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=False)
    g1 = p1.groups()
    p1.close()
    assert path.exists()
    data = json.loads(path.read_text())
    assert data["version"] == 1 and len(data["entries"]) == 2
    assert all(g["from_cache"] == 0 for g in g1)
    p2 = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=False)
    g2 = p2.groups()
    p2.close()
    assert all(g["from_cache"] == 1 for g in g2)
    for a, b in zip(g1, g2):
        assert {k: a[k] for k in KEYS} == {k: b[k] for k in KEYS}
    # a damaged file counts as empty: the plan tunes again and rewrites it
    path.write_text("{not json")
    p3 = api.BatchPlan(trajs, ("discretize", "adjoint"), sched="tune", graph=False)
    g3 = p3.groups()
    p3.close()
    assert all(g["from_cache"] == 0 for g in g3)
    assert len(json.loads(path.read_text())["entries"]) == 2
