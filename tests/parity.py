"""Shared helpers for comparing the HIP path with the CPU oracle.

Parity metric (per interval, per output block A, B-, B+, S, d, F~):
    err = max_e |G_e - O_e| / max(|O_e|, phi * max_e' |O_e'|)
FP64: phi = 1e-3, pass <= 1e-10.  FP32: phi = 1 (normwise), pass <= 1e-4,
with the oracle run in FP64 on the FP32-rounded inputs.
"""
import numpy as np

TOL64 = 1e-10
PHI64 = 1e-3
TOL32 = 1e-4
PHI32 = 1.0


def block_err(G, O, phi):
    """Worst per-interval error of a block; arrays are [N, ...]."""
    G = np.asarray(G, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    assert G.shape == O.shape, (G.shape, O.shape)
    if O.size == 0:
        return 0.0
    worst = 0.0
    for k in range(O.shape[0]):
        o, g = O[k], G[k]
        mx = np.max(np.abs(o))
        if mx == 0.0:
            e = np.max(np.abs(g))
            worst = max(worst, 0.0 if e == 0.0 else np.inf)
            continue
        denom = np.maximum(np.abs(o), phi * mx)
        worst = max(worst, float(np.max(np.abs(g - o) / denom)))
    return worst


def compare_outputs(gpu, ref, keys=("A", "Bm", "Bp", "S", "d", "xprop"), phi=PHI64):
    """Dict of block errors for the given keys (gpu arrays already interval-major numpy)."""
    return {k: block_err(gpu[k], ref[k], phi) for k in keys}
