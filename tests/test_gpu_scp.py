"""GPU parity of the SCP driver's transcription (Sec. V; Sec. VI): the HIP
transcriber against the oracle transcriber on the same iterate, then whole
SCP iterations with each."""
import numpy as np
import pytest

from paper_2604_09993_amd import scp, synth

from parity import PHI64, TOL64, block_err
from scp_oracle import oracle_transcriber

pytestmark = pytest.mark.gpu


def _problem(N=14, K=10, seed=0):
    model = synth.make_hopper(np.random.default_rng(seed))
    xi = synth.standing_state(model, 0.0)
    xf = synth.standing_state(model, 0.3)
    pb = scp.CitoProblem(model, N, xi, xf, K=K)
    g = synth.scp_initial_guess(model, N, xi, xf, 0.05, np.random.default_rng(seed + 1))
    z = pb.pack(g["Xp"], g["Xm"], g["Phi"], g["Gamma"], g["Ua"], g["Ub"], g["S"])
    return pb, z


@pytest.mark.parametrize("integrator", ["rk4", "rkf"])
def test_gpu_transcription_matches_the_oracle(integrator):
    pb, z = _problem()
    v = pb.unpack(z)
    print(f"scp transcription hopper N=14 K=10 {integrator}", flush=True)
    got = scp.GpuTranscriber(pb, integrator)(v, 0.5)
    ref = oracle_transcriber(pb, integrator)(v, 0.5)
    for key in ("A", "Bm", "Bp", "S", "d", "G", "Theta", "Psi", "JG", "JT"):
        err = block_err(got[key], ref[key], PHI64)
        assert err <= TOL64, (key, err)


def test_scp_iterations_with_gpu_transcription_match_the_oracle():
    pb, z0 = _problem()
    print("scp iterations hopper N=14 K=10 rk4 x3", flush=True)
    runs = []
    for tr in (scp.GpuTranscriber(pb), oracle_transcriber(pb)):
        drv = scp.ScpDriver(pb, tr)
        zs = []
        drv.run(z0, max_iter=3, callback=lambda rec, z: zs.append(z.copy()))
        runs.append((zs, drv.hom.delta, [r.qp_status for r in drv.history]))
    (zg, dg, sg), (zo, do, so) = runs
    assert dg == do
    for a, b in zip(zg, zo):
        assert np.max(np.abs(a - b) / pb.zscale) <= 1e-6
