"""Oracle transcription of an SCP iterate (test infrastructure): the same
arrays as the GPU transcriber of the SCP driver, from the CPU oracles."""
import numpy as np

import oracle
from oracle import impact


def oracle_transcriber(pb, integrator="rk4"):
    def tr(v, delta):
        Xd, Ud, sd = pb.doubled(v)
        if integrator == "rk4":
            out = oracle.discretize(pb.model, Xd, Ud, sd, pb.p, pb.K)
        else:
            out = oracle.discretize_rkf(pb.model, Xd, Ud, sd, pb.p, pb.K)
        res = {k: np.ascontiguousarray(out[k][0::2]) for k in ("A", "Bm", "Bp", "S", "d")}
        lin = impact.linearize(pb.model, v["Xp"], v["Xm"], v["Phi"], v["Gamma"], pb.p, delta)
        res["G"], res["Theta"] = lin["G"], lin["Theta"]
        res["JG"] = lin["JG"][:, :, :pb.NB]
        res["JT"] = lin["JT"][:, :, :pb.NB]
        nq = pb.nq
        res["Psi"] = np.stack([impact.psi(pb.model, v["Xp"][k][2 * nq:], v["Xm"][k + 1][2 * nq:],
                                          delta, pb.eps_ctcs) for k in range(pb.N)])
        return res
    return tr
