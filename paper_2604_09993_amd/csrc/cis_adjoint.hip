// Reverse-mode sweep (vector-Jacobian product) of the discrete RK4 map of
// every interval, for a cotangent seed lambda_k = dJ/dF~_k; the penalized
// defect merit of the SCP subproblem (Sec. V) is one such J.
//
//   k_adjoint : two waves per interval.  Chunks of at most 8 substeps are
//               replayed by one wave from the checkpoints (x at substeps 0, C,
//               2C, ..), their stage inputs kept in LDS, while the other wave
//               reverses the previously recorded chunk's classical RK4 stages:  kbar_i = h/6 w_i xbar + h a_{i+1} Xbar_{i+1},
//               Xbar_i = s J_x(X_i)^T kbar_i, xbar <- xbar + sum_i Xbar_i,
//               with the control, dilation and parameter adjoints gathered
//               along the way.  The transposed Jacobian product is the
//               adjoint of the element-parallel forward product: each joint
//               or contact lane scatters into per-element slots, each body
//               lane sums its slots (fixed order, no atomics).
//   k_adjoint_reduce : gU_k = (interval k, left half) + (interval k-1, right
//               half); gp = sum over intervals in index order; gX_N = 0.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/cis.h"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_body.hpp"
#include "cis_model.hpp"

namespace cis {

constexpr int CHUNK = 8;   // substeps whose stage inputs are kept in LDS at once

template <class T, class TP, int NSLOT = 2>
struct AdjShared {
    Interval<T, TP> iv;
    RhsScratch<T, TP> se[NSLOT];        // stage evaluations (state, F~, rotations) in flight
    RhsScratch<T, TP> scr;              // replay wave
    T coef[NSLOT][Coef<TP>::SIZE];      // their Jacobian coefficients
    T hist[2][CHUNK * 4][TP::NX];       // stage inputs (x part) of two chunks
    T kb[TP::NXT];                      // kbar of the current stage
    T xbs[TP::NX];                      // Xbar of the current stage
    T jslot[cmax(TP::NJ, 1)][8];        // th_p, th_c, w_p, w_c, x_p, x_c, y_p, y_c
    T cslot[cmax(TP::NC, 1)][6];        // x, y, th, xd, yd, w of the contact body
    T red[64];
};

// Reverse one RK4 stage whose input is sc.ns.  EVAL: evaluate the stage
// (right-hand side and Jacobian coefficients into sc and cf) here; otherwise
// another wave has done it.  Lanes own rows r = lane, lane + 64.
template <class T, class TP, bool EVAL, int NS>
__device__ __forceinline__ void reverse_stage(AdjShared<T, TP, NS>& ax, RhsScratch<T, TP>& sc,
                                              T* cf, const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                              int lane, int st, T tau, T (&xbar)[2],
                                              T (&xprev)[2], T (&xsum)[2], T& sacc,
                                              T (&uacc)[3][2], T& muacc, T& macc) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, NX = TP::NX;
    constexpr int NXT = TP::NXT, M = TP::M;
    using C = Coef<TP>;
    const Interval<T, TP>& iv = ax.iv;
    const T s = iv.s, h = iv.h;
    // kbar_st = h/6 w_st xbar + h a_{st+1} Xbar_{st+1}
    const T w = (st == 0 || st == 3) ? T(1) : T(2);
    const T anext = st == 2 ? h : T(0.5) * h;   // multiplier of k_st in stage st+1's input
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NXT) ax.kb[r] = iv.h6 * w * xbar[q] + (st < 3 ? anext * xprev[q] : T(0));
    }
    if constexpr (EVAL) rhs_eval<T, TP, EMIT>(iv, sc, mc, lane, tau, cf);   // ends with a wave sync
    else wave_lds_sync();
    const T omt = T(1) - tau;
    const T lc = ax.kb[NX + NC];
    // phase A: element lanes scatter into their slots; control adjoints.  The
    // joint and the contact terms are formed on every lane (element index
    // clamped to a valid one) so that their loads issue together; only the
    // owning lanes store and accumulate.
    const bool jl = lane < NJ, cl = lane >= NJ && lane < NJ + NC;
    if constexpr (NJ > 0) {
        const int j = jl ? lane : 0, p = TP::parent(j), c = j + 1;
        const T gp = ax.kb[NQ + 3 * p + 2], gc = ax.kb[NQ + 3 * c + 2];
        const T t1 = iv.kc[j][0] * gp - iv.kc[j][2] * gc;
        const T t2 = iv.kc[j][1] * gp - iv.kc[j][3] * gc;
        const T* jh = cf + C::JH + 4 * j;
        const T jh0 = jh[0], jh1 = jh[1], jh2 = jh[2], jh3 = jh[3];
        const T* gv = cf + C::GV;
        const T kxp = ax.kb[NQ + 3 * p], kyp = ax.kb[NQ + 3 * p + 1];
        const T kxc = ax.kb[NQ + 3 * c], kyc = ax.kb[NQ + 3 * c + 1];
        const int ut = j, ux = NJ + 2 * j, uy = NJ + 2 * j + 1;
        const T at = gv[(3 * p + 2) * M + ut] * gp + gv[(3 * c + 2) * M + ut] * gc;
        const T axx = gv[(3 * p) * M + ux] * kxp + gv[(3 * c) * M + ux] * kxc +
                      gv[(3 * p + 2) * M + ux] * gp + gv[(3 * c + 2) * M + ux] * gc;
        const T ayy = gv[(3 * p + 1) * M + uy] * kyp + gv[(3 * c + 1) * M + uy] * kyc +
                      gv[(3 * p + 2) * M + uy] * gp + gv[(3 * c + 2) * M + uy] * gc;
        if (jl) {
            ax.jslot[j][0] = -t1 + jh2 * lc;
            ax.jslot[j][1] = t1 + jh3 * lc;
            ax.jslot[j][2] = -t2;
            ax.jslot[j][3] = t2;
            ax.jslot[j][4] = jh0 * lc;
            ax.jslot[j][5] = -jh0 * lc;
            ax.jslot[j][6] = jh1 * lc;
            ax.jslot[j][7] = -jh1 * lc;
            uacc[0][0] += omt * at;  uacc[0][1] += tau * at;
            uacc[1][0] += omt * axx; uacc[1][1] += tau * axx;
            uacc[2][0] += omt * ayy; uacc[2][1] += tau * ayy;
        }
    }
    if constexpr (NC > 0) {
        const int i = cl ? lane - NJ : 0, b = TP::cbody(i);
        const T* ct = cf + C::CT + C::NCT * i;
        const T kx = ax.kb[NQ + 3 * b], ky = ax.kb[NQ + 3 * b + 1], kw = ax.kb[NQ + 3 * b + 2];
        const T kcc = ax.kb[NX + i];
        const T pbx = ct[C_FXP] * kx + ct[C_FYP] * ky + ct[C_TP] * kw + ct[C_EPX] * kcc +
                      ct[C_ZPX] * lc;
        const T pby = ct[C_EPY] * kcc + ct[C_ZPY] * lc;
        const T c2 = -ct[C_AY] * pbx + ct[C_AX] * pby + ct[C_ETH] * kcc;
        const T c3 = ct[C_EXD] * kcc, c4 = ct[C_EYD] * kcc, c5 = ct[C_EOM] * kcc;
        const T jmu = ct[C_JMU] * kcc;
        const T* gv = cf + C::GV;
        const T* gc = cf + C::GC + i * M;
        const int u0 = 3 * NJ + 3 * i;
        T inst[3], bar[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int u = u0 + q;
            inst[q] = gv[(3 * b) * M + u] * kx + gv[(3 * b + 1) * M + u] * ky +
                      gv[(3 * b + 2) * M + u] * kw;
            bar[q] = gc[u] * kcc;
        }
        if (cl) {
            ax.cslot[i][0] = pbx;
            ax.cslot[i][1] = pby;
            ax.cslot[i][2] = c2;
            ax.cslot[i][3] = c3;
            ax.cslot[i][4] = c4;
            ax.cslot[i][5] = c5;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                uacc[q][0] += omt * inst[q] + bar[q];
                uacc[q][1] += tau * inst[q] + bar[q];
            }
            muacc += jmu;
        }
    }
    wave_lds_sync();
    // phase B: body lanes gather their slots into Xbar of the stage
    if (lane < NB) {
        const int b = lane;
        T xq = T(0), yq = T(0), th = T(0), xd = T(0), yd = T(0), om = T(0);
        auto contact = [&](int i) {
            xq += ax.cslot[i][0];
            yq += ax.cslot[i][1];
            th += ax.cslot[i][2];
            xd += ax.cslot[i][3];
            yd += ax.cslot[i][4];
            om += ax.cslot[i][5];
        };
        if constexpr (TP::D > 0) {
            // every lane reads the slots of all its possible elements (torso:
            // the L first joints; link: its own joint, the next joint or its
            // contact) so that the loads issue together; weights keep the
            // owning ones (x + 0 == x, so the sums are those of the owners)
            constexpr int D = TP::D;
            const bool link = b >= 1;
            const bool has_next = link && b % D != 0, foot = link && b % D == 0;
            auto take = [&](bool on, const T* e, int i0, int i1, int i2, int i3) {
                const T w = on ? T(1) : T(0);
                th += w * e[i0];
                om += w * e[i1];
                xq += w * e[i2];
                yq += w * e[i3];
            };
            take(link, ax.jslot[link ? b - 1 : 0], 1, 3, 5, 7);   // own joint, as child
#pragma unroll
            for (int l = 0; l < TP::L; ++l) {                       // as parent
                const bool on = link ? (l == 0 && has_next) : true;
                const int j = link ? (has_next ? b : 0) : l * D;
                take(on, ax.jslot[j], 0, 2, 4, 6);
            }
            {
                const int i = foot ? b / D - 1 : 0;
                const T w = foot ? T(1) : T(0);
                xq += w * ax.cslot[i][0];
                yq += w * ax.cslot[i][1];
                th += w * ax.cslot[i][2];
                xd += w * ax.cslot[i][3];
                yd += w * ax.cslot[i][4];
                om += w * ax.cslot[i][5];
            }
        } else if (b == 0) {
#pragma unroll
            for (int l = 0; l < TP::L; ++l) contact(l);
        }
        const T gw = ax.kb[NQ + 3 * b + 2];
        ax.xbs[3 * b] = xq;
        ax.xbs[3 * b + 1] = yq;
        ax.xbs[3 * b + 2] = th + cf[C::CTH + b] * gw;
        ax.xbs[NQ + 3 * b] = s * ax.kb[3 * b] + xd;
        ax.xbs[NQ + 3 * b + 1] = s * ax.kb[3 * b + 1] + yd;
        ax.xbs[NQ + 3 * b + 2] = s * ax.kb[3 * b + 2] + om;
        // d(s v')/d m_b = -(s/m_b) (v'_x, v'_y + g, w')
        macc -= s * iv.minv[b] *
                (sc.fn[NQ + 3 * b] * ax.kb[NQ + 3 * b] +
                 (sc.fn[NQ + 3 * b + 1] + T(mc.g)) * ax.kb[NQ + 3 * b + 1] +
                 sc.fn[NQ + 3 * b + 2] * ax.kb[NQ + 3 * b + 2]);
    }
    wave_lds_sync();
    // rows: collect Xbar_i, dilation adjoint F~ . kbar
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NX) {
            const T xb = ax.xbs[r];
            xsum[q] += xb;
            xprev[q] = xb;
        } else {
            xprev[q] = T(0);
        }
        if (r < NXT) {
            const T F = r < NQ ? sc.ns[NQ + r] : sc.fn[r];
            sacc += F * ax.kb[r];
        }
    }
    // With EVAL the next stage's evaluation rewrites sc, read above by other
    // lanes.  Without it the callers pass a workgroup barrier before the next
    // stage, and the only LDS the next stage writes before its first wave sync
    // is each lane's own kb rows, read above by the same lane.
    if constexpr (EVAL) wave_lds_sync();
}

// Outputs of the reverse wave: gX_k, the control partials of interval k
// (left: U_k, right: U_k+1), the dilation and parameter adjoints.
template <class T, class TP, int NS>
__device__ __forceinline__ void adjoint_outputs(AdjShared<T, TP, NS>& ax, const AdjArgs<T>& a,
                                                const int k, const int lane, const T (&xbar)[2],
                                                T sacc, const T (&uacc)[3][2], T muacc, T macc) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NXT = TP::NXT;
    const FwdArgs<T>& f = a.f;
    // gX_k = xbar
    const int64_t ldn = f.ldn;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NXT) a.gX[r * ldn + k] = xbar[q];
    }
    const int N = f.N;
    // control adjoints of this interval (left: U_k, right: U_k+1)
    if (lane < NJ) {
        const int us[3] = {lane, NJ + 2 * lane, NJ + 2 * lane + 1};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a.ws_uk[(int64_t)us[q] * N + k] = uacc[q][0];
            a.ws_uk1[(int64_t)us[q] * N + k] = uacc[q][1];
        }
    } else if (lane < NJ + NC) {
        const int u0 = 3 * NJ + 3 * (lane - NJ);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a.ws_uk[(int64_t)(u0 + q) * N + k] = uacc[q][0];
            a.ws_uk1[(int64_t)(u0 + q) * N + k] = uacc[q][1];
        }
    }
    // dilation adjoint: fixed-order sum of the lane partials
    ax.red[lane] = sacc;
    wave_lds_sync();
    if (lane == 0) {
        T acc = T(0);
        for (int l = 0; l < 64; ++l) acc += ax.red[l];
        a.gs[k] = acc;
    }
    wave_lds_sync();
    ax.red[lane] = muacc;
    wave_lds_sync();
    if (lane == 0) {
        T acc = T(0);
        for (int l = NJ; l < NJ + NC; ++l) acc += ax.red[l];
        a.ws_p[k] = acc;                 // mu
        a.ws_p[(int64_t)N + k] = T(0);   // restitution: no dependence on this path
    }
    if (lane < NB) a.ws_p[(int64_t)(2 + lane) * N + k] = macc;
}

// Chunk u of an interval's reverse order (segment g = nseg-1 - u / nch, chunk
// offset c0 inside the segment, len substeps).
struct ChunkPos {
    int g, c0, len;
};
__device__ __forceinline__ ChunkPos chunk_pos(int u, int nseg, int nch, int Cs) {
    ChunkPos c;
    c.g = nseg - 1 - u / nch;
    c.c0 = (nch - 1 - u % nch) * CHUNK;
    c.len = (Cs - c.c0) < CHUNK ? (Cs - c.c0) : CHUNK;
    return c;
}

// Replay from checkpoint g to the end of the chunk, recording the chunk's
// stage inputs (x part) into hist.  One wave, scratch ax.scr.
template <class T, class TP>
__device__ __forceinline__ void replay_chunk(AdjShared<T, TP>& ax, const FwdArgs<T>& f,
                                             const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                             const int k, const int lane, const ChunkPos cp,
                                             T (*hist)[TP::NX]) {
    constexpr int NX = TP::NX, NXT = TP::NXT;
    const int64_t ldi = f.ldi;
    RowState<T> rs;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        rs.xb[q] = r < NX ? f.ckpt[((int64_t)cp.g * NX + r) * ldi + k] : T(0);
        rs.xa[q] = T(0);
        if (r < NXT) ax.scr.ns[r] = rs.xb[q];
    }
    wave_lds_sync();
    const int base = cp.g * f.C;
    for (int jj = 0; jj < cp.c0 + cp.len; ++jj) {
        const int j = base + jj;
        for (int st = 0; st < 4; ++st) {
            if (jj >= cp.c0) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int r = lane + 64 * q;
                    if (r < NX) hist[(jj - cp.c0) * 4 + st][r] = ax.scr.ns[r];
                }
            }
            const T tau = (T(j) + T(stage_c(st))) / T(f.K);
            rhs_eval<T, TP, LEAN>(ax.iv, ax.scr, mc, lane, tau, (T*)nullptr);
            rk_rows<T, TP, NX>(ax.iv, ax.scr, rs, lane, st, ax.scr.ns, (T*)nullptr);
        }
    }
    wave_lds_sync();
}

// Reverse sweep over a recorded chunk (stages evaluated here).
template <class T, class TP>
__device__ __forceinline__ void reverse_chunk(AdjShared<T, TP>& ax, const FwdArgs<T>& f,
                                              const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                              const int lane, const ChunkPos cp,
                                              const T (*hist)[TP::NX], T (&xbar)[2],
                                              T (&xprev)[2], T (&xsum)[2], T& sacc,
                                              T (&uacc)[3][2], T& muacc, T& macc) {
    constexpr int NX = TP::NX;
    const int base = cp.g * f.C;
    for (int jj = cp.len - 1; jj >= 0; --jj) {
        const int j = base + cp.c0 + jj;
        for (int st = 3; st >= 0; --st) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int r = lane + 64 * q;
                if (r < NX) ax.se[0].ns[r] = hist[jj * 4 + st][r];
            }
            wave_lds_sync();
            const T tau = (T(j) + T(stage_c(st))) / T(f.K);
            reverse_stage<T, TP, true>(ax, ax.se[0], ax.coef[0], mc, lane, st, tau, xbar, xprev,
                                       xsum, sacc, uacc, muacc, macc);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            xbar[q] += xsum[q];
            xsum[q] = T(0);
            xprev[q] = T(0);
        }
    }
}

// One interval by NW waves.  NW = 2: the replay wave records chunk u+1 while
// the reverse wave sweeps chunk u (two history buffers, one workgroup barrier
// per chunk).  NW = 1: one wave replays and reverses each chunk in turn (the
// fewest wave-cycles per interval, for batches).
template <class T, class TP, int NW>
__device__ __forceinline__ void adjoint_item(AdjShared<T, TP>& ax, const AdjArgs<T>& a,
                                             const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                             const int k) {
    constexpr int NXT = TP::NXT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = 64 * NW;
    const FwdArgs<T>& f = a.f;
    load_interval<T, TP>(ax.iv, f, mc, k, tid, nth);
    for (int e = tid; e < 2 * Coef<TP>::SIZE; e += nth) (&ax.coef[0][0])[e] = T(0);
    __syncthreads();
    coef_constants<T, TP>(ax.iv, ax.coef[0], tid, nth);
    coef_constants<T, TP>(ax.iv, ax.coef[1], tid, nth);
    __syncthreads();

    const int64_t ldi = f.ldi;
    const int Cs = f.C;
    const int nseg = f.K / Cs;
    const int nch = (Cs + CHUNK - 1) / CHUNK;   // chunks per checkpoint segment
    const int U = nseg * nch;                   // chunks, last first
    if (NW == 2 && wave == 1) {
        for (int t = 0; t <= U; ++t) {
            if (t < U) replay_chunk<T, TP>(ax, f, mc, k, lane, chunk_pos(t, nseg, nch, Cs),
                                           ax.hist[t & 1]);
            __syncthreads();
        }
        return;
    }
    T xbar[2], xprev[2], xsum[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        xbar[q] = r < NXT ? a.seed[r * ldi + k] : T(0);
        xprev[q] = T(0);
        xsum[q] = T(0);
    }
    T sacc = T(0), muacc = T(0), macc = T(0);
    T uacc[3][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    if constexpr (NW == 2) {
        for (int t = 0; t <= U; ++t) {
            if (t >= 1)
                reverse_chunk<T, TP>(ax, f, mc, lane, chunk_pos(t - 1, nseg, nch, Cs),
                                     ax.hist[(t - 1) & 1], xbar, xprev, xsum, sacc, uacc, muacc,
                                     macc);
            __syncthreads();
        }
    } else {
        for (int u = 0; u < U; ++u) {
            const ChunkPos cp = chunk_pos(u, nseg, nch, Cs);
            replay_chunk<T, TP>(ax, f, mc, k, lane, cp, ax.hist[0]);
            reverse_chunk<T, TP>(ax, f, mc, lane, cp, ax.hist[0], xbar, xprev, xsum, sacc, uacc,
                                 muacc, macc);
        }
    }
    adjoint_outputs<T, TP>(ax, a, k, lane, xbar, sacc, uacc, muacc, macc);
}

// Body-lane replay wave of the four-wave reverse sweep (checkpoints at most
// CHUNK substeps apart): at step 0 it records the stage inputs of the last
// checkpoint segment, then one stage per step those of the segment before,
// into the other history buffer.  (The three-wave form keeps the
// element-lane replay: fewer registers, which batches need for occupancy.)
template <class T, class TP, int NS>
__device__ __forceinline__ void replay_wave(AdjShared<T, TP, NS>& ax, const FwdArgs<T>& f,
                                            const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                            const int k, const int lane, const int nsteps) {
    constexpr int NX = TP::NX;
    const int64_t ldi = f.ldi;
    const int K = f.K, Cs = f.C;
    const int nseg = K / Cs, S4 = 4 * Cs;
    const int nst = 4 * K;
    // One lane per body runs the nominal RK4 stages (the state wave of the
    // forward kernel) and writes each next stage input straight into the
    // chunk's history; one workgroup barrier per step.
    constexpr int NB = TP::NB, NQ = TP::NQ;
    const BodyConst<T, TP> c = body_const<T, TP>(ax.iv, mc, lane);
    BodyRK<T> bs;
#pragma unroll
    for (int kk = 0; kk < 6; ++kk) bs.xb[kk] = bs.xs[kk] = bs.xa[kk] = T(0);
    for (int t = 0; t < nsteps; ++t) {
        int u = -1, q0 = 0, q1 = 0;   // record stages [q0, q1) of chunk u
        if (t == 0) {
            u = 0;
            q1 = S4;
        } else if (t <= nst) {
            const int r = t - 1;
            u = r / S4 + 1;
            q0 = r % S4;
            q1 = q0 + 1;
            if (u >= nseg) u = -1;
        }
        if (u >= 0) {
            const int g = nseg - 1 - u;
            T(*hist)[NX] = ax.hist[u & 1];
            for (int q = q0; q < q1; ++q) {
                if (q == 0 && lane < NB) {
                    const T* ck = f.ckpt + (int64_t)g * NX * ldi + k;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        bs.xb[kk] = ck[(3 * c.b + kk) * ldi];
                        bs.xb[3 + kk] = ck[(NQ + 3 * c.b + kk) * ldi];
                    }
#pragma unroll
                    for (int kk = 0; kk < 6; ++kk) {
                        bs.xs[kk] = bs.xb[kk];
                        bs.xa[kk] = T(0);
                    }
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        hist[0][3 * c.b + kk] = bs.xs[kk];
                        hist[0][NQ + 3 * c.b + kk] = bs.xs[3 + kk];
                    }
                }
                const int jj = q >> 2, st = q & 3, j = g * Cs + jj;
                const T tau = (T(j) + T(stage_c(st))) / T(K);
                // the state after the segment's last stage is not needed
                T* nxt = q + 1 < S4 ? hist[q + 1] : ax.scr.ns;
                switch (st) {
                    case 0:
                        state_stage<T, TP, 0>(ax.iv, mc, c, bs, tau, nxt, ax.scr.cs,
                                              ax.scr.fn, lane);
                        break;
                    case 1:
                        state_stage<T, TP, 1>(ax.iv, mc, c, bs, tau, nxt, ax.scr.cs,
                                              ax.scr.fn, lane);
                        break;
                    case 2:
                        state_stage<T, TP, 2>(ax.iv, mc, c, bs, tau, nxt, ax.scr.cs,
                                              ax.scr.fn, lane);
                        break;
                    default:
                        state_stage<T, TP, 3>(ax.iv, mc, c, bs, tau, nxt, ax.scr.cs,
                                              ax.scr.fn, lane);
                        break;
                }
            }
            wave_lds_sync();
        }
        __syncthreads();
    }
}

// Checkpoints at most CHUNK substeps apart (one chunk per segment, 4C stages
// each): three waves pipelined stage by stage, one workgroup barrier per step.
// With r the stage index counted backwards from the end of the interval:
//   step 0      : the replay wave records the last segment's stage inputs;
//   step t >= 1 : the evaluation wave evaluates stage r = t-1 (right-hand side
//                 and Jacobian coefficients into slot t & 1), the reverse wave
//                 reverses stage r = t-2 (slot (t-1) & 1), and the replay wave
//                 records one stage of the next segment;
//   4K + 2 steps in all.
template <class T, class TP>
__device__ __forceinline__ void adjoint_item3(AdjShared<T, TP>& ax, const AdjArgs<T>& a,
                                              const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                              const int k) {
    constexpr int NX = TP::NX, NXT = TP::NXT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = 192;
    const FwdArgs<T>& f = a.f;
    load_interval<T, TP>(ax.iv, f, mc, k, tid, nth);
    for (int e = tid; e < 2 * Coef<TP>::SIZE; e += nth) (&ax.coef[0][0])[e] = T(0);
    __syncthreads();
    coef_constants<T, TP>(ax.iv, ax.coef[0], tid, nth);
    coef_constants<T, TP>(ax.iv, ax.coef[1], tid, nth);
    __syncthreads();

    const int64_t ldi = f.ldi;
    const int K = f.K, Cs = f.C;
    const int nseg = K / Cs, S4 = 4 * Cs;
    const int nst = 4 * K, nsteps = nst + 2;
    if (wave == 1) {
        // ---------------- replay wave ----------------
        RowState<T> rs;
        for (int t = 0; t < nsteps; ++t) {
            int u = -1, q0 = 0, q1 = 0;   // record stages [q0, q1) of chunk u
            if (t == 0) {
                u = 0;
                q1 = S4;
            } else if (t <= nst) {
                const int r = t - 1;
                u = r / S4 + 1;
                q0 = r % S4;
                q1 = q0 + 1;
                if (u >= nseg) u = -1;
            }
            if (u >= 0) {
                const int g = nseg - 1 - u;
                T(*hist)[NX] = ax.hist[u & 1];
                for (int q = q0; q < q1; ++q) {
                    if (q == 0) {
#pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            const int r = lane + 64 * i;
                            rs.xb[i] = r < NX ? f.ckpt[((int64_t)g * NX + r) * ldi + k] : T(0);
                            rs.xa[i] = T(0);
                            if (r < NXT) ax.scr.ns[r] = rs.xb[i];
                        }
                        wave_lds_sync();
                    }
                    const int jj = q >> 2, st = q & 3, j = g * Cs + jj;
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int r = lane + 64 * i;
                        if (r < NX) hist[q][r] = ax.scr.ns[r];
                    }
                    const T tau = (T(j) + T(stage_c(st))) / T(K);
                    rhs_eval<T, TP, LEAN>(ax.iv, ax.scr, mc, lane, tau, (T*)nullptr);
                    rk_rows<T, TP, NX>(ax.iv, ax.scr, rs, lane, st, ax.scr.ns, (T*)nullptr);
                }
                wave_lds_sync();
            }
            __syncthreads();
        }
        return;
    }
    if (wave == 2) {
        // ---------------- evaluation wave ----------------
        for (int t = 0; t < nsteps; ++t) {
            if (t >= 1 && t <= nst) {
                const int r = t - 1, u = r / S4, pp = r % S4;
                const int g = nseg - 1 - u;
                const int jj = Cs - 1 - (pp >> 2), st = 3 - (pp & 3), j = g * Cs + jj;
                RhsScratch<T, TP>& sc = ax.se[t & 1];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int rr = lane + 64 * i;
                    if (rr < NX) sc.ns[rr] = ax.hist[u & 1][jj * 4 + st][rr];
                }
                wave_lds_sync();
                const T tau = (T(j) + T(stage_c(st))) / T(K);
                rhs_eval<T, TP, EMIT>(ax.iv, sc, mc, lane, tau, ax.coef[t & 1]);
            }
            __syncthreads();
        }
        return;
    }
    // ---------------- reverse wave ----------------
    T xbar[2], xprev[2], xsum[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        xbar[q] = r < NXT ? a.seed[r * ldi + k] : T(0);
        xprev[q] = T(0);
        xsum[q] = T(0);
    }
    T sacc = T(0), muacc = T(0), macc = T(0);
    T uacc[3][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    for (int t = 0; t < nsteps; ++t) {
        if (t >= 2) {
            const int r = t - 2, u = r / S4, pp = r % S4;
            const int g = nseg - 1 - u;
            const int jj = Cs - 1 - (pp >> 2), st = 3 - (pp & 3), j = g * Cs + jj;
            const T tau = (T(j) + T(stage_c(st))) / T(K);
            reverse_stage<T, TP, false>(ax, ax.se[(t - 1) & 1], ax.coef[(t - 1) & 1], mc, lane,
                                        st, tau, xbar, xprev, xsum, sacc, uacc, muacc, macc);
            if (st == 0) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    xbar[q] += xsum[q];
                    xsum[q] = T(0);
                    xprev[q] = T(0);
                }
            }
        }
        __syncthreads();
    }
    adjoint_outputs<T, TP>(ax, a, k, lane, xbar, sacc, uacc, muacc, macc);
}

// Checkpoints at most CHUNK substeps apart, four waves: the replay wave; two
// evaluation waves take alternate reverse stages,
// each evaluation spanning two pipeline steps (a workgroup barrier between its
// element wrenches and its smooth functions); the reverse wave applies stage
// r at step r + 3.  Four evaluation slots: at step t the reverse reads r = t-3
// while the evaluations of t-2 (second half) and t-1 (first half) write theirs.
template <class T, class TP>
__device__ __forceinline__ void adjoint_item4(AdjShared<T, TP, 4>& ax, const AdjArgs<T>& a,
                                              const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                              const int k) {
    constexpr int NX = TP::NX, NXT = TP::NXT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = 256;
    const FwdArgs<T>& f = a.f;
    load_interval<T, TP>(ax.iv, f, mc, k, tid, nth);
    for (int e = tid; e < 4 * Coef<TP>::SIZE; e += nth) (&ax.coef[0][0])[e] = T(0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) coef_constants<T, TP>(ax.iv, ax.coef[q], tid, nth);
    __syncthreads();

    const int64_t ldi = f.ldi;
    const int K = f.K, Cs = f.C;
    const int nseg = K / Cs, S4 = 4 * Cs;
    const int nst = 4 * K, nsteps = nst + 3;
    if (wave == 1) {
        replay_wave<T, TP>(ax, f, mc, k, lane, nsteps);
        return;
    }
    if (wave >= 2) {
        // ------- evaluation waves: reverse stages r = e, e+2, ... at steps r+1, r+2 -------
        const int e = wave - 2;
        int done = 0;   // workgroup barriers passed
        for (; done < e + 1; ++done) __syncthreads();
        for (int r = e; r < nst; r += 2) {
            const int u = r / S4, pp = r % S4;
            const int g = nseg - 1 - u;
            const int jj = Cs - 1 - (pp >> 2), st = 3 - (pp & 3), j = g * Cs + jj;
            RhsScratch<T, TP>& sc = ax.se[r & 3];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int rr = lane + 64 * i;
                if (rr < NX) sc.ns[rr] = ax.hist[u & 1][jj * 4 + st][rr];
            }
            wave_lds_sync();
            const T tau = (T(j) + T(stage_c(st))) / T(K);
            rhs_eval<T, TP, EMIT, false, true>(ax.iv, sc, mc, lane, tau, ax.coef[r & 3]);
            __syncthreads();
            done += 2;
        }
        for (; done < nsteps; ++done) __syncthreads();
        return;
    }
    // ---------------- reverse wave ----------------
    T xbar[2], xprev[2], xsum[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        xbar[q] = r < NXT ? a.seed[r * ldi + k] : T(0);
        xprev[q] = T(0);
        xsum[q] = T(0);
    }
    T sacc = T(0), muacc = T(0), macc = T(0);
    T uacc[3][2] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    for (int t = 0; t < nsteps; ++t) {
        if (t >= 3) {
            const int r = t - 3, u = r / S4, pp = r % S4;
            const int g = nseg - 1 - u;
            const int jj = Cs - 1 - (pp >> 2), st = 3 - (pp & 3), j = g * Cs + jj;
            const T tau = (T(j) + T(stage_c(st))) / T(K);
            reverse_stage<T, TP, false>(ax, ax.se[r & 3], ax.coef[r & 3], mc, lane, st, tau,
                                        xbar, xprev, xsum, sacc, uacc, muacc, macc);
            if (st == 0) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    xbar[q] += xsum[q];
                    xsum[q] = T(0);
                    xprev[q] = T(0);
                }
            }
        }
        __syncthreads();
    }
    adjoint_outputs<T, TP>(ax, a, k, lane, xbar, sacc, uacc, muacc, macc);
}

template <class T, class TP>
__global__ void __launch_bounds__(256)
    k_adjoint4(AdjArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ AdjShared<T, TP, 4> ax;
    adjoint_item4<T, TP>(ax, a, mc, xcd_slot(blockIdx.x, gridDim.x));
}

template <class T, class TP>
__global__ void __launch_bounds__(256)
    k_adjoint4_batch(BatchArgs<AdjArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ AdjShared<T, TP, 4> ax;
    const int2 it = b.items[xcd_slot(blockIdx.x, gridDim.x)];
    const AdjArgs<T> a = b.descs[it.x];
    adjoint_item4<T, TP>(ax, a, mc, it.y);
}

template <class T, class TP>
__global__ void __launch_bounds__(192)
    k_adjoint3_batch(BatchArgs<AdjArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ AdjShared<T, TP> ax;
    const int2 it = b.items[xcd_slot(blockIdx.x, gridDim.x)];
    const AdjArgs<T> a = b.descs[it.x];
    adjoint_item3<T, TP>(ax, a, mc, it.y);
}

template <class T, class TP>
__global__ void __launch_bounds__(128)
    k_adjoint(AdjArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ AdjShared<T, TP> ax;
    adjoint_item<T, TP, 2>(ax, a, mc, xcd_slot(blockIdx.x, gridDim.x));
}

template <class T, class TP, int NW>
__global__ void __launch_bounds__(64 * NW)
    k_adjoint_batch(BatchArgs<AdjArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ AdjShared<T, TP> ax;
    const int2 it = b.items[xcd_slot(blockIdx.x, gridDim.x)];
    const AdjArgs<T> a = b.descs[it.x];
    adjoint_item<T, TP, NW>(ax, a, mc, it.y);
}

// gU, gX_N and gp from the per-interval partials, in a fixed order.
template <class T>
__device__ __forceinline__ void adjoint_reduce_part(const T* ws_uk, const T* ws_uk1,
                                                    const T* ws_p, T* gU, T* gX, T* gp, int N,
                                                    int m, int nxt, int np, int64_t ldn,
                                                    int64_t t) {
    const int64_t nu = (int64_t)m * (N + 1);
    if (t < nu) {
        const int c = (int)(t / (N + 1)), k = (int)(t % (N + 1));
        const T left = k < N ? ws_uk[(int64_t)c * N + k] : T(0);
        const T right = k > 0 ? ws_uk1[(int64_t)c * N + k - 1] : T(0);
        gU[(int64_t)c * ldn + k] = left + right;
    } else if (t < nu + nxt) {
        gX[(t - nu) * ldn + N] = T(0);
    } else if (t < nu + nxt + np) {
        // index order (bitwise reproducible); unrolled so that the loads of
        // eight partials are in flight together instead of one at a time
        const int c = (int)(t - nu - nxt);
        const T* w = ws_p + (int64_t)c * N;
        T acc = T(0);
#pragma unroll 8
        for (int k = 0; k < N; ++k) acc += w[k];
        gp[c] = acc;
    }
}

// One workgroup per trajectory of a batch.
__global__ void __launch_bounds__(256) k_adjoint_reduce_batch(const RedDesc* rd) {
    const RedDesc r = rd[blockIdx.x];
    const int64_t work = (int64_t)r.m * (r.N + 1) + r.nxt + r.np;
    for (int64_t t = threadIdx.x; t < work; t += blockDim.x)
        adjoint_reduce_part<double>(r.ws_uk, r.ws_uk1, r.ws_p, r.gU, r.gX, r.gp, r.N, r.m, r.nxt,
                                    r.np, r.ldn, t);
}

template <class T>
__global__ void __launch_bounds__(256)
    k_adjoint_reduce(const T* ws_uk, const T* ws_uk1, const T* ws_p, T* gU, T* gX, T* gp, int N,
                     int m, int nxt, int np, int64_t ldn) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    adjoint_reduce_part<T>(ws_uk, ws_uk1, ws_p, gU, gX, gp, N, m, nxt, np, ldn, t);
}

static size_t ws_elems(const cis_model* m, int N) { return (size_t)(2 * m->m + m->np) * N; }

template <int L, int D>
static cis_status launch_adjoint(const cis_model* m, const cis_shape* sh, const void* X,
                                 const void* U, const void* s, const void* prm, const void* ckpt,
                                 int C, const void* seed, void* gX, void* gU, void* gs, void* gp,
                                 void* ws, hipStream_t stream) {
    using TP = Topo<L, D>;
    using T = double;
    auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
    AdjArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.f.X = (const T*)X;
    a.f.U = (const T*)U;
    a.f.s = (const T*)s;
    a.f.prm = (const T*)prm;
    a.f.ckpt = (T*)ckpt;
    a.f.ldn = sh->ld_node;
    a.f.ldi = sh->ld_int;
    a.f.N = sh->N;
    a.f.K = sh->substeps;
    a.f.C = C;
    a.seed = (const T*)seed;
    a.gX = (T*)gX;
    a.gs = (T*)gs;
    T* w = (T*)ws;
    const int N = sh->N;
    a.ws_uk = w;
    a.ws_uk1 = w + (size_t)m->m * N;
    a.ws_p = w + (size_t)2 * m->m * N;
    void* args[] = {&a, &mc};
    const bool four = C <= CHUNK;   // one chunk per checkpoint segment
    hipError_t e = hipLaunchKernel(four ? (const void*)&k_adjoint4<T, TP>
                                        : (const void*)&k_adjoint<T, TP>,
                                   dim3(N), dim3(four ? 256 : 128), args, 0,
                                   stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_adjoint launch: %s", hipGetErrorString(e));
    const int64_t work = (int64_t)m->m * (N + 1) + m->nx + m->np;
    const int blocks = (int)((work + 255) / 256);
    const T* wuk = a.ws_uk;
    const T* wuk1 = a.ws_uk1;
    const T* wp = a.ws_p;
    T* gUp = (T*)gU;
    T* gXp = (T*)gX;
    T* gpp = (T*)gp;
    int mm = m->m, nxt = m->nx, np = m->np;
    int64_t ldn = sh->ld_node;
    void* rargs[] = {&wuk, &wuk1, &wp, &gUp, &gXp, &gpp, (void*)&N, &mm, &nxt, &np, &ldn};
    e = hipLaunchKernel((const void*)&k_adjoint_reduce<T>, dim3(blocks), dim3(256), rargs, 0,
                        stream);
    if (e != hipSuccess)
        return fail(CIS_ERR_HIP, "k_adjoint_reduce launch: %s", hipGetErrorString(e));
    return CIS_OK;
}

template <int L, int D>
static cis_status prep_adj_t(const cis_model* m, const BatchGroupDev& g, int max_ckpt_every,
                             int waves, KLaunch* out) {
    using TP = Topo<L, D>;
    BatchArgs<AdjArgs<double>> b;
    b.descs = (const AdjArgs<double>*)g.adesc;
    b.items = g.items;
    b.n_items = g.n_items;
    b.cursor = g.cursor;
    out->arg(b);
    out->arg(make_const<TP::NB, TP::NJ, TP::NC>(m));
    if (waves >= 3 && max_ckpt_every > CHUNK) waves = 2;
    out->func = waves == 4   ? (const void*)&k_adjoint4_batch<double, TP>
                : waves == 3 ? (const void*)&k_adjoint3_batch<double, TP>
                : waves == 2 ? (const void*)&k_adjoint_batch<double, TP, 2>
                             : (const void*)&k_adjoint_batch<double, TP, 1>;
    out->grid = dim3(g.n_items);
    out->block = dim3(64 * waves);
    return out->ok() ? CIS_OK : fail(CIS_ERR_DIM, "prep_adjoint_batch: launch record refused");
}

cis_status prep_adjoint_batch(const cis_model* m, const BatchGroupDev& g, int max_ckpt_every,
                              int waves, KLaunch* out) {
#define CIS_PREP_ADJ(LL, DD) \
    if (m->L == LL && m->D == DD) return prep_adj_t<LL, DD>(m, g, max_ckpt_every, waves, out);
    CIS_TOPOLOGIES(CIS_PREP_ADJ)
#undef CIS_PREP_ADJ
    return fail(CIS_ERR_UNSUPPORTED, "prep_adjoint_batch: topology has no compiled kernel");
}

cis_status prep_adjoint_reduce_batch(const void* rdesc, int n_traj, KLaunch* out) {
    out->arg((const RedDesc*)rdesc);
    out->func = (const void*)&k_adjoint_reduce_batch;
    out->grid = dim3(n_traj);
    out->block = dim3(256);
    return out->ok() ? CIS_OK : fail(CIS_ERR_DIM, "prep_adjoint_reduce_batch: launch record refused");
}

// Workspace of the allocation-free reverse sweep: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never passes the array's name to a kernel: its device address is
// looked up once per device, with that device current, and kept here.
constexpr size_t NOALLOC_DOUBLES = (size_t)1 << 20;   // 8 MiB per GPU
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static double* scratch_dev[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
static cis_status scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(CIS_ERR_HIP, "cis_discretize_adjoint_noalloc: hipGetDevice: %s",
                    hipGetErrorString(e));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_adjoint_noalloc: device %d beyond %d",
                    dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(CIS_ERR_HIP, "cis_discretize_adjoint_noalloc: hipGetSymbolAddress: %s",
                        hipGetErrorString(e));
        scratch_dev[dev] = (double*)ptr;
    }
    *out = scratch_dev[dev];
    return CIS_OK;
}

}  // namespace cis

using namespace cis;

extern "C" cis_status cis_adjoint_workspace_size(const cis_model* m, const cis_shape* sh,
                                                 size_t* bytes) {
    if (!m || !sh || !bytes) return fail(CIS_ERR_NULL, "cis_adjoint_workspace_size: null argument");
    if (sh->N < 1) return fail(CIS_ERR_DIM, "cis_adjoint_workspace_size: N=%d must be >= 1", sh->N);
    *bytes = ws_elems(m, sh->N) * sizeof(double);
    return CIS_OK;
}

static cis_status discretize_adjoint_impl(const cis_model* model, const cis_shape* shape,
                                          const void* X, const void* U, const void* s,
                                          const void* params, const void* ckpt,
                                          int32_t ckpt_every, const void* seed, void* gX,
                                          void* gU, void* gs, void* gparams, void* ws,
                                          size_t ws_bytes, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (shape->dtype != CIS_F64)
        return fail(CIS_ERR_DTYPE, "cis_discretize_adjoint: only CIS_F64 is offered");
    if (!ckpt || !seed || !gX || !gs || !gparams || (model->m > 0 && !gU))
        return fail(CIS_ERR_NULL, "cis_discretize_adjoint: ckpt, seed, gX, gs, gparams (and gU when m > 0) are required");
    if (ckpt_every < 1 || shape->substeps % ckpt_every != 0)
        return fail(CIS_ERR_DIM, "cis_discretize_adjoint: ckpt_every=%d must divide K=%d",
                    ckpt_every, shape->substeps);
    const size_t need = ws_elems(model, shape->N) * sizeof(double);
    if (!ws || ws_bytes < need)
        return fail(CIS_ERR_WORKSPACE, "cis_discretize_adjoint: workspace of %zu bytes needed",
                    need);
    const size_t es = sizeof(double);
    if (!aligned(ckpt, es) || !aligned(seed, es) || !aligned(gX, es) || !aligned(gU, es) ||
        !aligned(gs, es) || !aligned(gparams, es) || !aligned(ws, es))
        return fail(CIS_ERR_LAYOUT, "cis_discretize_adjoint: pointer not aligned to 8 bytes");
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_ADJ(LL, DD)                                                               \
    if (model->L == LL && model->D == DD)                                                     \
        return launch_adjoint<LL, DD>(model, shape, X, U, s, params, ckpt, ckpt_every, seed,   \
                                      gX, gU, gs, gparams, ws, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_ADJ)
#undef CIS_DISPATCH_ADJ
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_adjoint: topology has no compiled kernel");
}

extern "C" cis_status cis_discretize_adjoint(const cis_model* model, const cis_shape* shape,
                                             const void* X, const void* U, const void* s,
                                             const void* params, const void* ckpt,
                                             int32_t ckpt_every, const void* seed, void* gX,
                                             void* gU, void* gs, void* gparams, void* ws,
                                             size_t ws_bytes, void* stream) {
    const cis_status st = discretize_adjoint_impl(model, shape, X, U, s, params, ckpt,
                                                  ckpt_every, seed, gX, gU, gs, gparams, ws,
                                                  ws_bytes, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    const int64_t N = shape->N, ln = shape->ld_node, li = shape->ld_int;
    const DebugArr arr[] = {
        {"X", X, model->nx, N + 1, ln, false},   {"U", U, model->m, N + 1, ln, false},
        {"s", s, 1, N, N, false},                {"params", params, 1, model->np, model->np, false},
        {"seed", seed, model->nx, N, li, false}, {"gX", gX, model->nx, N + 1, ln, true},
        {"gU", gU, model->m, N + 1, ln, true},   {"gs", gs, 1, N, N, true},
        {"gparams", gparams, 1, model->np, model->np, true},
    };
    return debug_scan("cis_discretize_adjoint", CIS_F64, stream, arr,
                      (int)(sizeof(arr) / sizeof(arr[0])));
}

extern "C" cis_status cis_discretize_adjoint_noalloc(const cis_model* model,
                                                     const cis_shape* shape, const void* X,
                                                     const void* U, const void* s,
                                                     const void* params, const void* ckpt,
                                                     int32_t ckpt_every, const void* seed,
                                                     void* gX, void* gU, void* gs,
                                                     void* gparams, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    const size_t need = ws_elems(model, shape->N);
    if (need > NOALLOC_DOUBLES)
        return fail(CIS_ERR_WORKSPACE,
                    "cis_discretize_adjoint_noalloc: needs %zu bytes of workspace, more than "
                    "the %zu bytes it holds ((2 m + P) N doubles; use cis_discretize_adjoint)",
                    need * sizeof(double), NOALLOC_DOUBLES * sizeof(double));
    double* ws = nullptr;
    st = scratch_address(&ws);
    if (st != CIS_OK) return st;
    // same validation and kernels as cis_discretize_adjoint, with the device
    // array as the workspace
    return discretize_adjoint_impl(model, shape, X, U, s, params, ckpt, ckpt_every, seed, gX,
                                   gU, gs, gparams, ws, NOALLOC_DOUBLES * sizeof(double), stream);
}
