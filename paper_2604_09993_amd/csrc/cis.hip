// MI355X (gfx950) kernels and C ABI for the CI-SCvx interval
// linearize-and-discretize step (arxiv 2604.09993, Sec. IV-B and Sec. VI).
//
// Kernels (one workgroup per interval):
//   k_discretize : nominal RK4 + variational equations -> A, B-, B+, S, d, F~
//   k_defects    : nominal RK4 only -> d, F~ and substep checkpoints
// The adjoint kernels live in cis_adjoint.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <type_traits>
#include <utility>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cis.h"
#include "cis_model.hpp"
#include "cis_body.hpp"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"

namespace cis {

// ---------------------------------------------------------------------------
// Tangent lanes.  Column c of Z = [Phi_x | B- | B+ | S] is spread over G
// lanes, one per leg: each lane holds the torso rows (replicated, computed
// identically in the G lanes) and the rows of its own leg.  The only values a
// lane needs from the other legs are the angle and rate of their first links
// (hip stiffness and damping on the torso), read with DPP quad permutes.
// ---------------------------------------------------------------------------
template <class T, class TP>
struct TLane {
    T zb[6 * TP::LB], za[6 * TP::LB], zs[6 * TP::LB];   // local rows: q(lb,k), v(lb,k)
    T ycc, yct;                                          // own contact row, violation partial
};

// value of `v` in lane (lane & ~(G-1)) + SRC of the same quad
template <int G, int SRC>
__device__ __forceinline__ int dpp_from(int v) {
    constexpr int p0 = G == 4 ? SRC : SRC, p1 = p0;
    constexpr int p2 = G == 4 ? SRC : 2 + SRC, p3 = p2;
    constexpr int ctrl = p0 | (p1 << 2) | (p2 << 4) | (p3 << 6);
    return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, false);
}
template <int G, int SRC>
__device__ __forceinline__ double dpp_from(double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    const int2 r = make_int2(dpp_from<G, SRC>(w.x), dpp_from<G, SRC>(w.y));
    return __builtin_bit_cast(double, r);
}
template <int G, int SRC>
__device__ __forceinline__ float dpp_from(float v) {
    return __builtin_bit_cast(float, dpp_from<G, SRC>(__builtin_bit_cast(int, v)));
}
// value of the leg-SRC lane of this column (the lane's own value when G == 1)
template <int G, int SRC, class T>
__device__ __forceinline__ T from_leg(T v) {
    if constexpr (G == 1) return v;
    else return dpp_from<G, SRC>(v);
}
// sum of v over the G lanes of a column (same order in every lane)
template <int G, class T>
__device__ __forceinline__ T column_sum(T v) {
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G == 2) {
        return dpp_from<2, 0>(v) + dpp_from<2, 1>(v);
    } else {
        return (dpp_from<4, 0>(v) + dpp_from<4, 1>(v)) + (dpp_from<4, 2>(v) + dpp_from<4, 3>(v));
    }
}

template <class T, class TP, int ST, bool HF>
__device__ __forceinline__ void tangent_stage(const Interval<T, TP>& iv, TLane<T, TP>& z,
                                              const T* __restrict__ cf, T tau, int leg, T wbm,
                                              T wbp, T fsel, T fct, int ctrl) {
    constexpr int LB = TP::LB, D = TP::D, L = TP::L, G = TP::G, NQ = TP::NQ, NX = TP::NX;
    constexpr int NC = TP::NC, M = TP::M;
    using C = Coef<TP>;
    const T s = iv.s, h = iv.h;
    // global body of local body lb (0 = torso, 1..D = own leg links)
    auto gb = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
#define ZQ(lb, k) z.zs[3 * (lb) + (k)]
#define ZV(lb, k) z.zs[3 * LB + 3 * (lb) + (k)]
    T kv[3 * LB];
#pragma unroll
    for (int lb = 0; lb < LB; ++lb) {
        kv[3 * lb] = T(0);
        kv[3 * lb + 1] = T(0);
        kv[3 * lb + 2] = cf[C::CTH + gb(lb)] * ZQ(lb, 2);
    }
    T kct = T(0), kcc = T(0);
    // Scheduling fences: the stage is limited by LDS latency under register
    // pressure, and where the compiler may move loads across sections was
    // chosen by measurement per type (FP64: only before the RK combination;
    // FP32: also here and between the joints).
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
    if constexpr (D >= 1) {
        // hip joints: torso-side stiffness and damping of every leg
        const T th1 = ZQ(1, 2), w1 = ZV(1, 2);
        const T th0 = ZQ(0, 2), w0 = ZV(0, 2);
        [&]<int... Ls>(std::integer_sequence<int, Ls...>) {
            ((kv[2] += iv.kc[Ls * D][0] * (from_leg<G, Ls>(th1) - th0) +
                       iv.kc[Ls * D][1] * (from_leg<G, Ls>(w1) - w0)),
             ...);
        }(std::make_integer_sequence<int, L>{});
#pragma unroll
        for (int lb = 1; lb <= D; ++lb) {
            const int j = leg * D + lb - 1;
            const T dth = ZQ(lb, 2) - ZQ(lb - 1, 2);
            const T dom = ZV(lb, 2) - ZV(lb - 1, 2);
            if (lb >= 2) kv[3 * (lb - 1) + 2] += iv.kc[j][0] * dth + iv.kc[j][1] * dom;
            kv[3 * lb + 2] -= iv.kc[j][2] * dth + iv.kc[j][3] * dom;
            const T* jh = cf + C::JH + 4 * j;
            kct += jh[0] * (ZQ(lb - 1, 0) - ZQ(lb, 0)) + jh[1] * (ZQ(lb - 1, 1) - ZQ(lb, 1)) +
                   jh[2] * ZQ(lb - 1, 2) + jh[3] * ZQ(lb, 2);
            if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
        }
    }
    if constexpr (L >= 1) {
        constexpr int lb = D;   // the contact sits on the last local body
        const T* ct = cf + C::CT + C::NCT * leg;
        const T dPx = ZQ(lb, 0) - ct[C_AY] * ZQ(lb, 2);
        const T dPy = ZQ(lb, 1) + ct[C_AX] * ZQ(lb, 2);
        kv[3 * lb] += ct[C_FXP] * dPx;
        kv[3 * lb + 1] += ct[C_FYP] * dPx;
        kv[3 * lb + 2] += ct[C_TP] * dPx;
        kcc = ct[C_EPX] * dPx + ct[C_EPY] * dPy + ct[C_EXD] * ZV(lb, 0) + ct[C_EYD] * ZV(lb, 1) +
              ct[C_EOM] * ZV(lb, 2) + ct[C_ETH] * ZQ(lb, 2);
        kct += ct[C_ZPX] * dPx + ct[C_ZPY] * dPy;
    }
    // FOH forcing of B-/B+ columns, s (J_u w(tau) + J_ubar / 2), and F~
    // forcing of the dilation column, without branches (the weights are zero in
    // the other columns) so that the loads issue with the stage's other loads
    if constexpr (M > 0) {
        const T wB = wbm * (T(1) - tau) + wbp * tau;
        const T wG = wbm + wbp;
#pragma unroll
        for (int lb = 0; lb < LB; ++lb)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                kv[3 * lb + k] += wB * cf[C::GV + (3 * gb(lb) + k) * M + ctrl];
        if constexpr (L >= 1) kcc += wG * cf[C::GC + leg * M + ctrl];
    }
    if constexpr (HF) {
#pragma unroll
        for (int lb = 0; lb < LB; ++lb)
#pragma unroll
            for (int k = 0; k < 3; ++k) kv[3 * lb + k] += fsel * cf[C::F + NQ + 3 * gb(lb) + k];
        if constexpr (L >= 1) kcc += fsel * cf[C::F + NX + leg];
        // violation row: per-body parts of the own bodies (torso on leg 0 only)
        T vp = fct * cf[C::CTP];
#pragma unroll
        for (int lb = 1; lb < LB; ++lb) vp += fsel * cf[C::CTP + gb(lb)];
        kct += vp;
    }
    __builtin_amdgcn_sched_barrier(0);
    // classical RK4 combination (stage ST known at compile time)
    constexpr int WK = (ST == 0 || ST == 3) ? 1 : 2;
    const T an = (ST == 2) ? h : T(0.5) * h;
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int r = 3 * lb + k;
            T kq = s * z.zs[3 * LB + r];
            if constexpr (HF) kq += fsel * cf[C::F + 3 * gb(lb) + k];
            if (ST == 0) z.za[r] = kq;
            else z.za[r] += T(WK) * kq;
            if (ST < 3) z.zs[r] = z.zb[r] + an * kq;
        }
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) {
        const T kk = kv[r];
        if (ST == 0) z.za[3 * LB + r] = kk;
        else z.za[3 * LB + r] += T(WK) * kk;
        if (ST < 3) z.zs[3 * LB + r] = z.zb[3 * LB + r] + an * kk;
    }
    const T h6 = iv.h6;
    z.ycc += (h6 * T(WK)) * kcc;
    z.yct += (h6 * T(WK)) * kct;
    if (ST == 3) {
#pragma unroll
        for (int r = 0; r < 6 * LB; ++r) {
            z.zb[r] += h6 * z.za[r];
            z.zs[r] = z.zb[r];
        }
    }
#undef ZQ
#undef ZV
}

// ---------------------------------------------------------------------------
// K2: discretize.  One workgroup per (interval, column group), three wave roles
// separated by one workgroup barrier per pipeline step:
//   state wave        : evaluates the accelerations at stage t and forms the
//                       input of stage t+1 (the only serial chain);
//   coefficient waves : full right-hand side and Jacobian nonzeros of stage
//                       t-1 (rotations reused from the state wave) and the
//                       integral rows.  With two such waves they take alternate
//                       stages and each stage spans steps t-1 and t-2;
//   tangent waves     : apply stage t-LAG to their columns.
// ---------------------------------------------------------------------------
// Workgroup layouts of the discretize kernel.  Latency (few intervals): two
// coefficient waves; FP64 one tangent wave per workgroup (512 registers per
// lane, one wave per SIMD), FP32 up to five (two waves per SIMD).  Narrow
// (FP64, as many workgroups as CUs): one coefficient wave and two tangent
// waves, still one wave per SIMD.  Throughput (large trajectories and
// batches): up to six tangent waves per workgroup, so the state and
// coefficient work is repeated over fewer column groups; a workgroup of more
// than four waves holds every wave to 256 registers.
template <class T, int L, int D>
using LatencyTopo = Topo<L, D, sizeof(T) == 8 ? 1 : 5, 2>;
// the latency layout with the S column on leg lanes (one column group fewer)
template <class T, int L, int D>
using LatencyTopoS = Topo<L, D, sizeof(T) == 8 ? 1 : 5, 2, false>;
template <class T, int L, int D>
using NarrowTopo = Topo<L, D, sizeof(T) == 8 ? 2 : 6, 1>;
template <class T, int L, int D>
using ThroughputTopo = Topo<L, D, 6, 1>;

template <class T, class TP>
struct DiscShared {
    Interval<T, TP> iv;
    T xring[4][TP::NX];        // stage inputs from the state wave
    T csring[4][TP::NB][2];    // their rotations
    T fring[4][3 * TP::NB];    // their accelerations
    T yshare[TP::NY];          // integral-row partial sums of the second coefficient wave
    T coef[TP::NCOEF][Coef<TP>::SIZE];
};

// Interval k, column group grp, by the whole workgroup.
template <class T, class TP>
__device__ __forceinline__ void discretize_item(DiscShared<T, TP>& sh, const FwdArgs<T>& a,
                                                const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                                const int k, const int grp) {
    constexpr int NB = TP::NB, NX = TP::NX, NXT = TP::NXT, M = TP::M, NY = TP::NY;
    constexpr int NQ = TP::NQ, NC = TP::NC, LB = TP::LB, G = TP::G, D = TP::D, L = TP::L;
    constexpr int NCW = TP::NCW, NCOEF = TP::NCOEF, LAG = TP::LAG;
    using C = Coef<TP>;
    static_assert(D > 0 || L <= 1, "several contacts on the torso are not laid out");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = TP::NTHREADS;
    // substep block of this item (whole interval when a.B <= 1)
    const bool blocked = a.B > 1;
    const int kin = blocked ? k % a.N : k;            // interval of the inputs
    const int Kb = blocked ? a.K / a.B : a.K;         // substeps of this item
    const int j0 = blocked ? (k / a.N) * Kb : 0;      // first substep
    load_interval<T, TP>(sh.iv, a, mc, kin, tid, nth);
    if (blocked) {
        // block start: x from the checkpoint slot, integral states from zero
        // (they feed back into nothing; only their sensitivities are kept)
        const T* xi = a.xinit + (int64_t)(k / a.N) * NX * a.ld_blk + kin;
        for (int e = tid; e < NXT; e += nth) sh.iv.x0[e] = e < NX ? xi[e * a.ld_blk] : T(0);
    }
    for (int e = tid; e < NCOEF * C::SIZE; e += nth) (&sh.coef[0][0])[e] = T(0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NCOEF; ++q) coef_constants<T, TP>(sh.iv, sh.coef[q], tid, nth);
    const int nst = 4 * Kb;
    const int nsteps = nst + LAG;
    const int64_t ldi = a.ldi;
    __syncthreads();

    // Each role runs its own loop with the same number of workgroup barriers
    // (nsteps), so the registers of one role are not live in the others.
    if (wave == TP::NTW) {
        // ---------------- state wave: stage t at step t ----------------
        const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
        BodyRK<T> bs;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            bs.xb[kk] = sh.iv.x0[3 * c.b + kk];
            bs.xb[3 + kk] = sh.iv.x0[NQ + 3 * c.b + kk];
        }
#pragma unroll
        for (int kk = 0; kk < 6; ++kk) {
            bs.xs[kk] = bs.xb[kk];
            bs.xa[kk] = T(0);
        }
        // stage t = 4 j + ST at step t, the four RK stages unrolled
        const T Kt = T(a.K);
        for (int j = 0; j < Kb; ++j) {
            const T jt = T(j0 + j);
            state_stage<T, TP, 0>(sh.iv, mc, c, bs, jt / Kt, sh.xring[1], sh.csring[0],
                                  sh.fring[0], lane);
            __syncthreads();
            state_stage<T, TP, 1>(sh.iv, mc, c, bs, (jt + T(0.5)) / Kt, sh.xring[2], sh.csring[1],
                                  sh.fring[1], lane);
            __syncthreads();
            state_stage<T, TP, 2>(sh.iv, mc, c, bs, (jt + T(0.5)) / Kt, sh.xring[3], sh.csring[2],
                                  sh.fring[2], lane);
            __syncthreads();
            state_stage<T, TP, 3>(sh.iv, mc, c, bs, (jt + T(1)) / Kt, sh.xring[0], sh.csring[3],
                                  sh.fring[3], lane);
            __syncthreads();
        }
        for (int t = nst; t < nsteps; ++t) __syncthreads();
        if constexpr (NCW > 1) __syncthreads();   // the integral-row hand-over step
        if (grp == 0 && lane < NB && !blocked) {
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) {
                const int r = kk < 3 ? 3 * c.b + kk : NQ + 3 * c.b + kk - 3;
                if (a.xprop) a.xprop[r * ldi + k] = bs.xb[kk];
                a.defect[r * ldi + k] = bs.xb[kk] - sh.iv.xk1[r];
            }
        }
    } else if (wave > TP::NTW) {
        // ---- coefficient waves: stage tc over steps tc+1 .. tc+NCW; integral rows ----
        const int w = wave - TP::NTW - 1;
        const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
        // integral rows: the contact's cc row on its lane, the violation row on lane 0
        const int ycc_row = NX + c.i;
        const bool own0 = w == 0;
        T ycb = (c.contact && own0) ? sh.iv.x0[ycc_row] : T(0), yca = T(0);
        T ytb = (lane == 0 && own0) ? sh.iv.x0[NX + NC] : T(0), yta = T(0);
        const T s = sh.iv.s;
        // leading steps before the first stage of this wave
        for (int t = 0; t < 1 + w; ++t) __syncthreads();
        for (int tc = w; tc < nst; tc += NCW) {
            const int st = tc & 3;
            const T tau = (T(j0 + (tc >> 2)) + T(stage_c(st))) / T(a.K);
            T ycc = T(0), yct = T(0);
            coef_stage<T, TP, (NCW > 1)>(sh.iv, mc, c, tc == 0 ? sh.iv.x0 : sh.xring[tc & 3],
                                         sh.csring[tc & 3], sh.fring[tc & 3], tau,
                                         sh.coef[tc & (NCOEF - 1)], ycc, yct, lane);
            const T wk = (st == 0 || st == 3) ? T(1) : T(2);
            if (st == w) {   // first stage of the substep handled by this wave
                yca = wk * s * ycc;
                yta = wk * s * yct;
            } else {
                yca += wk * s * ycc;
                yta += wk * s * yct;
            }
            if (st + NCW > 3) {   // last stage of the substep handled by this wave
                ycb += sh.iv.h6 * yca;
                ytb += sh.iv.h6 * yta;
            }
            __syncthreads();
        }
        // trailing steps: the wave's last stage ends at step nst - NCW + w + NCW
        for (int t = nst + w + 1; t < nsteps; ++t) __syncthreads();
        // violation row: the body lanes' parts, summed in lane order
        {
            T acc = T(0);
#pragma unroll
            for (int e = 0; e < NB; ++e) acc += lane_value(ytb, e);
            ytb = acc;
        }
        if constexpr (NCW > 1) {
            if (w == 1) {
                if (c.contact) sh.yshare[c.i] = ycb;
                if (lane == 0) sh.yshare[NC] = ytb;
            }
            __syncthreads();
            if (w == 0) {
                if (c.contact) ycb += sh.yshare[c.i];
                if (lane == 0) ytb += sh.yshare[NC];
            }
        }
        if (grp == 0 && w == 0) {
            if (c.contact && !blocked) {
                if (a.xprop) a.xprop[ycc_row * ldi + k] = ycb;
                a.defect[ycc_row * ldi + k] = ycb - sh.iv.xk1[ycc_row];
            }
            if (lane == 0 && !blocked) {
                if (a.xprop) a.xprop[(NX + NC) * ldi + k] = ytb;
                a.defect[(NX + NC) * ldi + k] = ytb - sh.iv.xk1[NX + NC];
            }
            // A[:, n:] = [0; I]: the integral states feed back into nothing
            for (int e = lane; e < NXT * NY; e += 64) {
                const int r = e / NY, cc = NX + e % NY;
                a.A[((int64_t)r * NXT + cc) * ldi + k] = (r == cc) ? T(1) : T(0);
            }
        }
    } else {
        if constexpr (TP::SEP_S) {
            if (grp == TP::NGRPT) {
                // ---------- the S column on body lanes (first wave of the group) ----------
                if (wave != 0) {
                    for (int t = 0; t < LAG + 4 * Kb + (NCW > 1 ? 1 : 0); ++t) __syncthreads();
                    return;
                }
                const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
                SLane<T, TP> z;
#pragma unroll
                for (int r = 0; r < 6; ++r) z.zs[r] = z.zb[r] = z.za[r] = T(0);
#pragma unroll
                for (int l = 0; l < SLane<T, TP>::NCL; ++l) z.ycc[l] = T(0);
                z.yct = T(0);
#pragma unroll
                for (int t = 0; t < LAG; ++t) __syncthreads();
                for (int j = 0; j < Kb; ++j) {
                    s_stage<T, TP, 0>(sh.iv, c, z, sh.coef[0], lane);
                    __syncthreads();
                    s_stage<T, TP, 1>(sh.iv, c, z, sh.coef[1], lane);
                    __syncthreads();
                    s_stage<T, TP, 2>(sh.iv, c, z, sh.coef[2 % NCOEF], lane);
                    __syncthreads();
                    s_stage<T, TP, 3>(sh.iv, c, z, sh.coef[3 % NCOEF], lane);
                    __syncthreads();
                }
                if constexpr (NCW > 1) __syncthreads();   // the integral-row hand-over step
                T yct = T(0);
#pragma unroll
                for (int e = 0; e < NB; ++e) yct += lane_value(z.yct, e);
                if (lane < NB) {
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        a.S[(int64_t)(3 * c.b + kk) * ldi + k] = z.zb[kk];
                        a.S[(int64_t)(NQ + 3 * c.b + kk) * ldi + k] = z.zb[3 + kk];
                    }
                    if constexpr (L >= 1) {
#pragma unroll
                        for (int l = 0; l < SLane<T, TP>::NCL; ++l) {
                            const bool on = D >= 1 ? c.contact : (lane == 0);
                            const int i = D >= 1 ? c.i : l;
                            if (on) a.S[(int64_t)(NX + i) * ldi + k] = z.ycc[l];
                        }
                    }
                    if (lane == 0) a.S[(int64_t)(NX + NC) * ldi + k] = yct;
                }
                return;
            }
        }
        // ---------------- tangent waves: stage t-LAG at step t ----------------
        const int col = grp * TP::CPG + (wave * 64 + lane) / G;
        const int leg = G == 1 ? 0 : (lane & (G - 1));
        T wbm = T(0), wbp = T(0), fsel = T(0);
        int ctrl = 0;
        if (col >= NX && col < NX + M) { wbm = T(1); ctrl = col - NX; }
        else if (col >= NX + M && col < NX + 2 * M) { wbp = T(1); ctrl = col - NX - M; }
        else if (col == NX + 2 * M) fsel = T(1);
        const T fct = leg == 0 ? fsel : T(0);
        auto gbody = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
        TLane<T, TP> z;
#pragma unroll
        for (int lb = 0; lb < LB; ++lb)
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const int gq = 3 * gbody(lb) + kk;
                z.zb[3 * lb + kk] = (gq == col) ? T(1) : T(0);
                z.zb[3 * LB + 3 * lb + kk] = (NQ + gq == col) ? T(1) : T(0);
            }
#pragma unroll
        for (int r = 0; r < 6 * LB; ++r) {
            z.zs[r] = z.zb[r];
            z.za[r] = T(0);
        }
        z.ycc = T(0);
        z.yct = T(0);
        // steps 0 .. LAG-1: nothing to apply yet
#pragma unroll
        for (int t = 0; t < LAG; ++t) __syncthreads();
        // steps LAG .. nst+LAG-1 apply stages 0 .. nst-1, unrolled by the 4 RK stages
        const T Kt = T(a.K);
        for (int j = 0; j < Kb; ++j) {
            const T jt = T(j0 + j);
            const T tau0 = jt / Kt, tauh = (jt + T(0.5)) / Kt, tau1 = (jt + T(1)) / Kt;
            tangent_stage<T, TP, 0, !TP::SEP_S>(sh.iv, z, sh.coef[0], tau0, leg, wbm, wbp, fsel, fct, ctrl);
            __syncthreads();
            tangent_stage<T, TP, 1, !TP::SEP_S>(sh.iv, z, sh.coef[1], tauh, leg, wbm, wbp, fsel, fct, ctrl);
            __syncthreads();
            tangent_stage<T, TP, 2, !TP::SEP_S>(sh.iv, z, sh.coef[2 % NCOEF], tauh, leg, wbm, wbp, fsel, fct,
                                    ctrl);
            __syncthreads();
            tangent_stage<T, TP, 3, !TP::SEP_S>(sh.iv, z, sh.coef[3 % NCOEF], tau1, leg, wbm, wbp, fsel, fct,
                                    ctrl);
            __syncthreads();
        }
        if constexpr (NCW > 1) __syncthreads();   // the integral-row hand-over step
        const T yct = column_sum<G>(z.yct);
        if (col < TP::NCOLT) {
            T* out;
            int64_t cstride, c0;   // element (row, column) at out[(row * cstride + c0) * ldi + k]
            if (col < NX) { out = a.A; cstride = NXT; c0 = col; }
            else if (col < NX + M) { out = a.Bm; cstride = M; c0 = col - NX; }
            else if (col < NX + 2 * M) { out = a.Bp; cstride = M; c0 = col - NX - M; }
            else { out = a.S; cstride = 1; c0 = 0; }
#pragma unroll
            for (int lb = 0; lb < LB; ++lb) {
                if (lb == 0 && leg != 0) continue;
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    const int gq = 3 * gbody(lb) + kk;
                    out[((int64_t)gq * cstride + c0) * ldi + k] = z.zb[3 * lb + kk];
                    out[((int64_t)(NQ + gq) * cstride + c0) * ldi + k] = z.zb[3 * LB + 3 * lb + kk];
                }
            }
            if constexpr (L >= 1) out[((int64_t)(NX + leg) * cstride + c0) * ldi + k] = z.ycc;
            if (leg == 0) out[((int64_t)(NX + NC) * cstride + c0) * ldi + k] = yct;
        }
    }
}

template <class T, class TP>
__global__ void __launch_bounds__(TP::NTHREADS)
    k_discretize(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ DiscShared<T, TP> sh;
    discretize_item<T, TP>(sh, a, mc, xcd_slot(blockIdx.x, gridDim.x), blockIdx.y);
}

// K5: a batch of trajectories of one model.  PERSIST = false: one workgroup per
// work unit (dispatch order follows the cost-sorted list); PERSIST = true: a
// resident grid draws units from an atomic cursor until the list is empty.
// WAVES: the waves per SIMD the register allocation is held to (1: no cap;
// 2: at most 256 registers per lane, which lets a second workgroup share the
// compute unit and hide the other's latency, at the price of spills).
template <class T, class TP, bool PERSIST, int WAVES>
__global__ void __launch_bounds__(TP::NTHREADS) __attribute__((amdgpu_waves_per_eu(WAVES)))
    k_discretize_batch(BatchArgs<FwdArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ DiscShared<T, TP> sh;
    const int total = b.n_items * TP::NGRP;
    if constexpr (!PERSIST) {
        int item, grp;
        unit_item(xcd_slot(blockIdx.x, gridDim.x), b.n_items, TP::NGRP, item, grp);
        const int2 it = b.items[item];
        const FwdArgs<T> a = b.descs[it.x];
        discretize_item<T, TP>(sh, a, mc, it.y, grp);
    } else {
        __shared__ int slot;
        for (;;) {
            const int u = fetch_unit(b.cursor, &slot);
            if (u >= total) break;
            int item, grp;
            unit_item(u, b.n_items, TP::NGRP, item, grp);
            const int2 it = b.items[item];
            const FwdArgs<T> a = b.descs[it.x];
            discretize_item<T, TP>(sh, a, mc, it.y, grp);
        }
        retire_block(b.cursor);
    }
}

// ---------------------------------------------------------------------------
// K1: defects and checkpoints.  Two waves per interval: the state wave of the
// discretize kernel (body lanes, stage t at step t; x checkpoints every C
// substeps) and one wave forming the integral-row integrands of stage t-1
// from the same rings (no Jacobian).
// ---------------------------------------------------------------------------
template <class T, class TP>
struct DefShared {
    Interval<T, TP> iv;
    T xring[4][TP::NX];
    T csring[4][TP::NB][2];
    T fring[4][3 * TP::NB];
};

template <class T, class TP>
__device__ __forceinline__ void defects_item(DefShared<T, TP>& sh, const FwdArgs<T>& a,
                                             const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                             const int k) {
    constexpr int NB = TP::NB, NX = TP::NX, NQ = TP::NQ, NC = TP::NC;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_interval<T, TP>(sh.iv, a, mc, k, tid, 128);
    const int nst = 4 * a.K;
    const int nsteps = nst + 1;
    const int64_t ldi = a.ldi;
    const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
    if (wave == 0) {
        BodyRK<T> bs;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            bs.xb[kk] = sh.iv.x0[3 * c.b + kk];
            bs.xb[3 + kk] = sh.iv.x0[NQ + 3 * c.b + kk];
        }
#pragma unroll
        for (int kk = 0; kk < 6; ++kk) {
            bs.xs[kk] = bs.xb[kk];
            bs.xa[kk] = T(0);
        }
        const T Kt = T(a.K);
        for (int j = 0; j < a.K; ++j) {
            if (a.ckpt && (j % a.C) == 0 && lane < NB) {
                T* ck = a.ckpt + (int64_t)(j / a.C) * NX * ldi + k;
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    ck[(3 * c.b + kk) * ldi] = bs.xb[kk];
                    ck[(NQ + 3 * c.b + kk) * ldi] = bs.xb[3 + kk];
                }
            }
            const T jt = T(j);
            state_stage<T, TP, 0>(sh.iv, mc, c, bs, jt / Kt, sh.xring[1], sh.csring[0],
                                  sh.fring[0], lane);
            __syncthreads();
            state_stage<T, TP, 1>(sh.iv, mc, c, bs, (jt + T(0.5)) / Kt, sh.xring[2], sh.csring[1],
                                  sh.fring[1], lane);
            __syncthreads();
            state_stage<T, TP, 2>(sh.iv, mc, c, bs, (jt + T(0.5)) / Kt, sh.xring[3], sh.csring[2],
                                  sh.fring[2], lane);
            __syncthreads();
            state_stage<T, TP, 3>(sh.iv, mc, c, bs, (jt + T(1)) / Kt, sh.xring[0], sh.csring[3],
                                  sh.fring[3], lane);
            __syncthreads();
        }
        for (int t = nst; t < nsteps; ++t) __syncthreads();
        if (lane < NB) {
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) {
                const int r = kk < 3 ? 3 * c.b + kk : NQ + 3 * c.b + kk - 3;
                if (a.xprop) a.xprop[r * ldi + k] = bs.xb[kk];
                a.defect[r * ldi + k] = bs.xb[kk] - sh.iv.xk1[r];
            }
        }
    } else {
        const int ycc_row = NX + c.i;
        T ycb = c.contact ? sh.iv.x0[ycc_row] : T(0), yca = T(0);
        T ytb = lane == 0 ? sh.iv.x0[NX + NC] : T(0), yta = T(0);
        const T s = sh.iv.s;
        for (int t = 0; t < nsteps; ++t) {
            const int tc = t - 1;
            if (tc >= 0 && tc < nst) {
                const int st = tc & 3;
                const T tau = (T(tc >> 2) + T(stage_c(st))) / T(a.K);
                T ycc = T(0), yct = T(0);
                coef_stage<T, TP, false, false>(sh.iv, mc, c,
                                                tc == 0 ? sh.iv.x0 : sh.xring[tc & 3],
                                                sh.csring[tc & 3], sh.fring[tc & 3], tau,
                                                (T*)nullptr, ycc, yct, lane);
                const T wk = (st == 0 || st == 3) ? T(1) : T(2);
                if (st == 0) {
                    yca = s * ycc;
                    yta = s * yct;
                } else {
                    yca += wk * s * ycc;
                    yta += wk * s * yct;
                }
                if (st == 3) {
                    ycb += sh.iv.h6 * yca;
                    ytb += sh.iv.h6 * yta;
                }
            }
            __syncthreads();
        }
        {   // violation row: the body lanes' parts, summed in lane order
            T acc = T(0);
#pragma unroll
            for (int e = 0; e < NB; ++e) acc += lane_value(ytb, e);
            ytb = acc;
        }
        if (c.contact) {
            if (a.xprop) a.xprop[ycc_row * ldi + k] = ycb;
            a.defect[ycc_row * ldi + k] = ycb - sh.iv.xk1[ycc_row];
        }
        if (lane == 0) {
            if (a.xprop) a.xprop[(NX + NC) * ldi + k] = ytb;
            a.defect[(NX + NC) * ldi + k] = ytb - sh.iv.xk1[NX + NC];
        }
    }
}

template <class T, class TP>
__global__ void __launch_bounds__(128)
    k_defects(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ DefShared<T, TP> sh;
    defects_item<T, TP>(sh, a, mc, xcd_slot(blockIdx.x, gridDim.x));
}

template <class T, class TP>
__global__ void __launch_bounds__(128)
    k_defects_batch(BatchArgs<FwdArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ DefShared<T, TP> sh;
    const int2 it = b.items[xcd_slot(blockIdx.x, gridDim.x)];
    const FwdArgs<T> a = b.descs[it.x];
    defects_item<T, TP>(sh, a, mc, it.y);
}

// Throughput form of K1 for batches: one wave per interval, element-parallel
// right-hand side (one lane per body, joint, contact or row), fewer wave-cycles
// per interval than the two body-lane waves above.
template <class T, class TP>
struct DefLaneShared {
    Interval<T, TP> iv;
    RhsScratch<T, TP> sc;
};

template <class T, class TP>
__device__ __forceinline__ void defects_item_lane(DefLaneShared<T, TP>& sh, const FwdArgs<T>& a,
                                                  const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                                  const int k) {
    constexpr int NX = TP::NX, NXT = TP::NXT;
    const int lane = threadIdx.x;
    load_interval<T, TP>(sh.iv, a, mc, k, lane, 64);
    RowState<T> rs;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        rs.xb[q] = r < NXT ? sh.iv.x0[r] : T(0);
        rs.xa[q] = T(0);
        if (r < NXT) sh.sc.ns[r] = rs.xb[q];
    }
    wave_lds_sync();
    const int64_t ldi = a.ldi;
    for (int j = 0; j < a.K; ++j) {
        if (a.ckpt && (j % a.C) == 0) {
            const int slot = j / a.C;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int r = lane + 64 * q;
                if (r < NX) a.ckpt[((int64_t)slot * NX + r) * ldi + k] = rs.xb[q];
            }
        }
        for (int st = 0; st < 4; ++st) {
            const T tau = (T(j) + T(stage_c(st))) / T(a.K);
            rhs_eval<T, TP, FULL>(sh.iv, sh.sc, mc, lane, tau, (T*)nullptr);
            rk_rows<T, TP, NXT>(sh.iv, sh.sc, rs, lane, st, sh.sc.ns, (T*)nullptr);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NXT) {
            if (a.xprop) a.xprop[r * ldi + k] = rs.xb[q];
            a.defect[r * ldi + k] = rs.xb[q] - sh.iv.xk1[r];
        }
    }
}

template <class T, class TP>
__global__ void __launch_bounds__(64)
    k_defects_lane_batch(BatchArgs<FwdArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    __shared__ DefLaneShared<T, TP> sh;
    const int2 it = b.items[xcd_slot(blockIdx.x, gridDim.x)];
    const FwdArgs<T> a = b.descs[it.x];
    defects_item_lane<T, TP>(sh, a, mc, it.y);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <class T>
static FwdArgs<T> make_args(const cis_shape* sh, const void* X, const void* U, const void* s,
                            const void* prm) {
    FwdArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.X = (const T*)X;
    a.U = (const T*)U;
    a.s = (const T*)s;
    a.prm = (const T*)prm;
    a.ldn = sh->ld_node;
    a.ldi = sh->ld_int;
    a.N = sh->N;
    a.K = sh->substeps;
    a.C = 1;
    return a;
}

// Compute units of the current device (cached per device id).
static int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

template <class T, class TP>
static cis_status launch_discretize_as(const cis_model* m, const cis_shape* sh, const void* X,
                                       const void* U, const void* s, const void* prm, void* A,
                                       void* Bm, void* Bp, void* S, void* d, void* xp,
                                       hipStream_t stream) {
    auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
    FwdArgs<T> a = make_args<T>(sh, X, U, s, prm);
    a.A = (T*)A;
    a.Bm = (T*)Bm;
    a.Bp = (T*)Bp;
    a.S = (T*)S;
    a.defect = (T*)d;
    a.xprop = (T*)xp;
    void* args[] = {&a, &mc};
    hipError_t e = hipLaunchKernel((const void*)&k_discretize<T, TP>, dim3(sh->N, TP::NGRP),
                                   dim3(TP::NTHREADS), args, 0, stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_discretize launch: %s", hipGetErrorString(e));
    return CIS_OK;
}

// One trajectory: unless cis_shape.layout names one, the first layout whose
// (interval, column group) workgroups can all be resident at once, one per CU:
// latency (S group of its own), the latency layout with S on leg lanes,
// narrow; the throughput layout beyond.
template <class T, int L, int D>
static cis_status launch_discretize(const cis_model* m, const cis_shape* sh, const void* X,
                                    const void* U, const void* s, const void* prm, void* A,
                                    void* Bm, void* Bp, void* S, void* d, void* xp,
                                    hipStream_t stream) {
    using TL = LatencyTopo<T, L, D>;
    using TLS = LatencyTopoS<T, L, D>;
    using TN = NarrowTopo<T, L, D>;
    using TT = ThroughputTopo<T, L, D>;
    // an explicit layout (cis_shape.layout 1..4) overrides the rule
    switch (sh->layout) {
    case 1: return launch_discretize_as<T, TL>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    case 2: return launch_discretize_as<T, TLS>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    case 3: return launch_discretize_as<T, TN>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    case 4: return launch_discretize_as<T, TT>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    default: break;
    }
    const int cus = device_cus();
    if ((int64_t)sh->N * TL::NGRP <= cus)
        return launch_discretize_as<T, TL>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    if ((int64_t)sh->N * TLS::NGRP <= cus)
        return launch_discretize_as<T, TLS>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    if ((int64_t)sh->N * TN::NGRP <= cus)
        return launch_discretize_as<T, TN>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
    return launch_discretize_as<T, TT>(m, sh, X, U, s, prm, A, Bm, Bp, S, d, xp, stream);
}

template <class T, int L, int D>
static cis_status launch_defects(const cis_model* m, const cis_shape* sh, const void* X,
                                 const void* U, const void* s, const void* prm, void* d,
                                 void* xp, void* ckpt, int C, hipStream_t stream) {
    using TP = Topo<L, D>;
    auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
    FwdArgs<T> a = make_args<T>(sh, X, U, s, prm);
    a.defect = (T*)d;
    a.xprop = (T*)xp;
    a.ckpt = (T*)ckpt;
    a.C = C;
    void* args[] = {&a, &mc};
    hipError_t e = hipLaunchKernel((const void*)&k_defects<T, TP>, dim3(sh->N), dim3(128), args,
                                   0, stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_defects launch: %s", hipGetErrorString(e));
    return CIS_OK;
}

// ---------------------------------------------------------------------------
// substep blocks: pass 1 (defects with checkpoints at the block starts) and
// pass 2 (one discretize work item per (block, interval))
// ---------------------------------------------------------------------------
template <int L, int D>
static cis_status blocked_passes_t(const cis_model* m, const cis_shape* sh, const void* X,
                                   const void* U, const void* s, const void* prm, int B,
                                   double* ckpt, double* Ab, double* Bmb, double* Bpb,
                                   double* Sb, void* defect, void* xprop, hipStream_t stream) {
    using T = double;
    cis_status st = launch_defects<T, L, D>(m, sh, X, U, s, prm, defect, xprop, ckpt,
                                            sh->substeps / B, stream);
    if (st != CIS_OK) return st;
    FwdArgs<T> a = make_args<T>(sh, X, U, s, prm);
    a.A = Ab;
    a.Bm = Bmb;
    a.Bp = Bpb;
    a.S = Sb;
    a.ldi = (int64_t)B * sh->N;   // block outputs: column b N + k
    a.xinit = ckpt;
    a.ld_blk = sh->ld_int;        // checkpoints as written by pass 1
    a.B = B;
    using TL = LatencyTopo<T, L, D>;
    using TLS = LatencyTopoS<T, L, D>;
    using TN = NarrowTopo<T, L, D>;
    using TT = ThroughputTopo<T, L, D>;
    const int64_t items = (int64_t)B * sh->N;
    auto launch = [&](auto tp) -> cis_status {
        using TP = decltype(tp);
        auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
        void* args[] = {&a, &mc};
        hipError_t e = hipLaunchKernel((const void*)&k_discretize<T, TP>,
                                       dim3((unsigned)items, TP::NGRP), dim3(TP::NTHREADS), args,
                                       0, stream);
        if (e != hipSuccess)
            return fail(CIS_ERR_HIP, "k_discretize (blocks) launch: %s", hipGetErrorString(e));
        return CIS_OK;
    };
    if (items * TL::NGRP <= device_cus()) return launch(TL{});
    if (items * TLS::NGRP <= device_cus()) return launch(TLS{});
    if (items * TN::NGRP <= device_cus()) return launch(TN{});
    return launch(TT{});
}

cis_status blocked_passes(const cis_model* m, const cis_shape* sh, const void* X, const void* U,
                          const void* s, const void* prm, int B, double* ckpt, double* Ab,
                          double* Bmb, double* Bpb, double* Sb, void* defect, void* xprop,
                          hipStream_t stream) {
#define CIS_BLK(LL, DD)                                                                     \
    if (m->L == LL && m->D == DD)                                                           \
        return blocked_passes_t<LL, DD>(m, sh, X, U, s, prm, B, ckpt, Ab, Bmb, Bpb, Sb,     \
                                        defect, xprop, stream);
    CIS_TOPOLOGIES(CIS_BLK)
#undef CIS_BLK
    return fail(CIS_ERR_UNSUPPORTED, "substep blocks: topology has no compiled kernel");
}

// ---------------------------------------------------------------------------
// batched launch preparation (one model group)
// ---------------------------------------------------------------------------
template <class T>
static BatchArgs<FwdArgs<T>> batch_args(const BatchGroupDev& g) {
    BatchArgs<FwdArgs<T>> b;
    b.descs = (const FwdArgs<T>*)g.fdesc;
    b.items = g.items;
    b.n_items = g.n_items;
    b.cursor = g.cursor;
    return b;
}

template <class T, int L, int D>
static cis_status prep_disc_t(const cis_model* m, const BatchGroupDev& g, int persist_blocks,
                              int waves, KLaunch* out) {
    using TP = ThroughputTopo<T, L, D>;
    out->arg(batch_args<T>(g));
    out->arg(make_const<TP::NB, TP::NJ, TP::NC>(m));
    out->block = dim3(TP::NTHREADS);
    const bool pers = persist_blocks > 0;
    out->grid = dim3(pers ? persist_blocks : g.n_items * TP::NGRP);
    if (waves == 1) {
        out->func = pers ? (const void*)&k_discretize_batch<T, TP, true, 1>
                         : (const void*)&k_discretize_batch<T, TP, false, 1>;
    } else if (waves == 2) {
        if constexpr (sizeof(T) == 8) {
            out->func = pers ? (const void*)&k_discretize_batch<T, TP, true, 2>
                             : (const void*)&k_discretize_batch<T, TP, false, 2>;
        } else {
            return fail(CIS_ERR_DTYPE, "prep_discretize_batch: the two-wave form is FP64 only");
        }
    } else {
        return fail(CIS_ERR_DIM, "prep_discretize_batch: waves=%d", waves);
    }
    return out->ok() ? CIS_OK : fail(CIS_ERR_DIM, "prep_discretize_batch: launch record refused");
}

template <class T, int L, int D>
static cis_status prep_def_t(const cis_model* m, const BatchGroupDev& g, bool body_lanes,
                             KLaunch* out) {
    using TP = Topo<L, D>;
    out->arg(batch_args<T>(g));
    out->arg(make_const<TP::NB, TP::NJ, TP::NC>(m));
    out->func = body_lanes ? (const void*)&k_defects_batch<T, TP>
                           : (const void*)&k_defects_lane_batch<T, TP>;
    out->grid = dim3(g.n_items);
    out->block = dim3(body_lanes ? 128 : 64);
    return out->ok() ? CIS_OK : fail(CIS_ERR_DIM, "prep_defects_batch: launch record refused");
}

template <class T, int L, int D>
static int units_t() {
    return ThroughputTopo<T, L, D>::NGRP;
}

cis_status prep_discretize_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g,
                                 int persist_blocks, int waves, KLaunch* out) {
#define CIS_PREP_DISC(LL, DD)                                                                \
    if (m->L == LL && m->D == DD)                                                            \
        return dtype == CIS_F64 ? prep_disc_t<double, LL, DD>(m, g, persist_blocks, waves, out) \
                                : prep_disc_t<float, LL, DD>(m, g, persist_blocks, waves, out);
    CIS_TOPOLOGIES(CIS_PREP_DISC)
#undef CIS_PREP_DISC
    return fail(CIS_ERR_UNSUPPORTED, "prep_discretize_batch: topology has no compiled kernel");
}

cis_status prep_defects_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g,
                              bool body_lanes, KLaunch* out) {
#define CIS_PREP_DEF(LL, DD)                                                                \
    if (m->L == LL && m->D == DD)                                                           \
        return dtype == CIS_F64 ? prep_def_t<double, LL, DD>(m, g, body_lanes, out)         \
                                : prep_def_t<float, LL, DD>(m, g, body_lanes, out);
    CIS_TOPOLOGIES(CIS_PREP_DEF)
#undef CIS_PREP_DEF
    return fail(CIS_ERR_UNSUPPORTED, "prep_defects_batch: topology has no compiled kernel");
}

int discretize_units_per_item(const cis_model* m, int32_t dtype) {
#define CIS_UNITS(LL, DD)                                                                   \
    if (m->L == LL && m->D == DD)                                                           \
        return dtype == CIS_F64 ? units_t<double, LL, DD>() : units_t<float, LL, DD>();
    CIS_TOPOLOGIES(CIS_UNITS)
#undef CIS_UNITS
    return 0;
}

}  // namespace cis

using namespace cis;

static cis_status discretize_impl(const cis_model* model, const cis_shape* shape,
                                  const void* X, const void* U, const void* s,
                                  const void* params, void* A, void* Bm, void* Bp, void* S,
                                  void* defect, void* xprop, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    const size_t es = elem_size(shape->dtype);
    const bool hasm = model->m > 0;
    if (!A || !S || !defect || (hasm && (!Bm || !Bp)))
        return fail(CIS_ERR_NULL, "cis_discretize: A, S, defect (and Bm, Bp when m > 0) are required");
    if (!aligned(A, es) || !aligned(S, es) || !aligned(defect, es) || !aligned(xprop, es) ||
        !aligned(Bm, es) || !aligned(Bp, es))
        return fail(CIS_ERR_LAYOUT, "cis_discretize: output pointer not aligned to %zu bytes", es);
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_DISC(LL, DD)                                                                \
    if (model->L == LL && model->D == DD)                                                        \
        return shape->dtype == CIS_F64                                                          \
                   ? launch_discretize<double, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp,  \
                                                     S, defect, xprop, hs)                       \
                   : launch_discretize<float, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp,   \
                                                    S, defect, xprop, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_DISC)
#undef CIS_DISPATCH_DISC
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize: topology has no compiled kernel");
}

// Debug mode (CIS_DEBUG_FINITE): the non-finite scan after the launch.
extern "C" cis_status cis_discretize(const cis_model* model, const cis_shape* shape,
                                     const void* X, const void* U, const void* s,
                                     const void* params, void* A, void* Bm, void* Bp, void* S,
                                     void* defect, void* xprop, void* stream) {
    const cis_status st =
        discretize_impl(model, shape, X, U, s, params, A, Bm, Bp, S, defect, xprop, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    return debug_scan_forward("cis_discretize", model, shape, model->nx, model->m, X, U, s,
                              params, A, Bm, Bp, S, defect, xprop, nullptr, stream);
}

static cis_status defects_impl(const cis_model* model, const cis_shape* shape, const void* X,
                               const void* U, const void* s, const void* params,
                               void* defect, void* xprop, void* ckpt, int32_t ckpt_every,
                               void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    const size_t es = elem_size(shape->dtype);
    if (!defect) return fail(CIS_ERR_NULL, "cis_defects: defect is required");
    if (ckpt && (ckpt_every < 1 || shape->substeps % ckpt_every != 0))
        return fail(CIS_ERR_DIM, "cis_defects: ckpt_every=%d must divide K=%d", ckpt_every,
                    shape->substeps);
    if (!aligned(defect, es) || !aligned(xprop, es) || !aligned(ckpt, es))
        return fail(CIS_ERR_LAYOUT, "cis_defects: output pointer not aligned to %zu bytes", es);
    const int C = ckpt ? ckpt_every : 1;
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_DEF(LL, DD)                                                              \
    if (model->L == LL && model->D == DD)                                                      \
        return shape->dtype == CIS_F64                                                        \
                   ? launch_defects<double, LL, DD>(model, shape, X, U, s, params, defect,      \
                                                  xprop, ckpt, C, hs)                          \
                   : launch_defects<float, LL, DD>(model, shape, X, U, s, params, defect,       \
                                                 xprop, ckpt, C, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_DEF)
#undef CIS_DISPATCH_DEF
    return fail(CIS_ERR_UNSUPPORTED, "cis_defects: topology has no compiled kernel");
}

extern "C" cis_status cis_defects(const cis_model* model, const cis_shape* shape, const void* X,
                                  const void* U, const void* s, const void* params,
                                  void* defect, void* xprop, void* ckpt, int32_t ckpt_every,
                                  void* stream) {
    const cis_status st =
        defects_impl(model, shape, X, U, s, params, defect, xprop, ckpt, ckpt_every, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    return debug_scan_forward("cis_defects", model, shape, model->nx, model->m, X, U, s, params,
                              nullptr, nullptr, nullptr, nullptr, defect, xprop, nullptr, stream);
}
