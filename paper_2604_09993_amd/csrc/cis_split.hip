// Split form of the discretize step for many intervals (arxiv 2604.09993,
// Sec. IV-B eq. intg-aug-sys-param; sensitivities by internal numerical
// differentiation, Sec. VI).  Two kernels per batch of intervals:
//
//   k_coefrec : per interval three waves, the nominal RK4 recursion on body
//               lanes, the right-hand side and Jacobian coefficients of
//               every stage, and the dilation column S on body lanes; writes
//               F~, the defect, S, the integral-state columns of A, and a
//               compact record of every stage's coefficients (CoefRec) to a
//               workspace in device memory.
//   k_tangent : per (interval, block of 64 tangent columns) one wave per leg.
//               Lane c holds column c of Z = [Phi_x | B- | B+] on the rows of
//               the torso and of the wave's leg; every coefficient a wave
//               needs is the same for all its lanes, so it is read with
//               scalar loads from the stage record and enters the FMAs as a
//               scalar operand (no LDS traffic for coefficients, no wait on
//               the nominal recursion).  The torso rows are integrated
//               identically in every leg wave; the only exchange is the hip
//               stiffness and damping torque of each leg on the torso (one
//               value per column and stage, through LDS).
//
// The two kernels exchange per interval 8 + 4 n_j constants and 4 K records
// of CoefRec<TP>::GLOBAL elements.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/cis.h"
#include "cis_body.hpp"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_model.hpp"
#include "cis_split.hpp"

namespace cis {

template <class T, class TP>
struct RecShared {
    Interval<T, TP> iv;
    T xring[4][TP::NX];        // stage inputs from the state wave
    T csring[4][TP::NB][2];    // their rotations
    T fring[4][3 * TP::NB];    // their accelerations
    T coef[2][CoefRec<TP>::SIZE];
};

// ---------------------------------------------------------------------------
// k_coefrec: interval k by two waves, one workgroup barrier per step:
//   wave 0 (state, S column): stage t of the nominal recursion at step t, and
//                          the S column's stage t-2 from coef[(t-2) & 1] with
//                          the copy of that record to device memory;
//   wave 1 (coefficients): stage t-1 at step t, into coef[(t-1) & 1].
// ---------------------------------------------------------------------------
template <class T, class TP>
__device__ __forceinline__ void coefrec_item(RecShared<T, TP>& sh, const FwdArgs<T>& a,
                                             const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                             const int k, T* __restrict__ rec) {
    constexpr int NB = TP::NB, NX = TP::NX, NXT = TP::NXT, NY = TP::NY, NQ = TP::NQ;
    constexpr int NC = TP::NC, NJ = TP::NJ, L = TP::L, D = TP::D;
    using R = CoefRec<TP>;
    using SR = SplitRec<TP>;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = 128;
    load_interval<T, TP>(sh.iv, a, mc, k, tid, nth);
    for (int e = tid; e < 2 * R::SIZE; e += nth) (&sh.coef[0][0])[e] = T(0);
    __syncthreads();
    coefrec_constants<T, TP>(sh.iv, sh.coef[0], tid, nth);
    coefrec_constants<T, TP>(sh.iv, sh.coef[1], tid, nth);
    // per-interval constants of the tangent kernel
    for (int e = tid; e < SR::CRS; e += nth) {
        T v = T(0);
        if (e == 0) v = sh.iv.s;
        else if (e == 1) v = sh.iv.h;
        else if (e == 2) v = sh.iv.h6;
        else if (e >= 8 && e < 8 + 4 * NJ) v = sh.iv.kc[(e - 8) >> 2][(e - 8) & 3];
        rec[e] = v;
    }
    const int nst = 4 * a.K;
    const int nsteps = nst + 2;
    const int64_t ldi = a.ldi;
    __syncthreads();

    if (wave == 0) {
        // ---- state wave: stage t at step t; S column: stage t-2 at step t ----
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
        SLane<T, TP> z;
#pragma unroll
        for (int r = 0; r < 6; ++r) z.zs[r] = z.zb[r] = z.za[r] = T(0);
#pragma unroll
        for (int l = 0; l < SLane<T, TP>::NCL; ++l) z.ycc[l] = T(0);
        z.yct = T(0);
        const T Kt = T(a.K);
        T* out = rec + SR::CRS;
        // steps t = 4 j + ST, t < nsteps: one barrier each (both stage indices
        // known at compile time inside the unrolled substep)
        auto step = [&](auto st_c, int j) {
            constexpr int ST = decltype(st_c)::value;
            constexpr int SS = (ST + 2) & 3;   // S stage of this step
            const int t = 4 * j + ST;
            if (t < nst) {
                const T jt = T(j);
                const T tau = ST == 0 ? jt / Kt : (ST == 3 ? (jt + T(1)) / Kt : (jt + T(0.5)) / Kt);
                state_stage<T, TP, ST>(sh.iv, mc, c, bs, tau, sh.xring[(ST + 1) & 3],
                                       sh.csring[ST], sh.fring[ST], lane);
            }
            if (t >= 2) {
                const T* cf = sh.coef[SS & 1];
                s_stage<T, TP, SS, R>(sh.iv, c, z, cf, lane);
#pragma unroll
                for (int e = lane; e < R::GLOBAL; e += 64) out[e] = cf[e];
                out += R::GLOBAL;
            }
            __syncthreads();
        };
        for (int j = 0; 4 * j < nsteps; ++j) {
            step(std::integral_constant<int, 0>{}, j);
            step(std::integral_constant<int, 1>{}, j);
            if (4 * j + 2 < nsteps) {
                step(std::integral_constant<int, 2>{}, j);
                step(std::integral_constant<int, 3>{}, j);
            }
        }
        if (lane < NB) {
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) {
                const int r = kk < 3 ? 3 * c.b + kk : NQ + 3 * c.b + kk - 3;
                if (a.xprop) a.xprop[r * ldi + k] = bs.xb[kk];
                a.defect[r * ldi + k] = bs.xb[kk] - sh.iv.xk1[r];
            }
        }
        T yct = T(0);
#pragma unroll
        for (int e = 0; e < NB; ++e) yct += lane_value(z.yct, e);
        if (lane < NB) {
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                a.S[(int64_t)(3 * c.b + kk) * ldi + k] = z.zb[kk];
                a.S[(int64_t)(NQ + 3 * c.b + kk) * ldi + k] = z.zb[3 + kk];
            }
            if (c.contact) a.S[(int64_t)(NX + c.i) * ldi + k] = z.ycc[0];
            if (lane == 0) a.S[(int64_t)(NX + NC) * ldi + k] = yct;
        }
    } else {
        // ------- coefficient wave: stage tc at step tc + 1; integral rows -------
        const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
        const int ycc_row = NX + c.i;
        T ycb = c.contact ? sh.iv.x0[ycc_row] : T(0), yca = T(0);
        T ytb = lane == 0 ? sh.iv.x0[NX + NC] : T(0), yta = T(0);
        const T s = sh.iv.s;
        __syncthreads();
        for (int tc = 0; tc < nst; ++tc) {
            const int st = tc & 3;
            const T tau = (T(tc >> 2) + T(stage_c(st))) / T(a.K);
            T ycc = T(0), yct = T(0);
            coef_stage<T, TP, false, true, R, 2>(sh.iv, mc, c,
                                                     tc == 0 ? sh.iv.x0 : sh.xring[tc & 3],
                                                     sh.csring[tc & 3], sh.fring[tc & 3], tau,
                                                     sh.coef[tc & 1], ycc, yct, lane);
            const T wk = (st == 0 || st == 3) ? T(1) : T(2);
            if (st == 0) {
                yca = wk * s * ycc;
                yta = wk * s * yct;
            } else {
                yca += wk * s * ycc;
                yta += wk * s * yct;
            }
            if (st == 3) {
                ycb += sh.iv.h6 * yca;
                ytb += sh.iv.h6 * yta;
            }
            __syncthreads();
        }
        __syncthreads();
        {
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
        // A[:, n:] = [0; I]: the integral states feed back into nothing
        for (int e = lane; e < NXT * NY; e += 64) {
            const int r = e / NY, cc = NX + e % NY;
            a.A[((int64_t)r * NXT + cc) * ldi + k] = (r == cc) ? T(1) : T(0);
        }
    }
    (void)L;
    (void)D;
}

// ---------------------------------------------------------------------------
// k_tangent: one classical RK4 stage of a leg wave (derivative from
// tangent_split_rhs, then the RK4 combination).
// ---------------------------------------------------------------------------
template <class T, class TP, int ST, bool FORCE, bool LDSF>
__device__ __forceinline__ void tangent_split_stage(TanLane<T, TP>& z, const T* __restrict__ cr,
                                                    const T* __restrict__ lr,
                                                    const T* __restrict__ rs, T* xch, int leg,
                                                    int lane, T tau, T wbm, T wbp,
                                                    const unsigned (&off)[3 * (TP::D + 1)],
                                                    unsigned offcc, T* fbuf,
                                                    const T* rs_next) {
    constexpr int LB = TP::D + 1;
    constexpr int FBUF = SplitRec<TP>::FBUF;
    const T s = cr[0], h = cr[1], h6 = cr[2];
    T kv[3 * LB], kcc, kct;
    // forcing regions alternate between the two LDS buffers stage by stage
    // (4 stages per substep, so the parity of the stage is that of ST)
    tangent_split_rhs<T, TP, FORCE, LDSF>(z.zs, cr, lr, rs, xch, leg, lane, tau, wbm, wbp, off,
                                          offcc, kv, kcc, kct, fbuf + (ST & 1) * FBUF, rs_next,
                                          fbuf + ((ST + 1) & 1) * FBUF);
    // classical RK4 combination (stage ST known at compile time)
    constexpr int WK = (ST == 0 || ST == 3) ? 1 : 2;
    const T an = (ST == 2) ? h : T(0.5) * h;
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) {
        const T kq = s * z.zs[3 * LB + r];
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
    z.ycc += (h6 * T(WK)) * kcc;
    z.yct += (h6 * T(WK)) * kct;
    if (ST == 3) {
#pragma unroll
        for (int r = 0; r < 6 * LB; ++r) {
            z.zb[r] += h6 * z.za[r];
            z.zs[r] = z.zb[r];
        }
    }
}

template <class T, class TP, bool FORCE, bool LDSF>
__device__ __forceinline__ void tangent_split_loop(TanLane<T, TP>& z, const T* __restrict__ cr,
                                                   const T* __restrict__ rec0, T* xch, int leg,
                                                   int lane, int K, T wbm, T wbp,
                                                   const unsigned (&off)[3 * (TP::D + 1)],
                                                   unsigned offcc, T* fbuf) {
    using R = CoefRec<TP>;
    constexpr int LEGB = R::LEGB, GL = R::GLOBAL, L = TP::L;
    const T Kt = T(K);
    const T* rs = rec0;
    for (int j = 0; j < K; ++j) {
        const T jt = T(j);
        const T tau0 = jt / Kt, tauh = (jt + T(0.5)) / Kt, tau1 = (jt + T(1)) / Kt;
        T* x0 = xch;
        T* x1 = xch + L * 64;
        tangent_split_stage<T, TP, 0, FORCE, LDSF>(z, cr, rs + leg * LEGB, rs, x0, leg, lane,
                                                   tau0, wbm, wbp, off, offcc, fbuf, rs + GL);
        rs += GL;
        tangent_split_stage<T, TP, 1, FORCE, LDSF>(z, cr, rs + leg * LEGB, rs, x1, leg, lane,
                                                   tauh, wbm, wbp, off, offcc, fbuf, rs + GL);
        rs += GL;
        tangent_split_stage<T, TP, 2, FORCE, LDSF>(z, cr, rs + leg * LEGB, rs, x0, leg, lane,
                                                   tauh, wbm, wbp, off, offcc, fbuf, rs + GL);
        rs += GL;
        // the last stage of the interval copies its own region (never read)
        tangent_split_stage<T, TP, 3, FORCE, LDSF>(z, cr, rs + leg * LEGB, rs, x1, leg, lane,
                                                   tau1, wbm, wbp, off, offcc, fbuf,
                                                   j + 1 < K ? rs + GL : rs);
        rs += GL;
    }
}

// Columns [64 cb, 64 cb + 64) of interval k, wave `leg` (all waves of the block).
template <class T, class TP>
__device__ __forceinline__ void tangent_item(const FwdArgs<T>& a, const T* __restrict__ rec,
                                             const int k, const int cb, T* xch, T* fbuf) {
    constexpr int D = TP::D, LB = D + 1;
    using SR = SplitRec<TP>;
    const int tid = threadIdx.x, lane = tid & 63;
    const int leg = __builtin_amdgcn_readfirstlane(tid >> 6);
    T wbm, wbp;
    TanLane<T, TP> z;
    const TanCol<TP> tc = tangent_column<T, TP>(cb, leg, lane, wbm, wbp, z.zb);
#pragma unroll
    for (int r = 0; r < 6 * LB; ++r) {
        z.zs[r] = z.zb[r];
        z.za[r] = T(0);
    }
    z.ycc = T(0);
    z.yct = T(0);
    const T* cr = rec;
    const T* rec0 = rec + SR::CRS;
    // blocks holding no B-/B+ column skip the forcing code (uniform branch)
    if constexpr (TP::L > 1) {
        // every block stages the records (in blocks without B-/B+ columns
        // only to bring the leg blocks into the L2 cache a stage early)
        stage_store<T, TP>(fbuf, stage_load<T, TP>(rec0, leg, lane), leg, lane);
    }
    if ((cb + 1) * 64 <= TP::NX) {
        tangent_split_loop<T, TP, false, (TP::L > 1)>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp,
                                                      tc.off, tc.offcc, fbuf);
    } else if constexpr (TP::L > 1) {
        // forcing from the stage records staged in LDS (stage 0's record
        // stored above, ordered before its reads by stage 0's barrier)
        tangent_split_loop<T, TP, true, true>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp, tc.off,
                                              tc.offcc, fbuf);
    } else {
        tangent_split_loop<T, TP, true, false>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp, tc.off,
                                               tc.offcc, fbuf);
    }
    tangent_store<T, TP>(a, k, leg, lane, tc, z.zb, z.ycc, z.yct, xch);
}

// Single trajectory: rec holds N interval parts of per_interval(K) elements.
// FP32 at four waves per SIMD (128 VGPRs, a few bytes of scratch), FP64 at two.
template <class T, class TP>
__global__ void __launch_bounds__(128)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
    k_coefrec(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc,
                                                 T* __restrict__ rec) {
    __shared__ RecShared<T, TP> sh;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    coefrec_item<T, TP>(sh, a, mc, k, rec + (int64_t)k * SplitRec<TP>::per_interval(a.K));
}

template <class T, class TP, int WAVES>
__global__ void __launch_bounds__(64 * TP::L) __attribute__((amdgpu_waves_per_eu(WAVES)))
    k_tangent(FwdArgs<T> a, const T* __restrict__ rec) {
    __shared__ T xch[2 * TP::L * 64];
    __shared__ T fbuf[2 * SplitRec<TP>::FBUF];
    int item, cb;
    unit_item(xcd_slot(blockIdx.x, gridDim.x), a.N, SplitRec<TP>::NBLK, item, cb);
    tangent_item<T, TP>(a, rec + (int64_t)item * SplitRec<TP>::per_interval(a.K), item, cb, xch,
                        fbuf);
}

// Batches: one launch per model over the work list; rec_off[item] is the
// element offset of the item's part of the workspace.
// FP32 at four waves per SIMD (128 VGPRs, a few bytes of scratch), FP64 at two.
template <class T, class TP>
__global__ void __launch_bounds__(128)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
    k_coefrec_batch(BatchArgs<FwdArgs<T>> b, MConst<TP::NB, TP::NJ, TP::NC> mc,
                    T* __restrict__ rec, const int64_t* __restrict__ rec_off) {
    __shared__ RecShared<T, TP> sh;
    const int item = xcd_slot(blockIdx.x, gridDim.x);
    const int2 it = b.items[item];
    const FwdArgs<T> a = b.descs[it.x];
    coefrec_item<T, TP>(sh, a, mc, it.y, rec + rec_off[item]);
}

template <class T, class TP, int WAVES>
__global__ void __launch_bounds__(64 * TP::L) __attribute__((amdgpu_waves_per_eu(WAVES)))
    k_tangent_batch(BatchArgs<FwdArgs<T>> b, const T* __restrict__ rec,
                    const int64_t* __restrict__ rec_off) {
    __shared__ T xch[2 * TP::L * 64];
    __shared__ T fbuf[2 * SplitRec<TP>::FBUF];
    int item, cb;
    unit_item(xcd_slot(blockIdx.x, gridDim.x), b.n_items, SplitRec<TP>::NBLK, item, cb);
    const int2 it = b.items[item];
    const FwdArgs<T> a = b.descs[it.x];
    tangent_item<T, TP>(a, rec + rec_off[item], it.y, cb, xch, fbuf);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <int L, int D>
struct SplitTopo {
    static constexpr bool ok = L >= 1 && D >= 1;
};

static bool split_supported(const cis_model* m) { return m->L >= 1 && m->D >= 1; }

template <int L, int D>
static int64_t split_elems_t(int K) {
    if constexpr (L >= 1 && D >= 1) return SplitRec<Topo<L, D>>::per_interval(K);
    else return -1;
}

int64_t split_elems_per_interval(const cis_model* m, int K) {
#define CIS_SPLIT_SZ(LL, DD) \
    if (m->L == LL && m->D == DD) return split_elems_t<LL, DD>(K);
    CIS_TOPOLOGIES(CIS_SPLIT_SZ)
#undef CIS_SPLIT_SZ
    return -1;
}

template <class T, int L, int D>
static cis_status launch_split_t(const cis_model* m, const cis_shape* sh, const void* X,
                                 const void* U, const void* s, const void* prm, void* A, void* Bm,
                                 void* Bp, void* S, void* defect, void* xprop, void* ws,
                                 int waves, hipStream_t stream) {
    if constexpr (L >= 1 && D >= 1) {
        using TP = Topo<L, D>;
        auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
        FwdArgs<T> a;
        std::memset(&a, 0, sizeof(a));
        a.X = (const T*)X;
        a.U = (const T*)U;
        a.s = (const T*)s;
        a.prm = (const T*)prm;
        a.A = (T*)A;
        a.Bm = (T*)Bm;
        a.Bp = (T*)Bp;
        a.S = (T*)S;
        a.defect = (T*)defect;
        a.xprop = (T*)xprop;
        a.ldn = sh->ld_node;
        a.ldi = sh->ld_int;
        a.N = sh->N;
        a.K = sh->substeps;
        a.C = 1;
        T* rec = (T*)ws;
        void* args_a[] = {&a, &mc, &rec};
        hipError_t e = hipLaunchKernel((const void*)&k_coefrec<T, TP>, dim3(sh->N), dim3(128),
                                       args_a, 0, stream);
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_coefrec launch: %s", hipGetErrorString(e));
        const T* crec = rec;
        void* args_b[] = {&a, &crec};
        e = hipLaunchKernel(waves == 2 ? (const void*)&k_tangent<T, TP, 2>
                                       : (const void*)&k_tangent<T, TP, 1>,
                            dim3(sh->N * SplitRec<TP>::NBLK), dim3(64 * TP::L), args_b, 0, stream);
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_tangent launch: %s", hipGetErrorString(e));
        return CIS_OK;
    } else {
        return fail(CIS_ERR_UNSUPPORTED, "split form needs legs with links");
    }
}

template <class T, int L, int D>
static cis_status prep_split_t(const cis_model* m, const BatchGroupDev& g, int waves,
                               KLaunch* ka, KLaunch* kb) {
    if constexpr (L >= 1 && D >= 1) {
        using TP = Topo<L, D>;
        BatchArgs<FwdArgs<T>> b;
        b.descs = (const FwdArgs<T>*)g.fdesc;
        b.items = g.items;
        b.n_items = g.n_items;
        b.cursor = g.cursor;
        ka->arg(b);
        ka->arg(make_const<TP::NB, TP::NJ, TP::NC>(m));
        ka->arg((T*)g.rec);
        ka->arg(g.rec_off);
        ka->func = (const void*)&k_coefrec_batch<T, TP>;
        ka->grid = dim3(g.n_items);
        ka->block = dim3(128);
        kb->arg(b);
        kb->arg((const T*)g.rec);
        kb->arg(g.rec_off);
        kb->func = waves == 2 ? (const void*)&k_tangent_batch<T, TP, 2>
                              : (const void*)&k_tangent_batch<T, TP, 1>;
        kb->grid = dim3(g.n_items * SplitRec<TP>::NBLK);
        kb->block = dim3(64 * TP::L);
        return ka->ok() && kb->ok() ? CIS_OK
                                    : fail(CIS_ERR_DIM, "prep_split_batch: launch record refused");
    } else {
        return fail(CIS_ERR_UNSUPPORTED, "split form needs legs with links");
    }
}

cis_status prep_split_batch(const cis_model* m, int32_t dtype, const BatchGroupDev& g,
                            int waves, KLaunch* ka, KLaunch* kb) {
#define CIS_PREP_SPLIT(LL, DD)                                                        \
    if (m->L == LL && m->D == DD)                                                     \
        return dtype == CIS_F64 ? prep_split_t<double, LL, DD>(m, g, waves, ka, kb)   \
                                : prep_split_t<float, LL, DD>(m, g, waves, ka, kb);
    CIS_TOPOLOGIES(CIS_PREP_SPLIT)
#undef CIS_PREP_SPLIT
    return fail(CIS_ERR_UNSUPPORTED, "prep_split_batch: topology has no compiled kernel");
}

bool split_form_supported(const cis_model* m) { return split_supported(m); }

}  // namespace cis

using namespace cis;

static cis_status split_ws_bytes(const cis_model* m, const cis_shape* sh, size_t* bytes) {
    const int64_t per = split_elems_per_interval(m, sh->substeps);
    if (per < 0)
        return fail(CIS_ERR_UNSUPPORTED, "split form: the model has no legs with links");
    *bytes = (size_t)per * (size_t)sh->N * elem_size(sh->dtype);
    return CIS_OK;
}

extern "C" cis_status cis_split_workspace_size(const cis_model* m, const cis_shape* sh,
                                               size_t* bytes) {
    if (!m || !sh || !bytes) return fail(CIS_ERR_NULL, "cis_split_workspace_size: null argument");
    if (sh->N < 1 || sh->substeps < 1 || sh->substeps > 4096)
        return fail(CIS_ERR_DIM, "cis_split_workspace_size: N=%d, K=%d out of range", sh->N,
                    sh->substeps);
    if (sh->dtype != CIS_F64 && sh->dtype != CIS_F32)
        return fail(CIS_ERR_DTYPE, "cis_split_workspace_size: unknown dtype %d", sh->dtype);
    return split_ws_bytes(m, sh, bytes);
}

static cis_status discretize_split_impl(const cis_model* model, const cis_shape* shape,
                                        const void* X, const void* U, const void* s,
                                        const void* params, int32_t waves, void* A, void* Bm,
                                        void* Bp, void* S, void* defect, void* xprop, void* ws,
                                        size_t ws_bytes, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (waves != 1 && waves != 2)
        return fail(CIS_ERR_DIM, "cis_discretize_split: waves=%d must be 1 or 2", waves);
    const bool hasm = model->m > 0;
    if (!A || !S || !defect || (hasm && (!Bm || !Bp)))
        return fail(CIS_ERR_NULL, "cis_discretize_split: A, S, defect (and Bm, Bp when m > 0) are required");
    const size_t es = elem_size(shape->dtype);
    if (!aligned(A, es) || !aligned(S, es) || !aligned(defect, es) || !aligned(xprop, es) ||
        !aligned(Bm, es) || !aligned(Bp, es) || !aligned(ws, 8))
        return fail(CIS_ERR_LAYOUT, "cis_discretize_split: pointer not aligned to %zu bytes", es);
    size_t need = 0;
    st = split_ws_bytes(model, shape, &need);
    if (st != CIS_OK) return st;
    if (!ws || ws_bytes < need)
        return fail(CIS_ERR_WORKSPACE, "cis_discretize_split: workspace of %zu bytes needed", need);
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_SPLIT(LL, DD)                                                             \
    if (model->L == LL && model->D == DD)                                                      \
        return shape->dtype == CIS_F64                                                         \
                   ? launch_split_t<double, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp, \
                                                    S, defect, xprop, ws, waves, hs)           \
                   : launch_split_t<float, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp,  \
                                                   S, defect, xprop, ws, waves, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_SPLIT)
#undef CIS_DISPATCH_SPLIT
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_split: topology has no compiled kernel");
}

extern "C" cis_status cis_discretize_split(const cis_model* model, const cis_shape* shape,
                                           const void* X, const void* U, const void* s,
                                           const void* params, int32_t waves, void* A, void* Bm,
                                           void* Bp, void* S, void* defect, void* xprop, void* ws,
                                           size_t ws_bytes, void* stream) {
    const cis_status st = discretize_split_impl(model, shape, X, U, s, params, waves, A, Bm, Bp,
                                                S, defect, xprop, ws, ws_bytes, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    return debug_scan_forward("cis_discretize_split", model, shape, model->nx, model->m, X, U,
                              s, params, A, Bm, Bp, S, defect, xprop, nullptr, stream);
}
