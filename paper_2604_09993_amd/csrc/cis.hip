// MI355X (gfx950) kernels and C ABI for the CI-SCvx interval
// linearize-and-discretize step (arxiv 2604.09993, Sec. IV-B and Sec. VI).
//
// Kernels (one workgroup per interval):
//   k_discretize : nominal RK4 + variational equations -> A, B-, B+, S, d, F~
//   k_defects    : nominal RK4 only -> d, F~ and substep checkpoints
// The adjoint kernels live in cis_adjoint.hip.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cis.h"
#include "cis_model.hpp"
#include "cis_host.hpp"

namespace cis {

// ---------------------------------------------------------------------------
// Tangent stage: one column of Z = [Phi_x | B- | B+ | S] per lane.
// zb: substep base, za: RK4 accumulator, zs: stage input (x rows only; no row
// of the right-hand side depends on the integral states y), zy: y rows.
// wbm / wbp / fsel select the forcing of a B-, B+ or S column.
// ---------------------------------------------------------------------------
template <class T, class TP>
struct Column {
    T zb[TP::NX], za[TP::NX], zs[TP::NX], zy[TP::NY];
};

template <class T, class TP, class SM>
__device__ __forceinline__ void tangent_stage(const SM& sm, Column<T, TP>& z, const T* cf,
                                              int st, T tau, T wbm, T wbp, T fsel, int ctrl) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, NX = TP::NX, M = TP::M;
    using C = Coef<TP>;
    const T s = sm.s, h = sm.h;
    T kv[3 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        kv[3 * b] = T(0);
        kv[3 * b + 1] = T(0);
        kv[3 * b + 2] = cf[C::CTH + b] * z.zs[3 * b + 2];
    }
    T kct = T(0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int p = TP::parent(j), c = j + 1;
        const T dth = z.zs[3 * c + 2] - z.zs[3 * p + 2];
        const T dom = z.zs[NQ + 3 * c + 2] - z.zs[NQ + 3 * p + 2];
        kv[3 * p + 2] += sm.kc[j][0] * dth + sm.kc[j][1] * dom;
        kv[3 * c + 2] -= sm.kc[j][2] * dth + sm.kc[j][3] * dom;
        const T* jh = cf + C::JH + 4 * j;
        kct += jh[0] * (z.zs[3 * p] - z.zs[3 * c]) + jh[1] * (z.zs[3 * p + 1] - z.zs[3 * c + 1]) +
               jh[2] * z.zs[3 * p + 2] + jh[3] * z.zs[3 * c + 2];
    }
    T kcc[cmax(NC, 1)];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int b = TP::cbody(i);
        const T* ct = cf + C::CT + C::NCT * i;
        const T dPx = z.zs[3 * b] - ct[C_AY] * z.zs[3 * b + 2];
        const T dPy = z.zs[3 * b + 1] + ct[C_AX] * z.zs[3 * b + 2];
        kv[3 * b] += ct[C_FXP] * dPx;
        kv[3 * b + 1] += ct[C_FYP] * dPx;
        kv[3 * b + 2] += ct[C_TP] * dPx;
        kcc[i] = ct[C_EPX] * dPx + ct[C_EPY] * dPy + ct[C_EXD] * z.zs[NQ + 3 * b] +
                 ct[C_EYD] * z.zs[NQ + 3 * b + 1] + ct[C_EOM] * z.zs[NQ + 3 * b + 2] +
                 ct[C_ETH] * z.zs[3 * b + 2];
        kct += ct[C_ZPX] * dPx + ct[C_ZPY] * dPy;
    }
    // FOH forcing of B-/B+ columns: s (J_u w(tau) + J_ubar / 2)
    if constexpr (M > 0) {
        const T wB = wbm * (T(1) - tau) + wbp * tau;
        const T wC = wbm + wbp;
#pragma unroll
        for (int r = 0; r < 3 * NB; ++r) kv[r] += wB * cf[C::GV + r * M + ctrl];
#pragma unroll
        for (int i = 0; i < NC; ++i) kcc[i] += wC * cf[C::GC + i * M + ctrl];
    }
    // dilation column forcing: F~ at the stage
#pragma unroll
    for (int r = 0; r < 3 * NB; ++r) kv[r] += fsel * cf[C::F + NQ + r];
#pragma unroll
    for (int i = 0; i < NC; ++i) kcc[i] += fsel * cf[C::F + NX + i];
    kct += fsel * cf[C::F + NX + NC];
    // classical RK4 combination
    const T wk = (st == 0 || st == 3) ? T(1) : T(2);
    const T an = (st == 2) ? h : T(0.5) * h;
    const T h6w = (h / T(6)) * wk;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const T kq = s * z.zs[NQ + r] + fsel * cf[C::F + r];
        if (st == 0) z.za[r] = kq;
        else z.za[r] += wk * kq;
        if (st < 3) z.zs[r] = z.zb[r] + an * kq;
    }
#pragma unroll
    for (int r = 0; r < 3 * NB; ++r) {
        const T kk = kv[r];
        if (st == 0) z.za[NQ + r] = kk;
        else z.za[NQ + r] += wk * kk;
        if (st < 3) z.zs[NQ + r] = z.zb[NQ + r] + an * kk;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) z.zy[i] += h6w * kcc[i];
    z.zy[NC] += h6w * kct;
    if (st == 3) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            z.zb[r] += (h / T(6)) * z.za[r];
            z.zs[r] = z.zb[r];
        }
    }
}

// ---------------------------------------------------------------------------
// K2: discretize.  Workgroup = NCW tangent waves + 1 nominal wave.  The
// nominal wave runs one stage ahead and fills the coefficient buffer of the
// next stage while the tangent waves consume the current one; one workgroup
// barrier per stage.
// ---------------------------------------------------------------------------
template <class T, class TP>
__global__ void __launch_bounds__(TP::NTHREADS)
    k_discretize(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NX = TP::NX, NXT = TP::NXT, M = TP::M;
    constexpr int NY = TP::NY;
    using C = Coef<TP>;
    __shared__ Shared<T, TP, 2> sm;
    const int k = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nth = TP::NTHREADS;
    load_interval<T, TP>(sm, a, mc, k, tid, nth);
    // zero both coefficient buffers, then the constant FOH forcing entries
    for (int e = tid; e < 2 * C::SIZE; e += nth) (&sm.coef[0][0])[e] = T(0);
    __syncthreads();
    const T s = sm.s;
    for (int j = tid; j < NJ; j += nth) {
        const int p = TP::parent(j), c = j + 1;
        sm.kc[j][0] = s * T(mc.ks[j]) * sm.iinv[p];
        sm.kc[j][1] = s * T(mc.ds[j]) * sm.iinv[p];
        sm.kc[j][2] = s * T(mc.ks[j]) * sm.iinv[c];
        sm.kc[j][3] = s * T(mc.ds[j]) * sm.iinv[c];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            T* gv = sm.coef[q] + C::GV;
            gv[(3 * p) * M + NJ + 2 * j] = s * sm.minv[p];
            gv[(3 * p + 1) * M + NJ + 2 * j + 1] = s * sm.minv[p];
            gv[(3 * c) * M + NJ + 2 * j] = -s * sm.minv[c];
            gv[(3 * c + 1) * M + NJ + 2 * j + 1] = -s * sm.minv[c];
            gv[(3 * p + 2) * M + j] = -s * sm.iinv[p];
            gv[(3 * c + 2) * M + j] = s * sm.iinv[c];
        }
    }
    __syncthreads();

    const bool nominal = wave == TP::NCW;
    const int nst = 4 * a.K;
    RowState<T> rs;
    Column<T, TP> z;
    const int col = wave * 64 + lane;
    T wbm = T(0), wbp = T(0), fsel = T(0);
    int ctrl = 0;
    if (nominal) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = lane + 64 * q;
            rs.xb[q] = r < NXT ? sm.ns[r] : T(0);
            rs.xa[q] = T(0);
        }
        nominal_rhs<T, TP, true>(sm, mc, lane, T(0), sm.coef[0]);
        nominal_update<T, TP, true>(sm, rs, lane, 0, sm.coef[0]);
    } else {
        if (col >= NX && col < NX + M) { wbm = T(1); ctrl = col - NX; }
        else if (col >= NX + M && col < NX + 2 * M) { wbp = T(1); ctrl = col - NX - M; }
        else if (col == NX + 2 * M) fsel = T(1);
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            z.zb[r] = (r == col) ? T(1) : T(0);
            z.zs[r] = z.zb[r];
            z.za[r] = T(0);
        }
#pragma unroll
        for (int i = 0; i < NY; ++i) z.zy[i] = T(0);
    }
    __syncthreads();
    for (int t = 0; t < nst; ++t) {
        if (nominal) {
            const int t1 = t + 1;
            if (t1 < nst) {
                const int st = t1 & 3;
                const T tau = (T(t1 >> 2) + T(stage_c(st))) / T(a.K);
                nominal_rhs<T, TP, true>(sm, mc, lane, tau, sm.coef[t1 & 1]);
                nominal_update<T, TP, true>(sm, rs, lane, st, sm.coef[t1 & 1]);
            }
        } else {
            const int st = t & 3;
            const T tau = (T(t >> 2) + T(stage_c(st))) / T(a.K);
            tangent_stage<T, TP>(sm, z, sm.coef[t & 1], st, tau, wbm, wbp, fsel, ctrl);
        }
        __syncthreads();
    }
    // outputs
    const int64_t ldi = a.ldi;
    if (nominal) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = lane + 64 * q;
            if (r < NXT) {
                if (a.xprop) a.xprop[r * ldi + k] = rs.xb[q];
                a.defect[r * ldi + k] = rs.xb[q] - sm.xk1[r];
            }
        }
        // A[:, n:] = [0; I]: the integral states feed back into nothing
        for (int e = lane; e < NXT * NY; e += 64) {
            const int r = e / NY, c = NX + e % NY;
            a.A[((int64_t)r * NXT + c) * ldi + k] = (r == c) ? T(1) : T(0);
        }
    } else if (col < NX) {
#pragma unroll
        for (int r = 0; r < NX; ++r) a.A[((int64_t)r * NXT + col) * ldi + k] = z.zb[r];
#pragma unroll
        for (int i = 0; i < NY; ++i) a.A[((int64_t)(NX + i) * NXT + col) * ldi + k] = z.zy[i];
    } else if (col < NX + 2 * M) {
        T* B = col < NX + M ? a.Bm : a.Bp;
        const int c = col < NX + M ? col - NX : col - NX - M;
#pragma unroll
        for (int r = 0; r < NX; ++r) B[((int64_t)r * M + c) * ldi + k] = z.zb[r];
#pragma unroll
        for (int i = 0; i < NY; ++i) B[((int64_t)(NX + i) * M + c) * ldi + k] = z.zy[i];
    } else if (col == NX + 2 * M) {
#pragma unroll
        for (int r = 0; r < NX; ++r) a.S[(int64_t)r * ldi + k] = z.zb[r];
#pragma unroll
        for (int i = 0; i < NY; ++i) a.S[(int64_t)(NX + i) * ldi + k] = z.zy[i];
    }
}

// ---------------------------------------------------------------------------
// K1: defects and checkpoints.  One wave per interval (the nominal wave alone).
// ---------------------------------------------------------------------------
template <class T, class TP>
__global__ void __launch_bounds__(64)
    k_defects(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    constexpr int NX = TP::NX, NXT = TP::NXT;
    __shared__ Shared<T, TP, 0> sm;
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    load_interval<T, TP>(sm, a, mc, k, lane, 64);
    RowState<T> rs;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        rs.xb[q] = r < NXT ? sm.ns[r] : T(0);
        rs.xa[q] = T(0);
    }
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
            nominal_rhs<T, TP, false>(sm, mc, lane, tau, (T*)nullptr);
            nominal_update<T, TP, false>(sm, rs, lane, st, (T*)nullptr);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NXT) {
            if (a.xprop) a.xprop[r * ldi + k] = rs.xb[q];
            a.defect[r * ldi + k] = rs.xb[q] - sm.xk1[r];
        }
    }
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

template <class T, int L, int D>
static cis_status launch_discretize(const cis_model* m, const cis_shape* sh, const void* X,
                                    const void* U, const void* s, const void* prm, void* A,
                                    void* Bm, void* Bp, void* S, void* d, void* xp,
                                    hipStream_t stream) {
    using TP = Topo<L, D>;
    auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
    FwdArgs<T> a = make_args<T>(sh, X, U, s, prm);
    a.A = (T*)A;
    a.Bm = (T*)Bm;
    a.Bp = (T*)Bp;
    a.S = (T*)S;
    a.defect = (T*)d;
    a.xprop = (T*)xp;
    void* args[] = {&a, &mc};
    hipError_t e = hipLaunchKernel((const void*)&k_discretize<T, TP>, dim3(sh->N),
                                   dim3(TP::NTHREADS), args, 0, stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_discretize launch: %s", hipGetErrorString(e));
    return CIS_OK;
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
    hipError_t e = hipLaunchKernel((const void*)&k_defects<T, TP>, dim3(sh->N), dim3(64), args,
                                   0, stream);
    if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_defects launch: %s", hipGetErrorString(e));
    return CIS_OK;
}

}  // namespace cis

using namespace cis;

extern "C" cis_status cis_discretize(const cis_model* model, const cis_shape* shape,
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

extern "C" cis_status cis_defects(const cis_model* model, const cis_shape* shape, const void* X,
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
