// Device code shared by the split forms of the discretize step (classical
// RK4 in cis_split.hip, Runge-Kutta-Fehlberg in cis_rkf.hip): the compact
// stage records and the leg-wave tangent lanes that read them (arxiv
// 2604.09993, Sec. IV-B eq. intg-aug-sys-param; sensitivities by internal
// numerical differentiation, Sec. VI).
#pragma once
#include <hip/hip_runtime.h>

#include "cis_body.hpp"
#include "cis_model.hpp"

namespace cis {

// Layout of an interval's part of the split workspace (elements of T):
//   [0, CRS)                        s, h, h/6, 0 x5, then k/I terms kc[j][4]
//   CRS + t * GLOBAL, t < R K       stage record t (CoefRec<TP> prefix), R records
//                                   per substep (4 for RK4)
template <class TP>
struct SplitRec {
    using R = CoefRec<TP>;
    static constexpr int CRS = (8 + 4 * TP::NJ + 7) / 8 * 8;
    static constexpr int GLOBAL = R::GLOBAL;
    static constexpr int64_t per_interval(int K, int R = 4) {
        return CRS + (int64_t)R * K * GLOBAL;
    }
    static constexpr int NCOLT = TP::NX + 2 * TP::M;      // tangent columns of k_tangent
    static constexpr int NBLK = (NCOLT + 63) / 64;        // column blocks of 64 lanes
    // a stage record staged in LDS by the tangent kernels: SPT elements per
    // thread of the L-wave workgroup, buffers of FBUF elements
    static constexpr int SPT = (GLOBAL + 64 * TP::L - 1) / (64 * TP::L);
    static constexpr int FBUF = SPT * 64 * TP::L;
};

// Constant entries of a compact record (joint blocks) and its zero.
template <class T, class TP>
__device__ __forceinline__ void coefrec_constants(const Interval<T, TP>& iv, T* cf, int tid,
                                                  int nth) {
    using R = CoefRec<TP>;
    const T s = iv.s;
    for (int j = tid; j < TP::NJ; j += nth) {
        const int p = TP::parent(j), c = j + 1;
        T* jb = cf + R::JB + 8 * j;
        jb[4] = s * iv.minv[p];
        jb[5] = -s * iv.minv[c];
        jb[6] = -s * iv.iinv[p];
        jb[7] = s * iv.iinv[c];
    }
    if (tid == 0) cf[R::ZERO] = T(0);
}

// ---------------------------------------------------------------------------
// k_tangent: one stage of a leg wave.  Local body lb = 0 is the torso, lb =
// 1..D the links of leg `leg`; rows z[3 lb + k] (q) and z[3 LB + 3 lb + k] (v).
// lr: the wave's leg block of the stage record; rs: the whole stage record
// (forcing entries, read per lane at offsets off[], offcc).
// ---------------------------------------------------------------------------
template <class T, class TP>
struct TanLane {
    static constexpr int LB = TP::D + 1;
    T zb[6 * LB], za[6 * LB], zs[6 * LB];
    T ycc, yct;
};

// One element of a raw buffer at byte offset `off` (offsets within the
// resource's byte range only).
template <class T>
__device__ __forceinline__ T buffer_elem(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}


// A stage record staged in LDS one stage ahead: thread t of the workgroup
// (leg wave `leg`, lane `lane`) carries elements t + 64 L e, e < SPT, of the
// record (indices clamped into the record, so every thread loads and stores
// without a branch; the buffers are padded to FBUF elements).  The forcing
// entries are read from the copy; the same loads bring the leg blocks, which
// the leg waves read with scalar loads, into the L2 cache a stage early.
template <class T, class TP>
struct StagedRec {
    T v[SplitRec<TP>::SPT];
};

template <class T, class TP>
__device__ __forceinline__ StagedRec<T, TP> stage_load(const T* rs, int leg, int lane) {
    constexpr int GL = CoefRec<TP>::GLOBAL, NT = 64 * TP::L;
    StagedRec<T, TP> r;
#pragma unroll
    for (int e = 0; e < SplitRec<TP>::SPT; ++e) {
        const int c = e * NT + leg * 64 + lane;
        r.v[e] = rs[c < GL ? c : GL - 1];
    }
    return r;
}

template <class T, class TP>
__device__ __forceinline__ void stage_store(T* lbuf, const StagedRec<T, TP>& r, int leg,
                                            int lane) {
    constexpr int NT = 64 * TP::L;
#pragma unroll
    for (int e = 0; e < SplitRec<TP>::SPT; ++e) lbuf[e * NT + leg * 64 + lane] = r.v[e];
}

// Derivative of the lane's column on its rows at the stage input zs (local
// body lb = 0 the torso, lb = 1..D the links of leg `leg`; rows zs[3 lb + k]
// (q) and zs[3 LB + 3 lb + k] (v)): kv for the velocity rows, kcc for the
// leg's cross-complementarity row and kct for the leg's part of the violation
// row (the pose rows are s zs_v).  lr: the wave's leg block of the stage
// record; rs: the whole stage record (forcing entries, read per lane at
// offsets off[], offcc).  Contains one workgroup barrier when L > 1.
//
// LDSF (L > 1 only): the forcing entries come from this stage's record
// staged in LDS (fcur, the same byte offsets as in the record), stored there
// during the previous stage; this stage loads its thread's elements of the
// next stage's record (rs_next) at its start and stores them to fnext after
// its barrier (rs_next = rs for the last stage: loaded and stored, never
// read).
template <class T, class TP, bool FORCE, bool LDSF = false>
__device__ __forceinline__ void tangent_split_rhs(const T (&zs)[6 * (TP::D + 1)],
                                                  const T* __restrict__ cr,
                                                  const T* __restrict__ lr,
                                                  const T* __restrict__ rs, T* xch, int leg,
                                                  int lane, T tau, T wbm, T wbp,
                                                  const unsigned (&off)[3 * (TP::D + 1)],
                                                  unsigned offcc, T (&kv)[3 * (TP::D + 1)],
                                                  T& kcc, T& kct, const T* fcur = nullptr,
                                                  const T* rs_next = nullptr,
                                                  T* fnext = nullptr) {
    constexpr int LB = TP::D + 1, D = TP::D, L = TP::L;
    static_assert(!LDSF || L > 1, "the LDS forcing path rides on the hip-exchange barrier");
    StagedRec<T, TP> fpre;
    if constexpr (LDSF) fpre = stage_load<T, TP>(rs_next, leg, lane);
#define ZQ(lb, k) zs[3 * (lb) + (k)]
#define ZV(lb, k) zs[3 * LB + 3 * (lb) + (k)]
    // forcing of B-/B+ columns (zero offsets and weights elsewhere): issued
    // first, used last; buffer loads at per-lane byte offsets from the stage
    // record (a scalar resource, so no per-lane 64-bit addresses)
    T g[3 * LB];
    T gcc = T(0);
    if constexpr (FORCE && !LDSF) {
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<T*>(rs), (short)0, (int)(CoefRec<TP>::GLOBAL * sizeof(T)), 0x00020000);
#pragma unroll
        for (int r = 0; r < 3 * LB; ++r) g[r] = buffer_elem<T>(rsrc, off[r]);
        gcc = buffer_elem<T>(rsrc, offcc);
    }
    // hip stiffness and damping of this leg on the torso, exchanged
    const T* kcl = cr + 8 + 4 * leg * D;   // kc[j][4] of the leg's joints
    T hip = kcl[0] * (ZQ(1, 2) - ZQ(0, 2)) + kcl[1] * (ZV(1, 2) - ZV(0, 2));
    if constexpr (L > 1) {
        xch[leg * 64 + lane] = hip;
        __syncthreads();
        // every wave has passed its reads of the previous stage's region,
        // which the next stage's region replaces
        if constexpr (LDSF) stage_store<T, TP>(fnext, fpre, leg, lane);
        hip = xch[lane];
#pragma unroll
        for (int l = 1; l < L; ++l) hip += xch[l * 64 + lane];
    }
    kv[0] = T(0);
    kv[1] = T(0);
    kv[2] = lr[0] * ZQ(0, 2) + hip;
#pragma unroll
    for (int lb = 1; lb <= D; ++lb) {
        kv[3 * lb] = T(0);
        kv[3 * lb + 1] = T(0);
        kv[3 * lb + 2] = lr[lb] * ZQ(lb, 2);
    }
    kct = T(0);
#pragma unroll
    for (int lb = 1; lb <= D; ++lb) {
        const T* kc = kcl + 4 * (lb - 1);
        const T dth = ZQ(lb, 2) - ZQ(lb - 1, 2);
        const T dom = ZV(lb, 2) - ZV(lb - 1, 2);
        if (lb >= 2) kv[3 * (lb - 1) + 2] += kc[0] * dth + kc[1] * dom;
        kv[3 * lb + 2] -= kc[2] * dth + kc[3] * dom;
        const T* jh = lr + 1 + D + 4 * (lb - 1);
        kct += jh[0] * (ZQ(lb - 1, 0) - ZQ(lb, 0)) + jh[1] * (ZQ(lb - 1, 1) - ZQ(lb, 1)) +
               jh[2] * ZQ(lb - 1, 2) + jh[3] * ZQ(lb, 2);
    }
    {
        const T* ct = lr + 1 + 5 * D;   // contact terms C_AX .. C_ZPY of the leg's contact
        constexpr int lb = D;
        const T dPx = ZQ(lb, 0) - ct[C_AY] * ZQ(lb, 2);
        const T dPy = ZQ(lb, 1) + ct[C_AX] * ZQ(lb, 2);
        kv[3 * lb] += ct[C_FXP] * dPx;
        kv[3 * lb + 1] += ct[C_FYP] * dPx;
        kv[3 * lb + 2] += ct[C_TP] * dPx;
        kcc = ct[C_EPX] * dPx + ct[C_EPY] * dPy + ct[C_EXD] * ZV(lb, 0) + ct[C_EYD] * ZV(lb, 1) +
              ct[C_EOM] * ZV(lb, 2) + ct[C_ETH] * ZQ(lb, 2);
        kct += ct[C_ZPX] * dPx + ct[C_ZPY] * dPy;
    }
    if constexpr (FORCE && LDSF) {
        // read where used (after this stage's barrier)
        const char* fb = (const char*)fcur;
#pragma unroll
        for (int r = 0; r < 3 * LB; ++r) g[r] = *(const T*)(fb + off[r]);
        gcc = *(const T*)(fb + offcc);
    }
    if constexpr (FORCE) {
        const T wB = wbm * (T(1) - tau) + wbp * tau;
#pragma unroll
        for (int r = 0; r < 3 * LB; ++r) kv[r] += wB * g[r];
        kcc += (wbm + wbp) * gcc;
    }
#undef ZQ
#undef ZV
}

// Record offset of the forcing entry of control `ctrl` in row k (0: x, 1: y,
// 2: theta) of body gb, or the zero entry (Sec. IV-B FOH: dF~/du of the
// joint torques, joint forces and contact forces).
template <class TP>
__device__ __forceinline__ int forcing_offset(int ctrl, int gb, int k) {
    using R = CoefRec<TP>;
    constexpr int NJ = TP::NJ;
    if (ctrl < NJ) {
        const int j = ctrl, p = TP::parent(j), c = j + 1;
        if (k == 2 && gb == p) return R::JB + 8 * j + 6;
        if (k == 2 && gb == c) return R::JB + 8 * j + 7;
        return R::ZERO;
    }
    if (ctrl < 3 * NJ) {
        const int j = (ctrl - NJ) >> 1, ax = (ctrl - NJ) & 1, p = TP::parent(j), c = j + 1;
        if (k == ax && gb == p) return R::JB + 8 * j + 4;
        if (k == ax && gb == c) return R::JB + 8 * j + 5;
        if (k == 2 && gb == p) return R::JB + 8 * j + ax;
        if (k == 2 && gb == c) return R::JB + 8 * j + 2 + ax;
        return R::ZERO;
    }
    const int i = (ctrl - 3 * NJ) / 3, q = (ctrl - 3 * NJ) % 3;
    return gb == TP::cbody(i) ? R::CB + 12 * i + 3 * k + q : R::ZERO;
}

// The lane's column of a block of 64 tangent columns: its index, the FOH
// weights of a B- / B+ column (zero elsewhere), the record byte offsets of
// its forcing entries (the zero entry elsewhere), and its initial value on
// the lane's rows (a unit column of Phi_x, else zero).
template <class TP>
struct TanCol {
    int col;
    bool active;
    unsigned off[3 * (TP::D + 1)];
    unsigned offcc;
};

template <class T, class TP>
__device__ __forceinline__ TanCol<TP> tangent_column(int cb, int leg, int lane, T& wbm, T& wbp,
                                                     T (&z0)[6 * (TP::D + 1)]) {
    constexpr int NX = TP::NX, NQ = TP::NQ, M = TP::M, D = TP::D, LB = D + 1;
    using SR = SplitRec<TP>;
    TanCol<TP> tc;
    const int col = cb * 64 + lane;
    tc.col = col;
    tc.active = col < SR::NCOLT;
    auto gbody = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
    wbm = T(0);
    wbp = T(0);
    int ctrl = 0;
    if (col >= NX && col < NX + M) { wbm = T(1); ctrl = col - NX; }
    else if (col >= NX + M && col < NX + 2 * M) { wbp = T(1); ctrl = col - NX - M; }
    const bool bcol = wbm != T(0) || wbp != T(0);
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
            tc.off[3 * lb + kk] = sizeof(T) * (unsigned)(bcol ? forcing_offset<TP>(ctrl, gbody(lb), kk)
                                                              : CoefRec<TP>::ZERO);
    tc.offcc = sizeof(T) * (unsigned)CoefRec<TP>::ZERO;
    if (bcol && ctrl >= 3 * TP::NJ && (ctrl - 3 * TP::NJ) / 3 == leg)
        tc.offcc = sizeof(T) * (unsigned)CoefRec<TP>::gc(leg, (ctrl - 3 * TP::NJ) % 3);
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const int gq = 3 * gbody(lb) + kk;
            z0[3 * lb + kk] = (gq == col) ? T(1) : T(0);
            z0[3 * LB + 3 * lb + kk] = (NQ + gq == col) ? T(1) : T(0);
        }
    return tc;
}

// Stores of the lane's column of interval k (rows of the torso from leg 0
// only): z on the lane's rows, the leg's cross-complementarity row ycc, and
// the violation row summed over the legs in leg order (contains workgroup
// barriers when L > 1: every wave of the block calls it).
template <class T, class TP>
__device__ __forceinline__ void tangent_store(const FwdArgs<T>& a, int k, int leg, int lane,
                                              const TanCol<TP>& tc,
                                              const T (&z)[6 * (TP::D + 1)], T ycc, T yct,
                                              T* xch) {
    constexpr int NX = TP::NX, NXT = TP::NXT, NQ = TP::NQ, M = TP::M, NC = TP::NC;
    constexpr int D = TP::D, L = TP::L, LB = D + 1;
    auto gbody = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
    if constexpr (L > 1) {
        __syncthreads();
        xch[leg * 64 + lane] = yct;
        __syncthreads();
        yct = xch[lane];
#pragma unroll
        for (int l = 1; l < L; ++l) yct += xch[l * 64 + lane];
    }
    if (!tc.active) return;
    const int col = tc.col;
    const int64_t ldi = a.ldi;
    T* out;
    int64_t cstride, c0;   // element (row, column) at out[(row * cstride + c0) * ldi + k]
    if (col < NX) { out = a.A; cstride = NXT; c0 = col; }
    else if (col < NX + M) { out = a.Bm; cstride = M; c0 = col - NX; }
    else { out = a.Bp; cstride = M; c0 = col - NX - M; }
#pragma unroll
    for (int lb = 0; lb < LB; ++lb) {
        if (lb == 0 && leg != 0) continue;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            const int gq = 3 * gbody(lb) + kk;
            out[((int64_t)gq * cstride + c0) * ldi + k] = z[3 * lb + kk];
            out[((int64_t)(NQ + gq) * cstride + c0) * ldi + k] = z[3 * LB + 3 * lb + kk];
        }
    }
    out[((int64_t)(NX + leg) * cstride + c0) * ldi + k] = ycc;
    if (leg == 0) out[((int64_t)(NX + NC) * cstride + c0) * ldi + k] = yct;
}

}  // namespace cis
