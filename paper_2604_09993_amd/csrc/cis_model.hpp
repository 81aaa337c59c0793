// Planar maximal-coordinate model evaluated on gfx950 (arxiv 2604.09993).
//
// Compile-time topology: a torso (body 0) with L legs of D rod links each.
// Joint j joins parent(j) to child j+1; the contact of leg l sits at the tip
// of that leg's last link (on the torso when D = 0).  Geometry, stiffness,
// damping, gravity and terrain are run-time constants passed by value in the
// kernel argument segment; masses and the friction coefficient are run-time
// device inputs (they are differentiated).
//
// Right-hand side of the time-dilated augmented system (Sec. IV-B) in three
// element-parallel steps executed by one wave: one lane per body for the
// rotations, one lane per joint or contact for forces and integrands, one
// lane per body for the Newton-Euler sums.  Three depths:
//   LEAN : accelerations only (what the state recursion needs),
//   FULL : + cross-complementarity and violation integrands,
//   EMIT : + every nonzero of dF~/dx, dF~/du, dF~/dubar at the stage, written
//          into a coefficient buffer read by the tangent lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "cis_host.hpp"

namespace cis {

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int even(int a) { return (a + 1) & ~1; }

template <int L_, int D_, int TW_MAX_ = 6, int NCW_ = 1, bool SEPS_ = (NCW_ == 2)>
struct Topo {
    static constexpr int L = L_, D = D_;
    static constexpr int NB = 1 + L * D, NJ = L * D, NC = L;
    static constexpr int NQ = 3 * NB, NX = 6 * NB, NY = NC + 1, NXT = NX + NY;
    static constexpr int M = 3 * NJ + 3 * NC, P = NB + 2;
    static constexpr int NCOL = NX + 2 * M + 1;   // tangent columns [Phi_x | B- | B+ | S]
    static constexpr int G = L > 1 ? L : 1;       // lanes per tangent column (one per leg)
    static constexpr int LB = D + 1;              // bodies held by one tangent lane
    // SEP_S (by default with two coefficient waves, the latency layout): the
    // dilation column S has a column group of its own, integrated on body
    // lanes by one wave, so the leg-lane tangent waves carry no F~ forcing.
    static constexpr bool SEP_S = SEPS_;
    static_assert(!SEPS_ || NCW_ == 2, "the S group is laid out with two coefficient waves");
    static constexpr int NCOLT = NCOL - (SEP_S ? 1 : 0);   // columns on leg lanes
    static constexpr int NTW_ALL = (NCOLT * G + 63) / 64;  // leg-lane tangent waves per interval
    // columns are split over NGRPT workgroups of at most TW_MAX_ tangent waves
    // (TW_MAX_ = 6: two waves per SIMD, 256 VGPRs each; TW_MAX_ = 2: one wave
    // per SIMD and 512 registers, for the FP64 columns)
    static constexpr int NGRPT = (NTW_ALL + TW_MAX_ - 1) / TW_MAX_;
    static constexpr int NGRP = NGRPT + (SEP_S ? 1 : 0);    // + the S group
    static constexpr int NTW = (NTW_ALL + NGRPT - 1) / NGRPT;  // tangent waves per workgroup
    static constexpr int CPG = NTW * 64 / G;                  // columns per workgroup
    // coefficient waves: with NCW_ = 2 two waves take alternate stages, each
    // stage spread over two pipeline steps
    static constexpr int NCW = NCW_;
    static constexpr int NCOEF = NCW == 1 ? 2 : 4;            // coefficient buffers in flight
    static constexpr int LAG = NCW + 1;                       // steps from state to tangent
    static constexpr int NTHREADS = 64 * (NTW + 1 + NCW);     // + state wave + coefficient waves
    static_assert(NCW == 1 || NCW == 2, "one or two coefficient waves");
    static_assert(NXT <= 128, "state rows are owned two per lane");
    static_assert(NB < 64 && NJ + NC <= 64, "one lane per body / element");
    static_assert(G == 1 || G == 2 || G == 4, "legs must map onto a DPP quad");
    static_assert(NTHREADS <= 512, "at most 8 waves per workgroup");
    __host__ __device__ static constexpr int parent(int j) {
        return D == 0 ? 0 : ((j % D == 0) ? 0 : j);
    }
    __host__ __device__ static constexpr int cbody(int i) { return D * (i + 1); }
};

// Geometry and constants of a model (host fills it, passed by value).
template <int NB, int NJ, int NC>
struct MConst {
    double ipm[NB];                 // rod inertia per unit mass, L^2 / 12
    double rp[cmax(NJ, 1)][2];      // joint anchors, parent frame
    double rc[cmax(NJ, 1)][2];      // joint anchors, child frame
    double ks[cmax(NJ, 1)];         // joint stiffness
    double ds[cmax(NJ, 1)];         // joint damping
    double cr[cmax(NC, 1)][2];      // contact points, body frame
    double g, A, kappa;             // gravity, terrain amplitude, wavenumber
};

// Layout of one per-stage coefficient buffer (LDS), in elements.
template <class TP>
struct Coef {
    static constexpr int NCT = 14;                     // per-contact terms
    static constexpr int CTH = 0;                      // [NB] s dT_b/dth_b / I_b
    static constexpr int JH = even(TP::NB);            // [NJ][4] violation row, joints
    static constexpr int CT = JH + 4 * TP::NJ;         // [NC][NCT] contact terms
    static constexpr int GV = CT + NCT * TP::NC;       // [3NB][M] s dv'/du
    static constexpr int GC = GV + 3 * TP::NB * TP::M; // [NC][M] (s/2) dOmega_cc/dubar
    static constexpr int F = GC + TP::NC * TP::M;      // [NXT] F~ (unscaled; the violation row unused)
    static constexpr int CTP = F + TP::NXT;            // [NB] violation integrand, per body
    // per-lane sink for stores of lanes without the datum: lane l stores at
    // TRASH + l + o with o < 16 (offsets within the contact block)
    static constexpr int TRASH = even(CTP + TP::NB);
    static constexpr int SIZE = TRASH + 64 + 16;
};
// per-contact slots (C_JMU = s lbar_n |v_t|_s = d(s Omega_cc)/d mu)
enum { C_AX = 0, C_AY, C_FXP, C_FYP, C_TP, C_EPX, C_EPY, C_EXD, C_EYD, C_EOM, C_ETH, C_ZPX, C_ZPY,
       C_JMU };

// Where a stage's coefficients sit in a coefficient buffer, as offsets
// (element units).  Dense: the Coef<TP> layout above, read in place by the
// leg-lane tangent waves and the reverse sweep.
template <class TP>
struct CoefDense {
    using C = Coef<TP>;
    static constexpr int SIZE = C::SIZE, TRASH = C::TRASH;
    // dT_b/dth_b; `copy` < L selects one of the copies of the torso entry
    // (the dense layout has one)
    __device__ static constexpr int cth(int b, int copy = 0) { return C::CTH + b + 0 * copy; }
    static constexpr int TORSO_COPIES = 1;
    __device__ static constexpr int jh(int j, int q) { return C::JH + 4 * j + q; }
    __device__ static constexpr int ct(int i, int q) { return C::CT + C::NCT * i + q; }
    // theta row of the parent (side 0, body p) or child (side 1, body c) of
    // joint j, column of its force component ax
    __device__ static constexpr int gv_joint(int j, int side, int p, int c, int ax) {
        return C::GV + (3 * (side ? c : p) + 2) * TP::M + TP::NJ + 2 * j + ax;
    }
    // row r (0: x, 1: y, 2: theta) of contact body b, column of control q of contact i
    __device__ static constexpr int gv_contact(int i, int b, int r, int q) {
        return C::GV + (3 * b + r) * TP::M + 3 * TP::NJ + 3 * i + q;
    }
    __device__ static constexpr int gc(int i, int q) {
        return C::GC + i * TP::M + 3 * TP::NJ + 3 * i + q;
    }
    __device__ static constexpr int f(int r) { return C::F + r; }
    __device__ static constexpr int ctp(int b) { return C::CTP + b; }
};

// Compact stage record of the split discretize form (legs with links only).
// The first GLOBAL elements are what the tangent kernel reads, copied to
// device memory once per stage; F~ and the violation parts (used by the
// dilation column only) follow, then the per-lane sinks.
//   leg block l (LEGB elements, a multiple of 8 so each block starts on a
//   64-byte boundary): [0] dT/dth of the torso (one copy per leg),
//   [1 + d] dT/dth of link d of the leg, [1 + D + 4 d + q] violation-row
//   coefficients of joint l D + d, [1 + 5 D + q] the 13 contact terms C_AX..C_ZPY
//   of contact l;
//   joint block j (8): theta-row forcing of the parent and child for the
//   force components x, y: [th_p x, th_p y, th_c x, th_c y], then the
//   constant entries [s/m_p, -s/m_c, -s/I_p, s/I_c];
//   contact block i (12): x, y, theta rows of the contact body for
//   lambda_n, lambda_t+, lambda_t- ([3 r + q]), then the three
//   cross-complementarity entries (s/2) dOmega_cc/dubar;
//   one zero.
template <class TP>
struct CoefRec {
    static_assert(TP::L >= 1 && TP::D >= 1, "the compact record needs legs with links");
    static constexpr int L = TP::L, D = TP::D, NJ = TP::NJ, NC = TP::NC;
    static constexpr int LEGB = (5 * D + 14 + 7) / 8 * 8;
    static constexpr int JB = L * LEGB;                 // joint blocks
    static constexpr int CB = JB + 8 * NJ;              // contact blocks
    static constexpr int ZERO = CB + 12 * NC;
    static constexpr int GLOBAL = (ZERO + 1 + 7) / 8 * 8;   // elements copied per stage
    static constexpr int F = GLOBAL;                    // [NXT] F~
    static constexpr int CTP = F + TP::NXT;             // [NB] violation parts
    static constexpr int TRASH = (CTP + TP::NB + 1) / 2 * 2;
    static constexpr int SIZE = TRASH + 64 + 16;
    static constexpr int TORSO_COPIES = L;
    __device__ static constexpr int cth(int b, int copy = 0) {
        return b == 0 ? copy * LEGB : ((b - 1) / D) * LEGB + 1 + (b - 1) % D;
    }
    __device__ static constexpr int jh(int j, int q) {
        return (j / D) * LEGB + 1 + D + 4 * (j % D) + q;
    }
    __device__ static constexpr int ct(int i, int q) {
        // C_JMU (the friction-coefficient derivative) is not kept
        return q < 13 ? i * LEGB + 1 + 5 * D + q : TRASH + 15;
    }
    __device__ static constexpr int gv_joint(int j, int side, int, int, int ax) {
        return JB + 8 * j + 2 * side + ax;
    }
    __device__ static constexpr int gv_contact(int i, int, int r, int q) {
        return CB + 12 * i + 3 * r + q;
    }
    __device__ static constexpr int gc(int i, int q) { return CB + 12 * i + 9 + q; }
    __device__ static constexpr int f(int r) { return F + r; }
    __device__ static constexpr int ctp(int b) { return CTP + b; }
};

// Per-interval data shared by every role.
template <class T, class TP>
struct Interval {
    T kc[cmax(TP::NJ, 1)][4];                  // s k/I_p, s d/I_p, s k/I_c, s d/I_c
    T uk[cmax(TP::M, 1)], uk1[cmax(TP::M, 1)]; // FOH coefficients U_k, U_k+1
    T x0[TP::NXT];                             // X_k
    T xk1[TP::NXT];                            // X_{k+1}
    T prm[TP::P];                              // (mu, e, masses)
    T minv[TP::NB], iinv[TP::NB];              // 1/m_b, 1/I_b
    T s, h, h6;                                // dilation, RK4 step 1/K, h/6
};

// Scratch of one right-hand-side evaluation (one per concurrently evaluating wave).
template <class T, class TP>
struct RhsScratch {
    T ns[TP::NXT];                             // evaluation point (x part used)
    T fn[TP::NXT];                             // F~ rows v, y (q rows are ns[v])
    T cs[TP::NB][2];                           // cos, sin of body angles
    T slot[cmax(2 * TP::NJ + TP::NC, 1)][4];   // (Fx, Fy, T, dT/dth) per element end
    T ctp[cmax(TP::NJ + TP::NC, 1)];           // violation integrand parts
};

// LDS ordering between lanes of one wave (a wave's LDS instructions execute
// in order; the fences keep the compiler from moving loads and stores across
// the point and drain outstanding LDS traffic).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double sqrt_t(double a) { return sqrt(a); }
__device__ __forceinline__ float sqrt_t(float a) { return sqrtf(a); }

// sin and cos without branches (two evaluations interleave): Cody-Waite
// reduction r = a - k pi/2 with pi/2 split in three parts (the leading two
// with 30 significant bits, so k P1 and k P2 are exact for |k| < 2^23; pi
// from Machin's formula), then the Taylor series of sin and cos on
// [-pi/4, pi/4] through r^17 and r^18 (truncation below 1e-19), and the
// quadrant of k.  Arguments beyond 1e5 in any lane take the library routine.
__device__ __forceinline__ void sincos_cw(double a, double& sa, double& ca) {
    const double k = rint(a * 0.6366197723675814);
    double r = fma(-k, 1.570796325802803, a);
    r = fma(-k, 9.920935791635221e-10, r);
    r = fma(-k, 5.170182981794105e-19, r);
    const double z = r * r;
    double ps = 1.0 / 355687428096000.0;             // 1/17!
    ps = fma(ps, z, -1.0 / 1307674368000.0);         // 1/15!
    ps = fma(ps, z, 1.0 / 6227020800.0);             // 1/13!
    ps = fma(ps, z, -1.0 / 39916800.0);              // 1/11!
    ps = fma(ps, z, 1.0 / 362880.0);                 // 1/9!
    ps = fma(ps, z, -1.0 / 5040.0);                  // 1/7!
    ps = fma(ps, z, 1.0 / 120.0);                    // 1/5!
    ps = fma(ps, z, -1.0 / 6.0);                     // 1/3!
    double pc = -1.0 / 6402373705728000.0;           // 1/18!
    pc = fma(pc, z, 1.0 / 20922789888000.0);         // 1/16!
    pc = fma(pc, z, -1.0 / 87178291200.0);           // 1/14!
    pc = fma(pc, z, 1.0 / 479001600.0);              // 1/12!
    pc = fma(pc, z, -1.0 / 3628800.0);               // 1/10!
    pc = fma(pc, z, 1.0 / 40320.0);                  // 1/8!
    pc = fma(pc, z, -1.0 / 720.0);                   // 1/6!
    pc = fma(pc, z, 1.0 / 24.0);                     // 1/4!
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z * z, pc, fma(-0.5, z, 1.0));
    const int q = (int)k;
    const double s1 = (q & 1) ? cr : sr;
    const double c1 = (q & 1) ? sr : cr;
    sa = (q & 2) ? -s1 : s1;
    ca = ((q + 1) & 2) ? -c1 : c1;
}
__device__ __forceinline__ void sincos_t(double a, double* s, double* c) {
    if (__any(fabs(a) > 1e5)) {
        sincos(a, s, c);
    } else {
        sincos_cw(a, *s, *c);
    }
}
__device__ __forceinline__ void sincos_t(float a, float* s, float* c) { sincosf(a, s, c); }

// Pseudo-Huber absolute value with unit steepness (Sec. II notation):
// |a|_s = sqrt(a^2+1) - 1 = a^2 y/(1 + y) with y = 1/sqrt(a^2+1), and its
// slope a y.  y and 1/(1+y) start from the hardware reciprocal (square root)
// estimates and take two Newton steps each (w >= 1, 1 + y in [1, 2]).
__device__ __forceinline__ void sabs_d(double a, double& val, double& der) {
    const double w = fma(a, a, 1.0);
    double y = __builtin_amdgcn_rsq(w);
    double hw = 0.5 * w;
    y = y * fma(-hw * y, y, 1.5);
    y = y * fma(-hw * y, y, 1.5);
    const double d = 1.0 + y;
    double q = __builtin_amdgcn_rcp(d);
    q = q * fma(-d, q, 2.0);
    q = q * fma(-d, q, 2.0);
    der = a * y;
    val = (a * a) * (y * q);
}
// FP32: the same form with the hardware reciprocal square root and
// reciprocal (about 1 ulp each, far inside the FP32 tolerance).
__device__ __forceinline__ void sabs_d(float a, float& val, float& der) {
    const float y = __builtin_amdgcn_rsqf(fmaf(a, a, 1.0f));
    const float q = __builtin_amdgcn_rcpf(1.0f + y);
    der = a * y;
    val = (a * a) * (y * q);
}

enum RhsMode { LEAN = 0, FULL = 1, EMIT = 2 };

// ---------------------------------------------------------------------------
// One right-hand-side evaluation at sc.ns by the 64 lanes of one wave.
// If HAVE_CS the rotations sc.cs are already filled in.  Writes sc.fn (v rows
// always, y rows from FULL on) and, in EMIT mode, the coefficients into cf.
// SPLIT: one workgroup barrier between the element wrenches and the smooth
// functions, so that the evaluation spans two steps of a barrier pipeline.
// ---------------------------------------------------------------------------
template <class T, class TP, int MODE, bool HAVE_CS = false, bool SPLIT = false>
__device__ __forceinline__ void rhs_eval(const Interval<T, TP>& iv, RhsScratch<T, TP>& sc,
                                         const MConst<TP::NB, TP::NJ, TP::NC>& mc, int lane,
                                         T tau, T* cf) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, NX = TP::NX, M = TP::M;
    using C = Coef<TP>;
    const T s = iv.s;
    const T omt = T(1) - tau;
    if (!HAVE_CS) {
        if (lane < NB) {
            T sn, cn;
            sincos_t(sc.ns[3 * lane + 2], &sn, &cn);
            sc.cs[lane][0] = cn;
            sc.cs[lane][1] = sn;
        }
        wave_lds_sync();
    }
    const bool flat = mc.A == 0.0;
    // step 2a: element arguments and wrenches (cheap, divergent)
    T sa0 = T(0), sa1 = T(0);          // smooth-function arguments of this element
    T apx = T(0), apy = T(0), acx = T(0), acy = T(0);   // joint arms
    T ax = T(0), ay = T(0), om = T(0), sd = T(0), tx = T(1), ty = T(0), nx = T(0), ny = T(1);
    T dsd_px = T(0), dsd_py = T(1), dnx = T(0), dny = T(0), ln = T(0), ft = T(0);
    T lnb = T(0), ltpb = T(0), ltmb = T(0), vt = T(0), Pdx = T(0), Pdy = T(0);
    if (lane < NJ) {
        const int j = lane;
        const int p = TP::parent(j), c = j + 1;
        const T cp = sc.cs[p][0], sp = sc.cs[p][1], cc = sc.cs[c][0], scc = sc.cs[c][1];
        const T rpx = T(mc.rp[j][0]), rpy = T(mc.rp[j][1]);
        const T rcx = T(mc.rc[j][0]), rcy = T(mc.rc[j][1]);
        apx = cp * rpx - sp * rpy;
        apy = sp * rpx + cp * rpy;
        acx = cc * rcx - scc * rcy;
        acy = scc * rcx + cc * rcy;
        const T lx = omt * iv.uk[NJ + 2 * j] + tau * iv.uk1[NJ + 2 * j];
        const T ly = omt * iv.uk[NJ + 2 * j + 1] + tau * iv.uk1[NJ + 2 * j + 1];
        const T tq = omt * iv.uk[j] + tau * iv.uk1[j];
        const T k = T(mc.ks[j]), d = T(mc.ds[j]);
        const T tsd = -k * (sc.ns[3 * c + 2] - sc.ns[3 * p + 2]) -
                      d * (sc.ns[NQ + 3 * c + 2] - sc.ns[NQ + 3 * p + 2]);
        const T tt = tq + tsd;
        sc.slot[2 * j][0] = lx;
        sc.slot[2 * j][1] = ly;
        sc.slot[2 * j][2] = (apx * ly - apy * lx) - tt;
        sc.slot[2 * j][3] = -(apx * lx + apy * ly);
        sc.slot[2 * j + 1][0] = -lx;
        sc.slot[2 * j + 1][1] = -ly;
        sc.slot[2 * j + 1][2] = -(acx * ly - acy * lx) + tt;
        sc.slot[2 * j + 1][3] = acx * lx + acy * ly;
        if (MODE >= FULL) {
            sa0 = sc.ns[3 * p] + apx - sc.ns[3 * c] - acx;          // h_x
            sa1 = sc.ns[3 * p + 1] + apy - sc.ns[3 * c + 1] - acy;  // h_y
        }
    } else if (lane < NJ + NC) {
        const int i = lane - NJ;
        const int b = TP::cbody(i);
        const T cn = sc.cs[b][0], sn = sc.cs[b][1];
        const T rx = T(mc.cr[i][0]), ry = T(mc.cr[i][1]);
        ax = cn * rx - sn * ry;
        ay = sn * rx + cn * ry;
        const T Px = sc.ns[3 * b] + ax, Py = sc.ns[3 * b + 1] + ay;
        om = sc.ns[NQ + 3 * b + 2];
        Pdx = sc.ns[NQ + 3 * b] - om * ay;
        Pdy = sc.ns[NQ + 3 * b + 1] + om * ax;
        if (flat) {
            sd = Py;   // h = P_y, n = (0, 1), t = (1, 0)
        } else {
            // terrain frame at P (Sec. II contact frame; Sec. VI-B sd = h/||grad h||)
            const T A = T(mc.A), kap = T(mc.kappa);
            T sw, cw;
            sincos_t(kap * Px, &sw, &cw);
            const T H = Py - A * sw;
            const T Hx = -A * kap * cw;
            const T Hxx = A * kap * kap * sw;
            const T G = sqrt_t(T(1) + Hx * Hx);
            const T rG = T(1) / G;
            const T rG3 = rG * rG * rG;
            sd = H * rG;
            nx = Hx * rG;
            ny = rG;
            tx = ny;
            ty = -nx;
            dsd_px = Hx * rG - H * Hx * Hxx * rG3;
            dsd_py = rG;
            dnx = Hxx * rG3;
            dny = -Hx * Hxx * rG3;
        }
        const int u0 = 3 * NJ + 3 * i;
        ln = omt * iv.uk[u0] + tau * iv.uk1[u0];
        const T ltp = omt * iv.uk[u0 + 1] + tau * iv.uk1[u0 + 1];
        const T ltm = omt * iv.uk[u0 + 2] + tau * iv.uk1[u0 + 2];
        ft = ltp - ltm;
        const T fx = tx * ft + nx * ln, fy = ty * ft + ny * ln;
        sc.slot[2 * NJ + i][0] = fx;
        sc.slot[2 * NJ + i][1] = fy;
        sc.slot[2 * NJ + i][2] = ax * fy - ay * fx;
        sc.slot[2 * NJ + i][3] = -(ax * fx + ay * fy);
        if (MODE >= FULL) {
            lnb = T(0.5) * (iv.uk[u0] + iv.uk1[u0]);
            ltpb = T(0.5) * (iv.uk[u0 + 1] + iv.uk1[u0 + 1]);
            ltmb = T(0.5) * (iv.uk[u0 + 2] + iv.uk1[u0 + 2]);
            vt = tx * Pdx + ty * Pdy;
            sa0 = vt;
            sa1 = -sd;
        }
    }
    if constexpr (SPLIT) __syncthreads();
    if (MODE >= FULL && NJ + NC > 0) {
        // step 2b: smooth functions, one code path for joints and contacts
        T v0, d0, v1, d1;
        sabs_d(sa0, v0, d0);
        sabs_d(sa1, v1, d1);
        if (lane < NJ) {
            const int j = lane;
            const int p = TP::parent(j), c = j + 1;
            sc.ctp[j] = v0 + v1;   // |h_x|_s + |h_y|_s
            if (MODE == EMIT) {
                cf[C::JH + 4 * j + 0] = s * d0;
                cf[C::JH + 4 * j + 1] = s * d1;
                cf[C::JH + 4 * j + 2] = s * (d1 * apx - d0 * apy);
                cf[C::JH + 4 * j + 3] = s * (d0 * acy - d1 * acx);
                const T ip = s * iv.iinv[p], ic = s * iv.iinv[c];
                cf[C::GV + (3 * p + 2) * M + NJ + 2 * j] = -apy * ip;
                cf[C::GV + (3 * p + 2) * M + NJ + 2 * j + 1] = apx * ip;
                cf[C::GV + (3 * c + 2) * M + NJ + 2 * j] = acy * ic;
                cf[C::GV + (3 * c + 2) * M + NJ + 2 * j + 1] = -acx * ic;
            }
        } else if (lane < NJ + NC) {
            const int i = lane - NJ;
            const int b = TP::cbody(i);
            const T av = v0, dav = d0;                   // |v_t|_s and its slope
            const T rp = vt > T(0) ? av : T(0);          // ramp_s(v_t)
            const T rm = vt < T(0) ? av : T(0);          // ramp_s(-v_t)
            const T mu = iv.prm[0];
            const T slack = mu * lnb - ltpb - ltmb;
            // integral cross-complementarity integrand (pairs of Sec. III)
            sc.fn[NX + i] = lnb * sd + ltpb * rp + ltmb * rm + slack * av;
            sc.ctp[NJ + i] = -sd > T(0) ? v1 : T(0);     // ramp_s(-sd)
            if (MODE == EMIT) {
                const T gv = ltpb * (vt > T(0) ? dav : T(0)) + ltmb * (vt < T(0) ? dav : T(0)) +
                             slack * dav;
                const T Dg = -(-sd > T(0) ? d1 : T(0));
                const T dtx = dny, dty = -dnx;
                const T dfx = dtx * ft + dnx * ln, dfy = dty * ft + dny * ln;
                const T dvt_px = dtx * Pdx + dty * Pdy;
                const T im = s * iv.minv[b], ii = s * iv.iinv[b];
                T* ct = cf + C::CT + C::NCT * i;
                ct[C_AX] = ax;
                ct[C_AY] = ay;
                ct[C_FXP] = dfx * im;
                ct[C_FYP] = dfy * im;
                ct[C_TP] = (ax * dfy - ay * dfx) * ii;
                ct[C_EPX] = s * (lnb * dsd_px + gv * dvt_px);
                ct[C_EPY] = s * (lnb * dsd_py);
                ct[C_EXD] = s * (gv * tx);
                ct[C_EYD] = s * (gv * ty);
                ct[C_EOM] = s * (gv * (ty * ax - tx * ay));
                ct[C_ETH] = s * (-gv * om * (tx * ax + ty * ay));
                ct[C_ZPX] = s * (Dg * dsd_px);
                ct[C_ZPY] = s * (Dg * dsd_py);
                ct[C_JMU] = s * (lnb * av);
                const int u0 = 3 * NJ + 3 * i;
                T* gvb = cf + C::GV;
                gvb[(3 * b) * M + u0] = nx * im;
                gvb[(3 * b + 1) * M + u0] = ny * im;
                gvb[(3 * b + 2) * M + u0] = (ax * ny - ay * nx) * ii;
                gvb[(3 * b) * M + u0 + 1] = tx * im;
                gvb[(3 * b + 1) * M + u0 + 1] = ty * im;
                gvb[(3 * b + 2) * M + u0 + 1] = (ax * ty - ay * tx) * ii;
                gvb[(3 * b) * M + u0 + 2] = -tx * im;
                gvb[(3 * b + 1) * M + u0 + 2] = -ty * im;
                gvb[(3 * b + 2) * M + u0 + 2] = -(ax * ty - ay * tx) * ii;
                T* gcb = cf + C::GC + i * M;
                gcb[u0] = s * T(0.5) * (sd + mu * av);
                gcb[u0 + 1] = s * T(0.5) * (rp - av);
                gcb[u0 + 2] = s * T(0.5) * (rm - av);
            }
        }
    }
    wave_lds_sync();
    // step 3: Newton-Euler sums per body; violation sum on lane NB
    if (lane < NB) {
        const int b = lane;
        T Fx = T(0), Fy = T(0), Tq = T(0), dT = T(0);
        auto add = [&](int sl) {
            Fx += sc.slot[sl][0];
            Fy += sc.slot[sl][1];
            Tq += sc.slot[sl][2];
            dT += sc.slot[sl][3];
        };
        if (b == 0) {
#pragma unroll
            for (int l = 0; l < TP::L; ++l) {
                if (TP::D > 0) add(2 * (l * TP::D));
                else add(2 * NJ + l);
            }
        } else if constexpr (TP::D > 0) {
            add(2 * (b - 1) + 1);
            if (b % TP::D != 0) add(2 * b);
            else add(2 * NJ + b / TP::D - 1);
        }
        const T mi = iv.minv[b], ii = iv.iinv[b];
        sc.fn[NQ + 3 * b] = Fx * mi;
        sc.fn[NQ + 3 * b + 1] = Fy * mi - T(mc.g);
        sc.fn[NQ + 3 * b + 2] = Tq * ii;
        if (MODE == EMIT) cf[C::CTH + b] = s * dT * ii;
    } else if (MODE >= FULL && lane == NB) {
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < NJ + NC; ++e) acc += sc.ctp[e];
        sc.fn[NX + NC] = acc;
    }
    wave_lds_sync();
}

// Nominal RK4 row state of one lane: rows r = lane and lane + 64.
template <class T>
struct RowState {
    T xb[2], xa[2];
};

// RK4 update after evaluating stage `stage` (0..3) at sc.ns, rows r < NROWS
// (NX for the state recursion alone, NXT with the integral states).  The next
// stage input (or the new substep state after stage 3) goes to nxt[r] and, if
// nxt2 is not NULL, to nxt2[r] too.
template <class T, class TP, int NROWS>
__device__ __forceinline__ void rk_rows(const Interval<T, TP>& iv, RhsScratch<T, TP>& sc,
                                        RowState<T>& rs, int lane, int stage, T* nxt, T* nxt2) {
    constexpr int NQ = TP::NQ;
    T F[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        F[q] = T(0);
        if (r < NROWS) F[q] = r < NQ ? sc.ns[NQ + r] : sc.fn[r];
    }
    wave_lds_sync();
    const T s = iv.s, h = iv.h;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NROWS) {
            const T kk = s * F[q];
            if (stage == 0) rs.xa[q] = kk;
            else if (stage == 3) rs.xa[q] += kk;
            else rs.xa[q] += T(2) * kk;
            T next;
            if (stage == 0 || stage == 1) next = rs.xb[q] + (T(0.5) * h) * kk;
            else if (stage == 2) next = rs.xb[q] + h * kk;
            else {
                rs.xb[q] += iv.h6 * rs.xa[q];
                next = rs.xb[q];
            }
            nxt[r] = next;
            if (nxt2 != nullptr) nxt2[r] = next;
        }
    }
    wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Kernel arguments and the per-interval prologue shared by every kernel.
// ---------------------------------------------------------------------------
template <class T>
struct FwdArgs {
    const T* X;
    const T* U;
    const T* s;
    const T* prm;
    T* A;
    T* Bm;
    T* Bp;
    T* S;
    T* defect;
    T* xprop;
    T* ckpt;
    int64_t ldn, ldi;
    int N, K, C;
    // substep blocks (discretize only): with B > 1 work item i is block
    // b = i / N of interval i % N, substeps [b K/B, (b+1) K/B), started from
    // the x part of xinit slot b ([B][n][ld_blk], interval index contiguous);
    // outputs at column i, no defect or F~.
    const T* xinit;
    int64_t ld_blk;
    int B;
};

// Arguments of the reverse sweep of one trajectory.
template <class T>
struct AdjArgs {
    FwdArgs<T> f;
    const T* seed;
    T* gX;
    T* gs;
    T* ws_uk;    // [m][N] adjoint of U_k from interval k
    T* ws_uk1;   // [m][N] adjoint of U_{k+1} from interval k
    T* ws_p;     // [P][N] parameter adjoint from interval k
};

// Batched launches: one kernel per model over a device work list of
// (trajectory, interval) items sorted by decreasing cost; `descs` holds the
// per-trajectory argument blocks (FwdArgs or AdjArgs).
template <class DESC>
struct BatchArgs {
    const DESC* descs;
    const int2* items;   // {trajectory, interval}
    int n_items;
    int* cursor;         // [2] work cursor and finished-block count (persistent launches)
};

// Workgroups are handed to the 8 XCDs round-robin in dispatch order.  Map
// dispatch slot w (of n) to a logical index such that, inside every full block
// of 128 slots, 16 consecutive logical indices fall on one XCD, and the slots
// of the last partial block are split into 8 runs of consecutive indices, one
// per XCD: neighbouring intervals then write their output lines through the
// same L2.
__device__ __forceinline__ int xcd_slot(int w, int n) {
    const int full = n & ~127;
    if (w >= full) {
        const int r = n - full, j = w - full, x = j & 7;
        const int q = r >> 3, rem = r & 7;
        return full + x * q + (x < rem ? x : rem) + (j >> 3);
    }
    const int r = w & 127;
    return (w & ~127) | ((r & 7) << 4) | (r >> 3);
}

// Work unit u of a list of n_items items, each split into ngrp column groups:
// items are taken in blocks of 16, and inside a block all items of group 0
// come first, then group 1, ...  (a bijection onto [0, n_items * ngrp)).
__device__ __forceinline__ void unit_item(int u, int n_items, int ngrp, int& item, int& grp) {
    constexpr int BLK = 16;
    const int blk = u / (BLK * ngrp);
    const int base = blk * BLK;
    const int nb = n_items - base < BLK ? n_items - base : BLK;
    const int w = u - blk * BLK * ngrp;
    grp = w / nb;
    item = base + w % nb;
}

// Next unit of a persistent workgroup (one atomic per workgroup, broadcast
// through LDS).  Every thread of the block must call it.
__device__ __forceinline__ int fetch_unit(int* cursor, int* slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(cursor, 1);
    __syncthreads();
    const int u = *slot;
    __syncthreads();
    return u;
}

// Called once by every persistent workgroup after its last fetch: the last one
// to finish clears the cursor for the next launch (no host-side reset, so the
// launch can be replayed from a graph).
__device__ __forceinline__ void retire_block(int* cursor) {
    if (threadIdx.x == 0) {
        const unsigned nblk = gridDim.x * gridDim.y;
        if ((unsigned)atomicAdd(cursor + 1, 1) == nblk - 1) {
            atomicExch(cursor, 0);
            atomicExch(cursor + 1, 0);
        }
    }
}

__device__ __forceinline__ double stage_c(int st) { return st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5); }

// Interval inputs into LDS and per-interval constants (all threads of the block).
template <class T, class TP>
__device__ __forceinline__ void load_interval(Interval<T, TP>& iv, const FwdArgs<T>& a,
                                              const MConst<TP::NB, TP::NJ, TP::NC>& mc, int k,
                                              int tid, int nth) {
    for (int e = tid; e < TP::NXT; e += nth) {
        iv.x0[e] = a.X[e * a.ldn + k];
        iv.xk1[e] = a.X[e * a.ldn + k + 1];
    }
    for (int e = tid; e < TP::M; e += nth) {
        iv.uk[e] = a.U[e * a.ldn + k];
        iv.uk1[e] = a.U[e * a.ldn + k + 1];
    }
    for (int e = tid; e < TP::P; e += nth) iv.prm[e] = a.prm[e];
    if (tid == 0) {
        iv.s = a.s[k];
        iv.h = T(1) / T(a.K);
        iv.h6 = iv.h / T(6);
    }
    __syncthreads();
    for (int b = tid; b < TP::NB; b += nth) {
        const T m = iv.prm[2 + b];
        iv.minv[b] = T(1) / m;
        iv.iinv[b] = T(1) / (m * T(mc.ipm[b]));
    }
    __syncthreads();
    const T s = iv.s;
    for (int j = tid; j < TP::NJ; j += nth) {
        const int p = TP::parent(j), c = j + 1;
        iv.kc[j][0] = s * T(mc.ks[j]) * iv.iinv[p];
        iv.kc[j][1] = s * T(mc.ds[j]) * iv.iinv[p];
        iv.kc[j][2] = s * T(mc.ks[j]) * iv.iinv[c];
        iv.kc[j][3] = s * T(mc.ds[j]) * iv.iinv[c];
    }
    __syncthreads();
}

// Constant FOH forcing entries (s/m and s/I of joint forces and torques) of a
// zeroed coefficient buffer; called by the lanes tid = 0..nth-1.
template <class T, class TP>
__device__ __forceinline__ void coef_constants(const Interval<T, TP>& iv, T* cf, int tid,
                                               int nth) {
    using C = Coef<TP>;
    constexpr int NJ = TP::NJ, M = TP::M;
    const T s = iv.s;
    for (int j = tid; j < NJ; j += nth) {
        const int p = TP::parent(j), c = j + 1;
        T* gv = cf + C::GV;
        gv[(3 * p) * M + NJ + 2 * j] = s * iv.minv[p];
        gv[(3 * p + 1) * M + NJ + 2 * j + 1] = s * iv.minv[p];
        gv[(3 * c) * M + NJ + 2 * j] = -s * iv.minv[c];
        gv[(3 * c + 1) * M + NJ + 2 * j + 1] = -s * iv.minv[c];
        gv[(3 * p + 2) * M + j] = -s * iv.iinv[p];
        gv[(3 * c + 2) * M + j] = s * iv.iinv[c];
    }
}

template <int NB, int NJ, int NC>
inline MConst<NB, NJ, NC> make_const(const cis_model* m) {
    MConst<NB, NJ, NC> c;
    std::memset(&c, 0, sizeof(c));
    for (int b = 0; b < NB; ++b) c.ipm[b] = m->len[b] * m->len[b] / 12.0;
    for (int j = 0; j < NJ; ++j) {
        c.rp[j][0] = m->rp[2 * j];
        c.rp[j][1] = m->rp[2 * j + 1];
        c.rc[j][0] = m->rc[2 * j];
        c.rc[j][1] = m->rc[2 * j + 1];
        c.ks[j] = m->ks[j];
        c.ds[j] = m->ds[j];
    }
    for (int i = 0; i < NC; ++i) {
        c.cr[i][0] = m->cr[2 * i];
        c.cr[i][1] = m->cr[2 * i + 1];
    }
    c.g = m->g;
    c.A = m->A;
    c.kappa = m->kappa;
    return c;
}

}  // namespace cis
