// Planar maximal-coordinate model evaluated on gfx950 (arxiv 2604.09993).
//
// Compile-time topology: a torso (body 0) with L legs of D rod links each.
// Joint j joins parent(j) to child j+1; the contact of leg l sits at the tip
// of that leg's last link (on the torso when D = 0).  Geometry, stiffness,
// damping, gravity and terrain are run-time constants passed by value in the
// kernel argument segment; masses and the friction coefficient are run-time
// device inputs (they are differentiated).
//
// The per-stage work is split in two roles inside one workgroup:
//  * the nominal wave evaluates the right-hand side of the time-dilated
//    augmented system (Sec. IV-B) element-parallel: one lane per body for the
//    rotations, one lane per joint or contact for forces, violation and
//    cross-complementarity integrands, one lane per body for the Newton-Euler
//    sums, one lane per state row for the RK4 update.  It also writes the
//    nonzeros of the Jacobians at the stage state into an LDS coefficient
//    buffer;
//  * the tangent waves hold one column of [Phi | B- | B+ | S] per lane in
//    registers and apply the sparse Jacobian (a hand-written forward-mode
//    product, coefficients broadcast from LDS) plus the FOH forcing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "cis_host.hpp"

namespace cis {

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int even(int a) { return (a + 1) & ~1; }

template <int L_, int D_>
struct Topo {
    static constexpr int L = L_, D = D_;
    static constexpr int NB = 1 + L * D, NJ = L * D, NC = L;
    static constexpr int NQ = 3 * NB, NX = 6 * NB, NY = NC + 1, NXT = NX + NY;
    static constexpr int M = 3 * NJ + 3 * NC, P = NB + 2;
    static constexpr int NCOL = NX + 2 * M + 1;           // tangent columns
    static constexpr int NCW = (NCOL + 63) / 64;          // tangent waves
    static constexpr int NTHREADS = 64 * (NCW + 1);       // + one nominal wave
    static_assert(NXT <= 128, "the nominal wave owns at most two state rows per lane");
    static_assert(NB < 64 && NJ + NC <= 64, "one lane per body / element");
    __host__ __device__ static constexpr int parent(int j) {
        return D == 0 ? 0 : ((j % D == 0) ? 0 : j);
    }
    __host__ __device__ static constexpr int child(int j) { return j + 1; }
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
    static constexpr int CTH = 0;                         // [NB] s dT_b/dth_b / I_b
    static constexpr int JH = even(TP::NB);               // [NJ][4] violation row, joints
    static constexpr int CT = JH + 4 * TP::NJ;            // [NC][14] contact terms
    static constexpr int NCT = 14;
    static constexpr int GV = CT + NCT * TP::NC;          // [3NB][M] s dv'/du
    static constexpr int GC = GV + 3 * TP::NB * TP::M;    // [NC][M] (s/2) dOmega_cc/dubar
    static constexpr int F = GC + TP::NC * TP::M;         // [NXT] F~ (unscaled)
    static constexpr int SIZE = even(F + TP::NXT);
};
// per-contact slots inside Coef::CT
// (C_JMU = s lbar_n |v_t|_s is d(s Omega_cc)/d mu, used by the reverse sweep)
enum { C_AX = 0, C_AY, C_FXP, C_FYP, C_TP, C_EPX, C_EPY, C_EXD, C_EYD, C_EOM, C_ETH, C_ZPX, C_ZPY,
       C_JMU };

template <class T, class TP, int NBUF = 2>
struct Shared {
    using value_type = T;
    // stage coefficient buffers (double-buffered in the discretize kernel,
    // one in the reverse sweep, none in the defects-only kernel)
    T coef[NBUF > 0 ? NBUF : 1][NBUF > 0 ? Coef<TP>::SIZE : 2];
    T kc[cmax(TP::NJ, 1)][4];                  // s k/I_p, s d/I_p, s k/I_c, s d/I_c
    T ns[TP::NXT];                             // nominal stage input
    T fn[TP::NXT];                             // F~ at the stage
    T cs[TP::NB][2];                           // cos, sin of body angles
    T slot[cmax(2 * TP::NJ + TP::NC, 1)][4];   // (Fx, Fy, T, dT/dth) per element end
    T ctp[cmax(TP::NJ + TP::NC, 1)];           // violation integrand parts
    T uk[cmax(TP::M, 1)], uk1[cmax(TP::M, 1)]; // FOH coefficients U_k, U_k+1
    T xk1[TP::NXT];                            // X_{k+1}
    T prm[TP::P];                              // (mu, e, masses)
    T minv[TP::NB], iinv[TP::NB];              // 1/m_b, 1/I_b
    T s, h;                                    // dilation, RK4 step 1/K
};

// LDS ordering between lanes of one wave (no s_barrier needed: a wave's LDS
// instructions execute in order; the fences keep the compiler from moving
// loads and stores across the point and drain outstanding LDS traffic).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void sincos_t(double a, double* s, double* c) { sincos(a, s, c); }
__device__ __forceinline__ void sincos_t(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ __forceinline__ double sqrt_t(double a) { return sqrt(a); }
__device__ __forceinline__ float sqrt_t(float a) { return sqrtf(a); }

// Pseudo-Huber absolute value with unit steepness (Sec. II notation):
// |a|_s = sqrt(a^2+1) - 1 (evaluated as a^2/(sqrt(a^2+1)+1)) and its slope.
template <class T>
__device__ __forceinline__ void sabs_d(T a, T& val, T& der) {
    T r = sqrt_t(a * a + T(1));
    val = a * a / (r + T(1));
    der = a / r;
}

// ---------------------------------------------------------------------------
// Nominal wave: one RHS evaluation at the stage input held in sm.ns.
// Produces sm.fn (F~ without the dilation) and, if EMIT, the Jacobian
// coefficients of this stage into cf.  Called by all 64 lanes of one wave.
// ---------------------------------------------------------------------------
template <class T, class TP, bool EMIT, class SM>
__device__ __forceinline__ void nominal_rhs(SM& sm,
                                            const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                            int lane, T tau, T* cf) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, NX = TP::NX, M = TP::M;
    using C = Coef<TP>;
    const T s = sm.s;
    const T omt = T(1) - tau;
    // step 1: body rotations
    if (lane < NB) {
        T sn, cn;
        sincos_t(sm.ns[3 * lane + 2], &sn, &cn);
        sm.cs[lane][0] = cn;
        sm.cs[lane][1] = sn;
    }
    wave_lds_sync();
    // step 2: joints and contacts, one lane each
    if (lane < NJ) {
        const int j = lane;
        const int p = TP::parent(j), c = j + 1;
        const T cp = sm.cs[p][0], sp = sm.cs[p][1], cc = sm.cs[c][0], sc = sm.cs[c][1];
        const T rpx = T(mc.rp[j][0]), rpy = T(mc.rp[j][1]);
        const T rcx = T(mc.rc[j][0]), rcy = T(mc.rc[j][1]);
        const T apx = cp * rpx - sp * rpy, apy = sp * rpx + cp * rpy;
        const T acx = cc * rcx - sc * rcy, acy = sc * rcx + cc * rcy;
        const T hx = sm.ns[3 * p] + apx - sm.ns[3 * c] - acx;
        const T hy = sm.ns[3 * p + 1] + apy - sm.ns[3 * c + 1] - acy;
        const T lx = omt * sm.uk[NJ + 2 * j] + tau * sm.uk1[NJ + 2 * j];
        const T ly = omt * sm.uk[NJ + 2 * j + 1] + tau * sm.uk1[NJ + 2 * j + 1];
        const T tq = omt * sm.uk[j] + tau * sm.uk1[j];
        const T k = T(mc.ks[j]), d = T(mc.ds[j]);
        const T tsd = -k * (sm.ns[3 * c + 2] - sm.ns[3 * p + 2]) -
                      d * (sm.ns[NQ + 3 * c + 2] - sm.ns[NQ + 3 * p + 2]);
        const T tt = tq + tsd;
        sm.slot[2 * j][0] = lx;
        sm.slot[2 * j][1] = ly;
        sm.slot[2 * j][2] = (apx * ly - apy * lx) - tt;
        sm.slot[2 * j][3] = -(apx * lx + apy * ly);
        sm.slot[2 * j + 1][0] = -lx;
        sm.slot[2 * j + 1][1] = -ly;
        sm.slot[2 * j + 1][2] = -(acx * ly - acy * lx) + tt;
        sm.slot[2 * j + 1][3] = acx * lx + acy * ly;
        T vx, gx, vy, gy;
        sabs_d(hx, vx, gx);
        sabs_d(hy, vy, gy);
        sm.ctp[j] = vx + vy;
        if (EMIT) {
            cf[C::JH + 4 * j + 0] = s * gx;
            cf[C::JH + 4 * j + 1] = s * gy;
            cf[C::JH + 4 * j + 2] = s * (gy * apx - gx * apy);
            cf[C::JH + 4 * j + 3] = s * (gx * acy - gy * acx);
            const T ip = s * sm.iinv[p], ic = s * sm.iinv[c];
            cf[C::GV + (3 * p + 2) * M + NJ + 2 * j] = -apy * ip;
            cf[C::GV + (3 * p + 2) * M + NJ + 2 * j + 1] = apx * ip;
            cf[C::GV + (3 * c + 2) * M + NJ + 2 * j] = acy * ic;
            cf[C::GV + (3 * c + 2) * M + NJ + 2 * j + 1] = -acx * ic;
        }
    } else if (lane < NJ + NC) {
        const int i = lane - NJ;
        const int b = TP::cbody(i);
        const T cn = sm.cs[b][0], sn = sm.cs[b][1];
        const T rx = T(mc.cr[i][0]), ry = T(mc.cr[i][1]);
        const T ax = cn * rx - sn * ry, ay = sn * rx + cn * ry;
        const T Px = sm.ns[3 * b] + ax, Py = sm.ns[3 * b + 1] + ay;
        const T om = sm.ns[NQ + 3 * b + 2];
        const T Pdx = sm.ns[NQ + 3 * b] - om * ay, Pdy = sm.ns[NQ + 3 * b + 1] + om * ax;
        // terrain frame at P (Sec. II contact frame; Sec. VI-B sd = h/||grad h||)
        const T A = T(mc.A), kap = T(mc.kappa);
        T sw, cw;
        sincos_t(kap * Px, &sw, &cw);
        const T H = Py - A * sw;
        const T Hx = -A * kap * cw;
        const T Hxx = A * kap * kap * sw;
        const T G = sqrt_t(T(1) + Hx * Hx);
        const T G3 = G * G * G;
        const T sd = H / G;
        const T nx = Hx / G, ny = T(1) / G;
        const T tx = ny, ty = -nx;
        const T dsd_px = Hx / G - H * Hx * Hxx / G3, dsd_py = T(1) / G;
        const T dnx = Hxx / G3, dny = -Hx * Hxx / G3;
        const T dtx = dny, dty = -dnx;
        const int u0 = 3 * NJ + 3 * i;
        const T ln = omt * sm.uk[u0] + tau * sm.uk1[u0];
        const T ltp = omt * sm.uk[u0 + 1] + tau * sm.uk1[u0 + 1];
        const T ltm = omt * sm.uk[u0 + 2] + tau * sm.uk1[u0 + 2];
        const T lnb = T(0.5) * (sm.uk[u0] + sm.uk1[u0]);
        const T ltpb = T(0.5) * (sm.uk[u0 + 1] + sm.uk1[u0 + 1]);
        const T ltmb = T(0.5) * (sm.uk[u0 + 2] + sm.uk1[u0 + 2]);
        const T ft = ltp - ltm;
        const T fx = tx * ft + nx * ln, fy = ty * ft + ny * ln;
        const T vt = tx * Pdx + ty * Pdy;
        const T mu = sm.prm[0];
        const T slack = mu * lnb - ltpb - ltmb;
        T av, dav;
        sabs_d(vt, av, dav);
        const T rp = vt > T(0) ? av : T(0);     // ramp_s(v_t)
        const T rm = vt < T(0) ? av : T(0);     // ramp_s(-v_t)
        // integral cross-complementarity integrand (pairs of Sec. III)
        sm.fn[NX + i] = lnb * sd + ltpb * rp + ltmb * rm + slack * av;
        T as, das;
        sabs_d(-sd, as, das);
        sm.ctp[NJ + i] = -sd > T(0) ? as : T(0);   // ramp_s(-sd)
        sm.slot[2 * NJ + i][0] = fx;
        sm.slot[2 * NJ + i][1] = fy;
        sm.slot[2 * NJ + i][2] = ax * fy - ay * fx;
        sm.slot[2 * NJ + i][3] = -(ax * fx + ay * fy);
        if (EMIT) {
            const T gv = ltpb * (vt > T(0) ? dav : T(0)) + ltmb * (vt < T(0) ? dav : T(0)) +
                         slack * dav;
            const T Dg = -(-sd > T(0) ? das : T(0));
            const T dfx = dtx * ft + dnx * ln, dfy = dty * ft + dny * ln;
            const T dvt_px = dtx * Pdx + dty * Pdy;
            const T im = s * sm.minv[b], ii = s * sm.iinv[b];
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
    wave_lds_sync();
    // step 3: Newton-Euler sums per body; violation sum on lane NB
    if (lane < NB) {
        const int b = lane;
        T Fx = T(0), Fy = T(0), Tq = T(0), dT = T(0);
        auto add = [&](int sl) {
            Fx += sm.slot[sl][0];
            Fy += sm.slot[sl][1];
            Tq += sm.slot[sl][2];
            dT += sm.slot[sl][3];
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
        const T mi = sm.minv[b], ii = sm.iinv[b];
        sm.fn[NQ + 3 * b] = Fx * mi;
        sm.fn[NQ + 3 * b + 1] = Fy * mi - T(mc.g);
        sm.fn[NQ + 3 * b + 2] = Tq * ii;
        if (EMIT) cf[C::CTH + b] = s * dT * ii;
    } else if (lane == NB) {
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < NJ + NC; ++e) acc += sm.ctp[e];
        sm.fn[NX + NC] = acc;
    }
    wave_lds_sync();
}

// Nominal RK4 row state of one lane: rows r = lane and lane + 64.
template <class T>
struct RowState {
    T xb[2], xa[2];
};

// RK4 update of the nominal state after a stage evaluation.  stage in 0..3.
// Writes the next stage input into sm.ns (or the new substep state after
// stage 3) and, if EMIT, F~ into cf.
template <class T, class TP, bool EMIT, class SM>
__device__ __forceinline__ void nominal_update(SM& sm, RowState<T>& rs, int lane,
                                               int stage, T* cf) {
    constexpr int NXT = TP::NXT, NQ = TP::NQ;
    T F[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        F[q] = T(0);
        if (r < NXT) F[q] = r < NQ ? sm.ns[NQ + r] : sm.fn[r];
    }
    wave_lds_sync();
    const T s = sm.s, h = sm.h;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lane + 64 * q;
        if (r < NXT) {
            if (EMIT) cf[Coef<TP>::F + r] = F[q];
            const T kk = s * F[q];
            if (stage == 0) rs.xa[q] = kk;
            else if (stage == 3) rs.xa[q] += kk;
            else rs.xa[q] += T(2) * kk;
            T next;
            if (stage == 0 || stage == 1) next = rs.xb[q] + (T(0.5) * h) * kk;
            else if (stage == 2) next = rs.xb[q] + h * kk;
            else {
                rs.xb[q] += (h / T(6)) * rs.xa[q];
                next = rs.xb[q];
            }
            sm.ns[r] = next;
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
};

__device__ __forceinline__ double stage_c(int st) { return st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5); }

// Interval inputs into LDS and per-interval constants.
template <class T, class TP, class SM>
__device__ __forceinline__ void load_interval(SM& sm, const FwdArgs<T>& a,
                                              const MConst<TP::NB, TP::NJ, TP::NC>& mc, int k,
                                              int tid, int nth) {
    for (int e = tid; e < TP::NXT; e += nth) {
        sm.ns[e] = a.X[e * a.ldn + k];
        sm.xk1[e] = a.X[e * a.ldn + k + 1];
    }
    for (int e = tid; e < TP::M; e += nth) {
        sm.uk[e] = a.U[e * a.ldn + k];
        sm.uk1[e] = a.U[e * a.ldn + k + 1];
    }
    for (int e = tid; e < TP::P; e += nth) sm.prm[e] = a.prm[e];
    if (tid == 0) {
        sm.s = a.s[k];
        sm.h = T(1) / T(a.K);
    }
    __syncthreads();
    for (int b = tid; b < TP::NB; b += nth) {
        const T m = sm.prm[2 + b];
        sm.minv[b] = T(1) / m;
        sm.iinv[b] = T(1) / (m * T(mc.ipm[b]));
    }
    __syncthreads();
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
