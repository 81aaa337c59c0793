// Runge-Kutta-Fehlberg form of the discretize step (arxiv 2604.09993, Sec. VI:
// the transcription integrates every interval with a Runge-Kutta-Fehlberg
// method and a fixed number of steps, and differentiates it internally).
//
// The integrator is Fehlberg's 4(5) pair: six stages per step; the fourth-order
// solution is propagated (its weight on the sixth stage is zero, so the
// sensitivities need only the first five stages), and the fifth-order one
// gives the embedded error estimate
//     e_j = h sum_i (bh_i - b_i) K_i,
// reported per interval as the largest |e_j| over its steps and all augmented
// rows.  The stage times tau = (j + c_i) / K feed the FOH controls.
//
// Two kernels in the split layout (cis_split.hpp):
//   k_rkf_rec : per interval two waves, the nominal steps on body lanes
//               (with the sixth stage for the estimate), the Jacobian
//               coefficients of the five propagated stages into compact
//               records, the integral rows, and the dilation column S;
//   k_rkf_tan : per (interval, block of 64 columns of [Phi_x | B- | B+]) one
//               wave per leg; each lane carries its column through the five
//               stages of every step with partial sums of the later stage
//               inputs (the tableau is not diagonal, unlike classical RK4).
#include <hip/hip_runtime.h>

#include <cstring>
#include <utility>

#include "../../include/cis.h"
#include "cis_body.hpp"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_model.hpp"
#include "cis_split.hpp"

namespace cis {

// Fehlberg (1969) 4(5) tableau: nodes c, coefficients a, fourth-order weights
// b, and e = (fifth-order weights) - b.
struct Fehlberg45 {
    static constexpr int S = 6;   // stages
    static constexpr int R = 5;   // stages of the propagated solution
    __host__ __device__ static constexpr double c(int i) {
        constexpr double v[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
        return v[i];
    }
    __host__ __device__ static constexpr double a(int i, int l) {
        constexpr double v[6][5] = {
            {0, 0, 0, 0, 0},
            {1.0 / 4.0, 0, 0, 0, 0},
            {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
            {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
            {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
            {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
        return v[i][l];
    }
    __host__ __device__ static constexpr double b(int i) {
        constexpr double v[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0,
                                 0.0};
        return v[i];
    }
    __host__ __device__ static constexpr double bh(int i) {
        constexpr double v[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                                 -9.0 / 50.0, 2.0 / 55.0};
        return v[i];
    }
    __host__ __device__ static constexpr double e(int i) { return bh(i) - b(i); }
};
using RKF = Fehlberg45;

template <class T, class TP>
struct RkfShared {
    Interval<T, TP> iv;
    T xring[4][TP::NX];        // stage inputs (record stage t in slot t & 3)
    T csring[4][TP::NB][2];    // their rotations
    T fring[4][3 * TP::NB];    // their accelerations
    T x6[TP::NX];              // sixth-stage input of the current step
    T cs6[TP::NB][2];
    T f6[3 * TP::NB];
    T emax[2];                 // largest estimate: x rows, integral rows
    T coef[2][CoefRec<TP>::SIZE];
};

// h sum_{l <= I} a(I + 1, l) kd[l] (compile-time coefficients; zeros skipped)
template <int I, class T, int NR>
__device__ __forceinline__ T next_input(const T (&kd)[RKF::R][NR], int r) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l <= I; ++l)
        if (RKF::a(I + 1, l) != 0.0) acc += T(RKF::a(I + 1, l)) * kd[l][r];
    return acc;
}

// ---------------------------------------------------------------------------
// k_rkf_rec: interval k by two waves, one workgroup barrier per step (five
// steps per RKF step):
//   wave 0 (state, S)    : record stage t at step t; at the fifth stage also
//                          the sixth (estimate) and the step's end; then the
//                          S column's record stage t-2 and the copy of that
//                          record to device memory;
//   wave 1 (coefficients): record stage t-1 at step t, into coef[(t-1) & 1];
//                          the integral rows and their estimate.
// ---------------------------------------------------------------------------
template <class T, class TP>
__device__ __forceinline__ void rkf_rec_item(RkfShared<T, TP>& sh, const FwdArgs<T>& a,
                                             const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                             const int k, T* __restrict__ rec, T* __restrict__ err) {
    constexpr int NB = TP::NB, NX = TP::NX, NXT = TP::NXT, NY = TP::NY, NQ = TP::NQ;
    constexpr int NC = TP::NC, NJ = TP::NJ;
    using R = CoefRec<TP>;
    using SR = SplitRec<TP>;
    constexpr int NR = RKF::R;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    constexpr int nth = 128;
    load_interval<T, TP>(sh.iv, a, mc, k, tid, nth);
    for (int e = tid; e < 2 * R::SIZE; e += nth) (&sh.coef[0][0])[e] = T(0);
    __syncthreads();
    coefrec_constants<T, TP>(sh.iv, sh.coef[0], tid, nth);
    coefrec_constants<T, TP>(sh.iv, sh.coef[1], tid, nth);
    for (int e = tid; e < SR::CRS; e += nth) {
        T v = T(0);
        if (e == 0) v = sh.iv.s;
        else if (e == 1) v = sh.iv.h;
        else if (e == 2) v = sh.iv.h6;
        else if (e >= 8 && e < 8 + 4 * NJ) v = sh.iv.kc[(e - 8) >> 2][(e - 8) & 3];
        rec[e] = v;
    }
    const int64_t ldi = a.ldi;
    const T s = sh.iv.s, h = sh.iv.h, Kt = T(a.K);
    __syncthreads();

    if (wave == 0) {
        // ------- state wave (record stage t at step t) and S column (record
        // stage t-2 at step t, then the copy of that record) -------
        const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
        T xb[6], xs[6], kd[NR][6];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            xb[q] = sh.iv.x0[3 * c.b + q];
            xb[3 + q] = sh.iv.x0[NQ + 3 * c.b + q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) xs[q] = xb[q];
        T emax = T(0);
        constexpr int NCL = SLane<T, TP>::NCL;
        T zb[6], zs[6], skd[NR][6], ycc[NCL], yct = T(0);
#pragma unroll
        for (int q = 0; q < 6; ++q) zb[q] = zs[q] = T(0);
#pragma unroll
        for (int l = 0; l < NCL; ++l) ycc[l] = T(0);
        T* out = rec + SR::CRS;
        const int nst = NR * a.K, nsteps = nst + 2;
        for (int j = 0; NR * j < nsteps; ++j) {
            const T jt = T(j);
            [&]<int... Is>(std::integer_sequence<int, Is...>) {
                ([&] {
                    constexpr int I = Is;
                    const int t = NR * j + I;
                    if (t >= nsteps) return;
                    if (t < nst) {
                        T fv[3], cb, sb;
                        body_accel<T, TP>(sh.iv, mc, c, xs, (jt + T(RKF::c(I))) / Kt, fv, cb, sb);
#pragma unroll
                        for (int q = 0; q < 6; ++q) kd[I][q] = s * (q < 3 ? xs[3 + q] : fv[q - 3]);
                        if (lane < NB) {
#pragma unroll
                            for (int q = 0; q < 3; ++q) sh.fring[t & 3][3 * c.b + q] = fv[q];
                            sh.csring[t & 3][c.b][0] = cb;
                            sh.csring[t & 3][c.b][1] = sb;
                        }
                        if constexpr (I < NR - 1) {
#pragma unroll
                            for (int q = 0; q < 6; ++q) xs[q] = xb[q] + h * next_input<I>(kd, q);
                        } else {
                            // sixth stage (estimate only), then the step's end
                            T x6[6];
#pragma unroll
                            for (int q = 0; q < 6; ++q) x6[q] = xb[q] + h * next_input<I>(kd, q);
                            T f6[3], c6, s6;
                            body_accel<T, TP>(sh.iv, mc, c, x6, (jt + T(RKF::c(5))) / Kt, f6, c6,
                                              s6);
                            if (lane < NB) {
#pragma unroll
                                for (int q = 0; q < 3; ++q) {
                                    sh.x6[3 * c.b + q] = x6[q];
                                    sh.x6[NQ + 3 * c.b + q] = x6[3 + q];
                                    sh.f6[3 * c.b + q] = f6[q];
                                }
                                sh.cs6[c.b][0] = c6;
                                sh.cs6[c.b][1] = s6;
                            }
#pragma unroll
                            for (int q = 0; q < 6; ++q) {
                                const T k6 = s * (q < 3 ? x6[3 + q] : f6[q - 3]);
                                T ev = T(RKF::e(5)) * k6, xn = T(0);
#pragma unroll
                                for (int l = 0; l < NR; ++l) {
                                    if (RKF::e(l) != 0.0) ev += T(RKF::e(l)) * kd[l][q];
                                    if (RKF::b(l) != 0.0) xn += T(RKF::b(l)) * kd[l][q];
                                }
                                emax = fmax(emax, fabs(h * ev));
                                xb[q] += h * xn;
                                xs[q] = xb[q];
                            }
                        }
                        if (lane < NB) {
#pragma unroll
                            for (int q = 0; q < 3; ++q) {
                                sh.xring[(t + 1) & 3][3 * c.b + q] = xs[q];
                                sh.xring[(t + 1) & 3][NQ + 3 * c.b + q] = xs[3 + q];
                            }
                        }
                    }
                    if (t >= 2) {
                        // the S column's record stage t - 2 (its index within
                        // the step known at compile time)
                        constexpr int J = (I + NR - 2) % NR;
                        const T* cf = sh.coef[(t - 2) & 1];
                        T kv[3], kcc[NCL], kct;
                        s_rhs<T, TP, R>(sh.iv, c, zs, cf, lane, kv, kcc, kct);
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            skd[J][q] = s * zs[3 + q] + cf[R::f(3 * c.b + q)];
                            skd[J][3 + q] = kv[q];
                        }
                        if constexpr (RKF::b(J) != 0.0) {
#pragma unroll
                            for (int l = 0; l < NCL; ++l) ycc[l] += (h * T(RKF::b(J))) * kcc[l];
                            yct += (h * T(RKF::b(J))) * kct;
                        }
                        if constexpr (J < NR - 1) {
#pragma unroll
                            for (int q = 0; q < 6; ++q) zs[q] = zb[q] + h * next_input<J>(skd, q);
                        } else {
#pragma unroll
                            for (int q = 0; q < 6; ++q) {
                                T xn = T(0);
#pragma unroll
                                for (int l = 0; l < NR; ++l)
                                    if (RKF::b(l) != 0.0) xn += T(RKF::b(l)) * skd[l][q];
                                zb[q] += h * xn;
                                zs[q] = zb[q];
                            }
                        }
#pragma unroll
                        for (int e = lane; e < R::GLOBAL; e += 64) out[e] = cf[e];
                        out += R::GLOBAL;
                    }
                    __syncthreads();
                }(), ...);
            }(std::make_integer_sequence<int, NR>{});
        }
        if (lane < NB) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int r = q < 3 ? 3 * c.b + q : NQ + 3 * c.b + q - 3;
                if (a.xprop) a.xprop[r * ldi + k] = xb[q];
                a.defect[r * ldi + k] = xb[q] - sh.iv.xk1[r];
            }
        }
        T m = T(0);
#pragma unroll
        for (int e = 0; e < NB; ++e) m = fmax(m, lane_value(emax, e));
        if (lane == 0) sh.emax[0] = m;
        T yt = T(0);
#pragma unroll
        for (int e = 0; e < NB; ++e) yt += lane_value(yct, e);
        if (lane < NB) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                a.S[(int64_t)(3 * c.b + q) * ldi + k] = zb[q];
                a.S[(int64_t)(NQ + 3 * c.b + q) * ldi + k] = zb[3 + q];
            }
            if (c.contact) a.S[(int64_t)(NX + c.i) * ldi + k] = ycc[0];
            if (lane == 0) a.S[(int64_t)(NX + NC) * ldi + k] = yt;
        }
    } else {
        // ------- coefficient wave: record stage tc at step tc + 1; integral rows -------
        const BodyConst<T, TP> c = body_const<T, TP>(sh.iv, mc, lane);
        const int ycc_row = NX + c.i;
        T ycb = c.contact ? sh.iv.x0[ycc_row] : T(0), ytb = lane == 0 ? sh.iv.x0[NX + NC] : T(0);
        T emax = T(0);
        __syncthreads();
        for (int j = 0; j < a.K; ++j) {
            const T jt = T(j);
            T yac = T(0), yat = T(0), yec = T(0), yet = T(0);
            [&]<int... Is>(std::integer_sequence<int, Is...>) {
                ([&] {
                    constexpr int I = Is;
                    const int tc = NR * j + I;
                    T ycc = T(0), yct = T(0);
                    coef_stage<T, TP, false, true, R, 2>(
                        sh.iv, mc, c, tc == 0 ? sh.iv.x0 : sh.xring[tc & 3], sh.csring[tc & 3],
                        sh.fring[tc & 3], (jt + T(RKF::c(I))) / Kt, sh.coef[tc & 1], ycc, yct, lane);
                    if constexpr (RKF::b(I) != 0.0) {
                        yac += T(RKF::b(I)) * s * ycc;
                        yat += T(RKF::b(I)) * s * yct;
                    }
                    if constexpr (RKF::e(I) != 0.0) {
                        yec += T(RKF::e(I)) * s * ycc;
                        yet += T(RKF::e(I)) * s * yct;
                    }
                    if constexpr (I == NR - 1) {
                        T y6c = T(0), y6t = T(0);
                        coef_stage<T, TP, false, false>(sh.iv, mc, c, sh.x6, sh.cs6, sh.f6,
                                                        (jt + T(RKF::c(5))) / Kt, (T*)nullptr,
                                                        y6c, y6t, lane);
                        yec += T(RKF::e(5)) * s * y6c;
                        yet += T(RKF::e(5)) * s * y6t;
                        ycb += h * yac;
                        ytb += h * yat;
                        // estimate: the cross-complementarity rows on their lanes, the
                        // violation row from the body lanes' parts
                        T et = T(0);
#pragma unroll
                        for (int e = 0; e < NB; ++e) et += lane_value(yet, e);
                        if (c.contact) emax = fmax(emax, fabs(h * yec));
                        if (lane == 0) emax = fmax(emax, fabs(h * et));
                    }
                    __syncthreads();
                }(), ...);
            }(std::make_integer_sequence<int, NR>{});
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
        for (int e = lane; e < NXT * NY; e += 64) {
            const int r = e / NY, cc = NX + e % NY;
            a.A[((int64_t)r * NXT + cc) * ldi + k] = (r == cc) ? T(1) : T(0);
        }
        T m = T(0);
#pragma unroll
        for (int e = 0; e < NB; ++e) m = fmax(m, lane_value(emax, e));
        if (lane == 0) sh.emax[1] = m;
    }
    __syncthreads();
    if (err && tid == 0) err[k] = fmax(sh.emax[0], sh.emax[1]);
}

// ---------------------------------------------------------------------------
// k_rkf_tan: one Fehlberg stage I of a leg wave.  za = x_j + h sum b_l K_l so
// far, zs = the stage input, p2..p4 = the partial sums of the inputs of
// stages 2..4 (each starts at x_j).
// ---------------------------------------------------------------------------
template <class T, class TP>
struct RkfLane {
    static constexpr int NRW = 6 * (TP::D + 1);
    T za[NRW], zs[NRW], p2[NRW], p3[NRW], p4[NRW];
    T ycc, yct;
};

template <int I, class T>
__device__ __forceinline__ void rkf_combine(T& za, T& zs, T& p2, T& p3, T& p4, T hk) {
    // hk = h K_I of one row; the input of stage I sits in zs
    if constexpr (I == 0) {
        const T base = zs;
        za = base + T(RKF::b(0)) * hk;
        p2 = base + T(RKF::a(2, 0)) * hk;
        p3 = base + T(RKF::a(3, 0)) * hk;
        p4 = base + T(RKF::a(4, 0)) * hk;
        zs = base + T(RKF::a(1, 0)) * hk;
    } else if constexpr (I == 1) {
        zs = p2 + T(RKF::a(2, 1)) * hk;
        p3 += T(RKF::a(3, 1)) * hk;
        p4 += T(RKF::a(4, 1)) * hk;
    } else if constexpr (I == 2) {
        zs = p3 + T(RKF::a(3, 2)) * hk;
        p4 += T(RKF::a(4, 2)) * hk;
        za += T(RKF::b(2)) * hk;
    } else if constexpr (I == 3) {
        zs = p4 + T(RKF::a(4, 3)) * hk;
        za += T(RKF::b(3)) * hk;
    } else {
        za += T(RKF::b(4)) * hk;
        zs = za;
    }
}
static_assert(Fehlberg45::b(1) == 0.0 && Fehlberg45::b(5) == 0.0,
              "the tangent stages assume the propagated weights of Fehlberg's pair");

template <class T, class TP, int I, bool FORCE, bool LDSF>
__device__ __forceinline__ void tangent_rkf_stage(RkfLane<T, TP>& z, const T* __restrict__ cr,
                                                  const T* __restrict__ lr,
                                                  const T* __restrict__ rs, T* xch, int leg,
                                                  int lane, T tau, T wbm, T wbp,
                                                  const unsigned (&off)[3 * (TP::D + 1)],
                                                  unsigned offcc, const T* fcur,
                                                  const T* rs_next, T* fnext) {
    constexpr int LB = TP::D + 1;
    const T s = cr[0], h = cr[1];
    T kv[3 * LB], kcc, kct;
    tangent_split_rhs<T, TP, FORCE, LDSF>(z.zs, cr, lr, rs, xch, leg, lane, tau, wbm, wbp, off,
                                          offcc, kv, kcc, kct, fcur, rs_next, fnext);
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) {
        const T hk = h * (s * z.zs[3 * LB + r]);
        rkf_combine<I>(z.za[r], z.zs[r], z.p2[r], z.p3[r], z.p4[r], hk);
    }
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) {
        const int q = 3 * LB + r;
        rkf_combine<I>(z.za[q], z.zs[q], z.p2[q], z.p3[q], z.p4[q], h * kv[r]);
    }
    if constexpr (RKF::b(I) != 0.0) {
        z.ycc += (h * T(RKF::b(I))) * kcc;
        z.yct += (h * T(RKF::b(I))) * kct;
    }
}

template <class T, class TP, bool FORCE, bool LDSF>
__device__ __forceinline__ void tangent_rkf_loop(RkfLane<T, TP>& z, const T* __restrict__ cr,
                                                 const T* __restrict__ rec0, T* xch, int leg,
                                                 int lane, int K, T wbm, T wbp,
                                                 const unsigned (&off)[3 * (TP::D + 1)],
                                                 unsigned offcc, T* fbuf) {
    using R = CoefRec<TP>;
    constexpr int LEGB = R::LEGB, GL = R::GLOBAL, L = TP::L, FBUF = SplitRec<TP>::FBUF;
    const T Kt = T(K);
    const T* rs = rec0;
    T* xb[2] = {xch, xch + L * 64};
    T* fb[2] = {fbuf, fbuf + FBUF};
    int par = 0;   // exchange and forcing buffers of the stage (alternate stage by stage)
    for (int j = 0; j < K; ++j) {
        const T jt = T(j);
        [&]<int... Is>(std::integer_sequence<int, Is...>) {
            ([&] {
                constexpr int I = Is;
                // the interval's last stage copies its own forcing region (never read)
                const T* rsn = (I == RKF::R - 1 && j + 1 == K) ? rs : rs + GL;
                tangent_rkf_stage<T, TP, I, FORCE, LDSF>(z, cr, rs + leg * LEGB, rs, xb[par], leg,
                                                         lane, (jt + T(RKF::c(I))) / Kt, wbm,
                                                         wbp, off, offcc, fb[par], rsn,
                                                         fb[par ^ 1]);
                rs += GL;
                par ^= 1;
            }(), ...);
        }(std::make_integer_sequence<int, RKF::R>{});
    }
}

template <class T, class TP>
__device__ __forceinline__ void rkf_tangent_item(const FwdArgs<T>& a, const T* __restrict__ rec,
                                                 const int k, const int cb, T* xch, T* fbuf) {
    constexpr int LB = TP::D + 1;
    using SR = SplitRec<TP>;
    const int tid = threadIdx.x, lane = tid & 63;
    const int leg = __builtin_amdgcn_readfirstlane(tid >> 6);
    T wbm, wbp;
    RkfLane<T, TP> z;
    const TanCol<TP> tc = tangent_column<T, TP>(cb, leg, lane, wbm, wbp, z.zs);
#pragma unroll
    for (int r = 0; r < 6 * LB; ++r) z.za[r] = z.zs[r];
    z.ycc = T(0);
    z.yct = T(0);
    const T* cr = rec;
    const T* rec0 = rec + SR::CRS;
    if constexpr (TP::L > 1) {
        // every block stages the records (in blocks without B-/B+ columns
        // only to bring the leg blocks into the L2 cache a stage early)
        stage_store<T, TP>(fbuf, stage_load<T, TP>(rec0, leg, lane), leg, lane);
    }
    if ((cb + 1) * 64 <= TP::NX) {
        tangent_rkf_loop<T, TP, false, (TP::L > 1)>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp,
                                                    tc.off, tc.offcc, fbuf);
    } else if constexpr (TP::L > 1) {
        // forcing from the stage records staged in LDS (stage 0's record
        // stored above, ordered before its reads by stage 0's barrier)
        tangent_rkf_loop<T, TP, true, true>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp, tc.off,
                                            tc.offcc, fbuf);
    } else {
        tangent_rkf_loop<T, TP, true, false>(z, cr, rec0, xch, leg, lane, a.K, wbm, wbp, tc.off,
                                             tc.offcc, fbuf);
    }
    tangent_store<T, TP>(a, k, leg, lane, tc, z.za, z.ycc, z.yct, xch);
}

// FP64 at one wave per SIMD: two would spill the stage derivatives to scratch.
template <class T, class TP>
__global__ void __launch_bounds__(128)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 1 : 2)))
    k_rkf_rec(FwdArgs<T> a, MConst<TP::NB, TP::NJ, TP::NC> mc, T* __restrict__ rec,
              T* __restrict__ err) {
    __shared__ RkfShared<T, TP> sh;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    rkf_rec_item<T, TP>(sh, a, mc, k, rec + (int64_t)k * SplitRec<TP>::per_interval(a.K, RKF::R),
                        err);
}

template <class T, class TP, int WAVES>
__global__ void __launch_bounds__(64 * TP::L) __attribute__((amdgpu_waves_per_eu(WAVES)))
    k_rkf_tan(FwdArgs<T> a, const T* __restrict__ rec) {
    __shared__ T xch[2 * TP::L * 64];
    __shared__ T fbuf[2 * SplitRec<TP>::FBUF];
    int item, cb;
    unit_item(xcd_slot(blockIdx.x, gridDim.x), a.N, SplitRec<TP>::NBLK, item, cb);
    rkf_tangent_item<T, TP>(a, rec + (int64_t)item * SplitRec<TP>::per_interval(a.K, RKF::R),
                            item, cb, xch, fbuf);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <int L, int D>
static int64_t rkf_elems_t(int K) {
    if constexpr (L >= 1 && D >= 1) return SplitRec<Topo<L, D>>::per_interval(K, RKF::R);
    else return -1;
}

static int64_t rkf_elems_per_interval(const cis_model* m, int K) {
#define CIS_RKF_SZ(LL, DD) \
    if (m->L == LL && m->D == DD) return rkf_elems_t<LL, DD>(K);
    CIS_TOPOLOGIES(CIS_RKF_SZ)
#undef CIS_RKF_SZ
    return -1;
}

template <class T, int L, int D>
static cis_status launch_rkf_t(const cis_model* m, const cis_shape* sh, const void* X,
                               const void* U, const void* s, const void* prm, void* A, void* Bm,
                               void* Bp, void* S, void* defect, void* xprop, void* err, void* ws,
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
        T* e = (T*)err;
        void* args_a[] = {&a, &mc, &rec, &e};
        hipError_t st = hipLaunchKernel((const void*)&k_rkf_rec<T, TP>, dim3(sh->N), dim3(128),
                                        args_a, 0, stream);
        if (st != hipSuccess) return fail(CIS_ERR_HIP, "k_rkf_rec launch: %s", hipGetErrorString(st));
        const T* crec = rec;
        void* args_b[] = {&a, &crec};
        st = hipLaunchKernel(waves == 2 ? (const void*)&k_rkf_tan<T, TP, 2>
                                        : (const void*)&k_rkf_tan<T, TP, 1>,
                             dim3(sh->N * SplitRec<TP>::NBLK), dim3(64 * TP::L), args_b, 0,
                             stream);
        if (st != hipSuccess) return fail(CIS_ERR_HIP, "k_rkf_tan launch: %s", hipGetErrorString(st));
        return CIS_OK;
    } else {
        return fail(CIS_ERR_UNSUPPORTED, "the RKF form needs legs with links");
    }
}

}  // namespace cis

using namespace cis;

static cis_status rkf_ws_bytes(const cis_model* m, const cis_shape* sh, size_t* bytes) {
    const int64_t per = rkf_elems_per_interval(m, sh->substeps);
    if (per < 0) return fail(CIS_ERR_UNSUPPORTED, "RKF form: the model has no legs with links");
    *bytes = (size_t)per * (size_t)sh->N * elem_size(sh->dtype);
    return CIS_OK;
}

extern "C" cis_status cis_rkf_workspace_size(const cis_model* m, const cis_shape* sh,
                                             size_t* bytes) {
    if (!m || !sh || !bytes) return fail(CIS_ERR_NULL, "cis_rkf_workspace_size: null argument");
    if (sh->N < 1 || sh->substeps < 1 || sh->substeps > 4096)
        return fail(CIS_ERR_DIM, "cis_rkf_workspace_size: N=%d, K=%d out of range", sh->N,
                    sh->substeps);
    if (sh->dtype != CIS_F64 && sh->dtype != CIS_F32)
        return fail(CIS_ERR_DTYPE, "cis_rkf_workspace_size: unknown dtype %d", sh->dtype);
    return rkf_ws_bytes(m, sh, bytes);
}

static cis_status discretize_rkf_impl(const cis_model* model, const cis_shape* shape,
                                      const void* X, const void* U, const void* s,
                                      const void* params, int32_t waves, void* A, void* Bm,
                                      void* Bp, void* S, void* defect, void* xprop, void* err,
                                      void* ws, size_t ws_bytes, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (waves != 1 && waves != 2)
        return fail(CIS_ERR_DIM, "cis_discretize_rkf: waves=%d must be 1 or 2", waves);
    const bool hasm = model->m > 0;
    if (!A || !S || !defect || (hasm && (!Bm || !Bp)))
        return fail(CIS_ERR_NULL, "cis_discretize_rkf: A, S, defect (and Bm, Bp when m > 0) are required");
    const size_t es = elem_size(shape->dtype);
    if (!aligned(A, es) || !aligned(S, es) || !aligned(defect, es) || !aligned(xprop, es) ||
        !aligned(Bm, es) || !aligned(Bp, es) || !aligned(err, es) || !aligned(ws, 8))
        return fail(CIS_ERR_LAYOUT, "cis_discretize_rkf: pointer not aligned to %zu bytes", es);
    size_t need = 0;
    st = rkf_ws_bytes(model, shape, &need);
    if (st != CIS_OK) return st;
    if (!ws || ws_bytes < need)
        return fail(CIS_ERR_WORKSPACE, "cis_discretize_rkf: workspace of %zu bytes needed", need);
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_RKF(LL, DD)                                                               \
    if (model->L == LL && model->D == DD)                                                      \
        return shape->dtype == CIS_F64                                                         \
                   ? launch_rkf_t<double, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp, S, \
                                                  defect, xprop, err, ws, waves, hs)           \
                   : launch_rkf_t<float, LL, DD>(model, shape, X, U, s, params, A, Bm, Bp, S,  \
                                                 defect, xprop, err, ws, waves, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_RKF)
#undef CIS_DISPATCH_RKF
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_rkf: topology has no compiled kernel");
}

extern "C" cis_status cis_discretize_rkf(const cis_model* model, const cis_shape* shape,
                                         const void* X, const void* U, const void* s,
                                         const void* params, int32_t waves, void* A, void* Bm,
                                         void* Bp, void* S, void* defect, void* xprop, void* err,
                                         void* ws, size_t ws_bytes, void* stream) {
    const cis_status st = discretize_rkf_impl(model, shape, X, U, s, params, waves, A, Bm, Bp, S,
                                              defect, xprop, err, ws, ws_bytes, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    return debug_scan_forward("cis_discretize_rkf", model, shape, model->nx, model->m, X, U, s,
                              params, A, Bm, Bp, S, defect, xprop, err, stream);
}
