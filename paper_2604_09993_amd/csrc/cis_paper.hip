// Discretize step of the paper-faithful dynamics variant (arxiv 2604.09993):
// joint reaction forces eliminated at the acceleration level (Sec. II-A,
// eq. joint-cnstr-acc), controls u = (tau, (phi_t, phi_n, gamma) per contact)
// (the state-space form after it), and the auxiliary system of eq. aux-dynamics
// with four integral states per contact (phi_n, lambda_c, gamma, rho_c) and one
// violation state summing ramp_s(g) over g = (-phi_n, -sd, -gamma, -rho_c).
// Classical RK4 with K substeps and the variational equations through the same
// stages (Sec. IV-B, Sec. VI), FP64.
//
// With M v' = W + J^T R phi + grad h^T lambda and grad h v' + c = 0
// (c_j = -w_p^2 a_p + w_c^2 a_c), the joint forces solve A lambda =
// -(grad h M^-1 (W + J^T R phi) + c), A = grad h M^-1 grad h^T.  For a
// direction z of the state (or of the controls) the acceleration moves by
//     dv' = M^-1 u - Wm b,   Wm = M^-1 grad h^T A^-1,
//     u = dF + dgrad_h^T lambda,   b = grad h M^-1 u + dgrad_h v' + dc,
// where u and b are local: u on the bodies z touches and their joint
// neighbours, b on the joints at those bodies.  Two kernels:
//   k_paper_rec : one wave per interval; the nominal RK4 on body lanes, and
//                 per stage the values, A and its Gauss-Jordan elimination in
//                 registers (one lane per column of [A | grad h M^-1 | r]),
//                 which leave Wm and lambda; a stage record to device memory;
//   k_paper_tan : per (interval, block of 64 columns of [Phi_x | B- | B+ | S])
//                 one wave per leg, a lane holding its column on the torso and
//                 leg rows; per stage u on those rows (the torso's hip terms
//                 of the other legs through LDS), b on the leg's joints (all
//                 joints through LDS), then dv' with the record's Wm rows read
//                 by scalar loads.
#include <hip/hip_runtime.h>

#include <cstring>
#include <utility>

#include "../../include/cis.h"
#include "cis_debug.hpp"
#include "cis_host.hpp"
#include "cis_launch.hpp"
#include "cis_model.hpp"

namespace cis {

template <int L_, int D_>
struct PTopo {
    static constexpr int L = L_, D = D_;
    static constexpr int NB = 1 + L * D, NJ = L * D, NC = L;
    static constexpr int NQ = 3 * NB, N6 = 6 * NB;
    static constexpr int NY = 4 * NC + 1, NX = N6 + NY;   // augmented state
    static constexpr int M = NJ + 3 * NC, P = NB + 2;
    static constexpr int NJ2 = 2 * NJ, LB = D + 1;
    static constexpr int NCOL = N6 + 2 * M + 1;            // [Phi_x | B- | B+ | S]
    static constexpr int NBLK = (NCOL + 63) / 64;
    static_assert(NJ2 + NQ + 1 <= 64, "one lane per column of the augmented system");
    __host__ __device__ static constexpr int parent(int j) { return (j % D == 0) ? 0 : j; }
    __host__ __device__ static constexpr int cbody(int i) { return D * (i + 1); }
};

// Layout of an interval's record area (doubles):
//   header [HDR]: s, h, h/6, 0 x5, then 1/m, 1/m, 1/I per body, then (k_j, d_j)
//   stage t < 4 K at HDR + t * STAGE:
//     WM   [NQ][NJ2]  Wm = M^-1 grad h^T A^-1
//     BODY [NB][6]    v (stage input), v'
//     JNT  [NJ][6]    a_p, a_c (world), lambda
//     CON  [NC][CN]   contact terms (offsets C_*)
//     CT   [8]        violation integrand value
template <class TP>
struct PRec {
    static constexpr int CN = 32;
    static constexpr int HDR = (8 + TP::NQ + 2 * TP::NJ + 7) / 8 * 8;
    static constexpr int WM = 0;
    static constexpr int BODY = WM + TP::NQ * TP::NJ2;
    static constexpr int JNT = BODY + 6 * TP::NB;
    static constexpr int CON = JNT + 6 * TP::NJ;
    static constexpr int CT = CON + CN * TP::NC;
    static constexpr int STAGE = (CT + 8 + 7) / 8 * 8;
    static constexpr int64_t per_interval(int K) { return HDR + (int64_t)4 * K * STAGE; }
};
// contact slots: arm a, tangent t, normal n, dt/dPx, dn/dPx, grad sd, force F,
// contact-point velocity J v, integrands (phi_n, lambda_c, gamma, rho_c), and
// the control partials of the integrands
enum {
    P_AX = 0, P_AY, P_TX, P_TY, P_NX, P_NY, P_DTX, P_DTY, P_DNX, P_DNY, P_GSX, P_GSY, P_FX, P_FY,
    P_JVX, P_JVY, P_OPN, P_OLC, P_OGM, P_ORC,
    P_LCT,   // d lambda_c / d phi_t = gamma / (phi_t^2 + 1)^(3/2)
    P_LCG,   // d lambda_c / d gamma = phi_t / sqrt(phi_t^2 + 1)
    P_RCN,   // d rho_c / d phi_n
    P_RCT,   // d rho_c / d phi_t
    P_CCN,   // d ramp_s(-phi_n) / d phi_n
    P_CCG,   // d ramp_s(-gamma) / d gamma
    P_CCR,   // d ramp_s(-rho_c) / d rho_c
    P_CCS,   // d ramp_s(-sd) / d sd
    P_PT, P_PN
};

struct PaperArgs {
    const double* X;    // [NX][ldn]
    const double* U;    // [M][ldn]
    const double* s;    // [N]
    const double* prm;  // [P]
    double* A;          // [NX][NX][ldi]
    double* Bm;         // [NX][M][ldi]
    double* Bp;
    double* S;          // [NX][ldi]
    double* defect;
    double* xprop;
    double* rec;        // records of every interval
    int64_t ldn, ldi;
    int N, K;
};

__device__ __forceinline__ double pbcast(double v, int src) {
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(w.x, src),
                                                __builtin_amdgcn_readlane(w.y, src)));
}
__device__ __forceinline__ void plds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// |a|_s = sqrt(a^2+1) - 1 and its slope; ramp_s and its slope
__device__ __forceinline__ double psabs(double a) { return a * a / (sqrt(a * a + 1.0) + 1.0); }
__device__ __forceinline__ double pdsabs(double a) { return a / sqrt(a * a + 1.0); }
__device__ __forceinline__ double psramp(double a) { return a > 0.0 ? psabs(a) : 0.0; }
__device__ __forceinline__ double pdsramp(double a) { return a > 0.0 ? pdsabs(a) : 0.0; }

template <class TP>
struct PShared {
    double x0[TP::NX], xk1[TP::NX];
    double uk[TP::M], uk1[TP::M];
    double prm[TP::P];
    double minv[TP::NQ];
    double xs[TP::N6];                 // stage input (q, v)
    double cs[TP::NB][2];
    double arm[TP::NJ][4];
    double tt[TP::NJ];                 // joint torque + spring-damper torque
    double cw[TP::NC][3];              // contact wrench on the contact body
    double W[TP::NQ];                  // generalized force
    double cv[TP::NJ2];                // velocity-product term c
    double lam[TP::NJ2];
    double vd[TP::NQ];                 // v'
    double om[TP::NY];                 // Omega at the stage
};

// ---------------------------------------------------------------------------
// k_paper_rec: interval k, one wave.
// ---------------------------------------------------------------------------
template <class TP>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
    k_paper_rec(PaperArgs a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, N6 = TP::N6;
    constexpr int NX = TP::NX, NY = TP::NY, M = TP::M, NJ2 = TP::NJ2;
    using R = PRec<TP>;
    __shared__ PShared<TP> sh;
    const int lane = threadIdx.x;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    const int64_t ldn = a.ldn, ldi = a.ldi;
    double* rec = a.rec + (int64_t)k * R::per_interval(a.K);
    for (int e = lane; e < NX; e += 64) {
        sh.x0[e] = a.X[e * ldn + k];
        sh.xk1[e] = a.X[e * ldn + k + 1];
    }
    for (int e = lane; e < M; e += 64) {
        sh.uk[e] = a.U[e * ldn + k];
        sh.uk1[e] = a.U[e * ldn + k + 1];
    }
    if (lane < TP::P) sh.prm[lane] = a.prm[lane];
    plds_sync();
    if (lane < NB) {
        const double m = sh.prm[2 + lane];
        sh.minv[3 * lane] = 1.0 / m;
        sh.minv[3 * lane + 1] = 1.0 / m;
        sh.minv[3 * lane + 2] = 1.0 / (m * mc.ipm[lane]);
    }
    plds_sync();
    const double s = a.s[k], h = 1.0 / double(a.K), mu = sh.prm[0];
    // header
    for (int e = lane; e < R::HDR; e += 64) {
        double v = 0.0;
        if (e == 0) v = s;
        else if (e == 1) v = h;
        else if (e == 2) v = h / 6.0;
        else if (e >= 8 && e < 8 + NQ) v = sh.minv[e - 8];
        else if (e >= 8 + NQ && e < 8 + NQ + 2 * NJ) {
            const int j = (e - 8 - NQ) >> 1;
            v = ((e - 8 - NQ) & 1) ? mc.ds[j] : mc.ks[j];
        }
        rec[e] = v;
    }
    // nominal RK4 on body lanes: rows (q_b, v_b); integral rows on lanes < NY
    const int bl = lane < NB ? lane : 0;
    double xb[6], xa[6], xsl[6];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        xb[q] = sh.x0[3 * bl + q];
        xb[3 + q] = sh.x0[NQ + 3 * bl + q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) xsl[q] = xb[q];
    double yb = lane < NY ? sh.x0[N6 + lane] : 0.0, ya = 0.0;
    for (int t = 0; t < 4 * a.K; ++t) {
        const int st = t & 3, j = t >> 2;
        const double tau = (double(j) + (st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5))) * h;
        const double omt = 1.0 - tau;
        double* sr = rec + R::HDR + (int64_t)t * R::STAGE;
        // ---- stage input and rotations ----
        if (lane < NB) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                sh.xs[3 * lane + q] = xsl[q];
                sh.xs[NQ + 3 * lane + q] = xsl[3 + q];
            }
            double sn, cn;
            sincos_t(xsl[2], &sn, &cn);
            sh.cs[lane][0] = cn;
            sh.cs[lane][1] = sn;
        }
        plds_sync();
        const double* qs = sh.xs;
        const double* vs = sh.xs + NQ;
        // ---- joint arms, torques, velocity products; contact terms ----
        if (lane < NJ) {
            const int p = TP::parent(lane), c = lane + 1;
            const double cp = sh.cs[p][0], sp = sh.cs[p][1], cc = sh.cs[c][0], sc = sh.cs[c][1];
            const double apx = cp * mc.rp[lane][0] - sp * mc.rp[lane][1];
            const double apy = sp * mc.rp[lane][0] + cp * mc.rp[lane][1];
            const double acx = cc * mc.rc[lane][0] - sc * mc.rc[lane][1];
            const double acy = sc * mc.rc[lane][0] + cc * mc.rc[lane][1];
            sh.arm[lane][0] = apx;
            sh.arm[lane][1] = apy;
            sh.arm[lane][2] = acx;
            sh.arm[lane][3] = acy;
            const double tq = omt * sh.uk[lane] + tau * sh.uk1[lane];
            sh.tt[lane] = tq - mc.ks[lane] * (qs[3 * c + 2] - qs[3 * p + 2]) -
                          mc.ds[lane] * (vs[3 * c + 2] - vs[3 * p + 2]);
            const double wp = vs[3 * p + 2], wc = vs[3 * c + 2];
            sh.cv[2 * lane] = -wp * wp * apx + wc * wc * acx;
            sh.cv[2 * lane + 1] = -wp * wp * apy + wc * wc * acy;
        }
        double ctcs_part = 0.0;
        if (lane >= 32 && lane < 32 + NC) {
            const int i = lane - 32, b = TP::cbody(i);
            const double cb = sh.cs[b][0], sb = sh.cs[b][1];
            const double ax = cb * mc.cr[i][0] - sb * mc.cr[i][1];
            const double ay = sb * mc.cr[i][0] + cb * mc.cr[i][1];
            const double Px = qs[3 * b] + ax, Py = qs[3 * b + 1] + ay;
            // terrain frame (Sec. II; sd = H / ||grad H||, Sec. VI-B) and its x-derivative
            double sw, cw;
            sincos_t(mc.kappa * Px, &sw, &cw);
            const double H = Py - mc.A * sw;
            const double Hx = -mc.A * mc.kappa * cw;
            const double Hxx = mc.A * mc.kappa * mc.kappa * sw;
            const double G = sqrt(1.0 + Hx * Hx), rG = 1.0 / G, rG3 = rG * rG * rG;
            const double sd = H * rG;
            const double nx = Hx * rG, ny = rG;
            const double dnx = Hxx * rG3, dny = -Hx * Hxx * rG3;
            const double tx = ny, ty = -nx, dtx = dny, dty = -dnx;
            const double gsx = Hx * rG - H * Hx * Hxx * rG3, gsy = rG;
            const int u0 = NJ + 3 * i;
            const double pt = omt * sh.uk[u0] + tau * sh.uk1[u0];
            const double pn = omt * sh.uk[u0 + 1] + tau * sh.uk1[u0 + 1];
            const double gm = omt * sh.uk[u0 + 2] + tau * sh.uk1[u0 + 2];
            const double Fx = tx * pt + nx * pn, Fy = ty * pt + ny * pn;
            sh.cw[i][0] = Fx;
            sh.cw[i][1] = Fy;
            sh.cw[i][2] = ax * Fy - ay * Fx;
            const double om = vs[3 * b + 2];
            const double jvx = vs[3 * b] - om * ay, jvy = vs[3 * b + 1] + om * ax;
            const double r1 = sqrt(pt * pt + 1.0);
            const double lc = tx * jvx + ty * jvy + gm * pt / r1;
            const double rc = psabs(mu * pn) - psabs(pt);
            sh.om[4 * i] = pn;
            sh.om[4 * i + 1] = lc;
            sh.om[4 * i + 2] = gm;
            sh.om[4 * i + 3] = rc;
            ctcs_part = psramp(-pn) + psramp(-sd) + psramp(-gm) + psramp(-rc);
            double* cr = sr + R::CON + R::CN * i;
            const double vals[R::CN] = {ax, ay, tx, ty, nx, ny, dtx, dty, dnx, dny, gsx, gsy, Fx, Fy,
                                        jvx, jvy, pn, lc, gm, rc,
                                        gm / (r1 * r1 * r1), pt / r1, mu * pdsabs(mu * pn),
                                        -pdsabs(pt), -pdsramp(-pn), -pdsramp(-gm), -pdsramp(-rc),
                                        -pdsramp(-sd), pt, pn, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < R::CN; ++q) cr[q] = vals[q];
        }
        {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) acc += pbcast(ctcs_part, 32 + i);
            if (lane == 0) sh.om[4 * NC] = acc;
        }
        plds_sync();
        // ---- generalized force W ----
        if (lane < NQ) {
            const int b = lane / 3, q = lane - 3 * b;
            double w = q == 1 ? -sh.prm[2 + b] * mc.g : 0.0;
            if (q == 2) {
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    if (TP::parent(jj) == b) w -= sh.tt[jj];
                    if (jj + 1 == b) w += sh.tt[jj];
                }
            }
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (TP::cbody(i) == b) w += sh.cw[i][q];
            sh.W[lane] = w;
        }
        plds_sync();
        // ---- Gauss-Jordan on [A | grad h M^-1 | r], r = -(grad h M^-1 W + c) ----
        {
            double y[NQ];
            const int jl = (lane < NJ2 ? lane : 0) >> 1, cl = lane & 1;
            const int pl = TP::parent(jl), chl = jl + 1;
            const double eap = cl == 0 ? -sh.arm[jl][1] : sh.arm[jl][0];
            const double eac = cl == 0 ? -sh.arm[jl][3] : sh.arm[jl][2];
#pragma unroll
            for (int r = 0; r < NQ; ++r) {
                const int b = r / 3, q = r % 3;
                double row = 0.0;
                if (b == pl) row += q == cl ? 1.0 : (q == 2 ? eap : 0.0);
                if (b == chl) row -= q == cl ? 1.0 : (q == 2 ? eac : 0.0);
                const double mi = sh.minv[r];
                y[r] = lane < NJ2 ? mi * row
                     : lane < NJ2 + NQ ? (lane - NJ2 == r ? mi : 0.0)
                                       : mi * sh.W[r];
            }
            double col[NJ2];
#pragma unroll
            for (int i = 0; i < NJ2; ++i) {
                const int jj = i >> 1, c = i & 1, p = TP::parent(jj), ch = jj + 1;
                const double ep = c == 0 ? -sh.arm[jj][1] : sh.arm[jj][0];
                const double ec = c == 0 ? -sh.arm[jj][3] : sh.arm[jj][2];
                col[i] = (y[3 * p + c] + y[3 * p + 2] * ep) - (y[3 * ch + c] + y[3 * ch + 2] * ec);
                if (lane == NJ2 + NQ) col[i] = -(col[i] + sh.cv[i]);
            }
#pragma unroll
            for (int kk = 0; kk < NJ2; ++kk) {
                double piv[NJ2];
#pragma unroll
                for (int i = 0; i < NJ2; ++i) piv[i] = pbcast(col[i], kk);
                const double tv = col[kk] / piv[kk];
#pragma unroll
                for (int i = 0; i < NJ2; ++i) col[i] = i == kk ? tv : fma(-piv[i], tv, col[i]);
            }
            // Wm[r][c] = (A^-1 grad h M^-1)[c][r]
            if (lane >= NJ2 && lane < NJ2 + NQ) {
                double* wr = sr + R::WM + (lane - NJ2) * NJ2;
#pragma unroll
                for (int i = 0; i < NJ2; ++i) wr[i] = col[i];
            }
            if (lane == NJ2 + NQ) {
#pragma unroll
                for (int i = 0; i < NJ2; ++i) sh.lam[i] = col[i];
            }
        }
        plds_sync();
        // ---- v' = M^-1 (W + grad h^T lambda) ----
        if (lane < NQ) {
            const int b = lane / 3, q = lane - 3 * b;
            double jt = 0.0;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const int p = TP::parent(jj), ch = jj + 1;
                const double lx = sh.lam[2 * jj], ly = sh.lam[2 * jj + 1];
                const double tp = sh.arm[jj][0] * ly - sh.arm[jj][1] * lx;
                const double tc = sh.arm[jj][2] * ly - sh.arm[jj][3] * lx;
                if (b == p) jt += q == 0 ? lx : (q == 1 ? ly : tp);
                if (b == ch) jt -= q == 0 ? lx : (q == 1 ? ly : tc);
            }
            sh.vd[lane] = sh.minv[lane] * (sh.W[lane] + jt);
        }
        plds_sync();
        // ---- rest of the stage record ----
        if (lane < NB) {
            double* br = sr + R::BODY + 6 * lane;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                br[q] = vs[3 * lane + q];
                br[3 + q] = sh.vd[3 * lane + q];
            }
        }
        if (lane < NJ) {
            double* jr = sr + R::JNT + 6 * lane;
#pragma unroll
            for (int q = 0; q < 4; ++q) jr[q] = sh.arm[lane][q];
            jr[4] = sh.lam[2 * lane];
            jr[5] = sh.lam[2 * lane + 1];
        }
        if (lane == 0) sr[R::CT] = sh.om[4 * NC];
        // ---- RK4 of the nominal ----
        {
            const double wk = (st == 0 || st == 3) ? 1.0 : 2.0;
            const double an = (st == 2) ? h : 0.5 * h;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const double kk = s * (q < 3 ? xsl[3 + q] : sh.vd[3 * bl + q - 3]);
                xa[q] = st == 0 ? kk : xa[q] + wk * kk;
                if (st < 3) xsl[q] = xb[q] + an * kk;
            }
            const double ky = lane < NY ? s * sh.om[lane] : 0.0;
            ya = st == 0 ? ky : ya + wk * ky;
            if (st == 3) {
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    xb[q] += (h / 6.0) * xa[q];
                    xsl[q] = xb[q];
                }
                yb += (h / 6.0) * ya;
            }
        }
        plds_sync();
    }
    // ---- outputs of the nominal ----
    if (lane < NB) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = q < 3 ? 3 * lane + q : NQ + 3 * lane + q - 3;
            if (a.xprop) a.xprop[r * ldi + k] = xb[q];
            a.defect[r * ldi + k] = xb[q] - sh.xk1[r];
        }
    }
    if (lane < NY) {
        if (a.xprop) a.xprop[(N6 + lane) * ldi + k] = yb;
        a.defect[(N6 + lane) * ldi + k] = yb - sh.xk1[N6 + lane];
    }
    // A[:, n:] = [0; I]: the integral states feed back into nothing
    for (int e = lane; e < NX * NY; e += 64) {
        const int r = e / NY, cc = N6 + e % NY;
        a.A[((int64_t)r * NX + cc) * ldi + k] = (r == cc) ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------
// k_paper_tan: columns [64 cb, 64 cb + 64) of interval k, wave `leg`.  Local
// body lb = 0 is the torso, lb = 1..D the links of the leg; rows zs[3 lb + q]
// (pose) and zs[3 LB + 3 lb + q] (velocity); the leg's contact rows y[0..3]
// and its share of the violation row y[4].
// ---------------------------------------------------------------------------
template <class TP>
struct PLane {
    static constexpr int NR = 6 * TP::LB;
    double zb[NR], za[NR], zs[NR];
    double yc[5];
};

// Threads of a tangent workgroup and the elements of a stage record each of
// them loads one stage ahead (into the LDS area `sink`, never read: the loads
// bring the record, which the leg waves then read with scalar loads, into the
// L2 cache before it is needed).
template <class TP>
struct PWarm {
    static constexpr int NT = 64 * TP::L;
    static constexpr int PW = (PRec<TP>::STAGE + NT - 1) / NT;
};

template <class TP>
__device__ __forceinline__ void paper_tangent_stage(PLane<TP>& z, const double* __restrict__ hd,
                                                    const double* __restrict__ sr, double* xch,
                                                    int leg, int lane, int st, double tau,
                                                    double wbm, double wbp, int ctrl,
                                                    double fsel,
                                                    const double* __restrict__ sr_next,
                                                    double* sink) {
    constexpr int D = TP::D, L = TP::L, LB = TP::LB, NJ = TP::NJ, NJ2 = TP::NJ2, NQ = TP::NQ;
    using R = PRec<TP>;
    constexpr int NT = PWarm<TP>::NT, PW = PWarm<TP>::PW;
    double warm[PW];
#pragma unroll
    for (int e = 0; e < PW; ++e) {
        const int c = e * NT + leg * 64 + lane;
        warm[e] = sr_next[c < R::STAGE ? c : R::STAGE - 1];
    }
    const double s = hd[0], h = hd[1], h6 = hd[2];
    const double* minv = hd + 8;
    const double* kd = hd + 8 + NQ;
    auto gb = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
#define ZQ(lb, q) z.zs[3 * (lb) + (q)]
#define ZV(lb, q) z.zs[3 * LB + 3 * (lb) + (q)]
    const double* bo = sr + R::BODY;
    const double* jn = sr + R::JNT;
    const double* co = sr + R::CON + R::CN * leg;
    // FOH weight of a B- / B+ column (0 for the other columns)
    const double w = wbm * (1.0 - tau) + wbp * tau;
    // ---- u = dF + dgrad_h^T lambda (+ control forcing) on the local bodies ----
    double u[3 * LB];
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) u[r] = 0.0;
    // spring-damper and torque of the leg's joints: dtt = -k dth_rel - d dw_rel
    double hip = 0.0;
#pragma unroll
    for (int lb = 1; lb <= D; ++lb) {
        const int j = leg * D + lb - 1;
        double dtt = -kd[2 * j] * (ZQ(lb, 2) - ZQ(lb - 1, 2)) - kd[2 * j + 1] * (ZV(lb, 2) - ZV(lb - 1, 2));
        if (ctrl == j) dtt += w;   // joint torque column
        if (lb == 1) hip = -dtt;   // torso share, summed over the legs below
        else u[3 * (lb - 1) + 2] -= dtt;
        u[3 * lb + 2] += dtt;
        // dgrad_h^T lambda on the theta rows: parent -dth_p (a_p . lam), child +dth_c (a_c . lam)
        const double* jj = jn + 6 * j;
        if (lb >= 2) u[3 * (lb - 1) + 2] -= ZQ(lb - 1, 2) * (jj[0] * jj[4] + jj[1] * jj[5]);
        else hip -= ZQ(0, 2) * (jj[0] * jj[4] + jj[1] * jj[5]);
        u[3 * lb + 2] += ZQ(lb, 2) * (jj[2] * jj[4] + jj[3] * jj[5]);
    }
    // contact at the leg tip: dF = (dt/dPx phi_t + dn/dPx phi_n) dPx, torque a x F
    {
        constexpr int lb = D;
        const double dPx = ZQ(lb, 0) - co[P_AY] * ZQ(lb, 2);
        const double dFx = (co[P_DTX] * co[P_PT] + co[P_DNX] * co[P_PN]) * dPx;
        const double dFy = (co[P_DTY] * co[P_PT] + co[P_DNY] * co[P_PN]) * dPx;
        u[3 * lb] += dFx;
        u[3 * lb + 1] += dFy;
        u[3 * lb + 2] += -(co[P_AX] * co[P_FX] + co[P_AY] * co[P_FY]) * ZQ(lb, 2) +
                         (co[P_AX] * dFy - co[P_AY] * dFx);
        // contact force columns of this leg's contact
        const int i0 = NJ + 3 * leg;
        const double wt = ctrl == i0 ? w : 0.0, wn = ctrl == i0 + 1 ? w : 0.0;
        const double fx = co[P_TX] * wt + co[P_NX] * wn, fy = co[P_TY] * wt + co[P_NY] * wn;
        u[3 * lb] += fx;
        u[3 * lb + 1] += fy;
        u[3 * lb + 2] += co[P_AX] * fy - co[P_AY] * fx;
    }
    // ---- exchange 1: the torso's hip terms of every leg ----
    if constexpr (L > 1) {
        xch[leg * 64 + lane] = hip;
        __syncthreads();
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) acc += xch[l * 64 + lane];
        u[2] += acc;
    } else {
        u[2] += hip;
    }
#pragma unroll
    for (int e = 0; e < PW; ++e) sink[e * NT + leg * 64 + lane] = warm[e];
    // ---- b on the leg's joints: grad h M^-1 u + dgrad_h v' + dc ----
    double y[3 * LB];
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int q = 0; q < 3; ++q) y[3 * lb + q] = minv[3 * gb(lb) + q] * u[3 * lb + q];
    double bl[2 * D];
#pragma unroll
    for (int lb = 1; lb <= D; ++lb) {
        const int j = leg * D + lb - 1;
        const double* jj = jn + 6 * j;
        const double apx = jj[0], apy = jj[1], acx = jj[2], acy = jj[3];
        const int pb = lb - 1, cb = lb;
        const double wp = bo[6 * gb(pb) + 2], wc = bo[6 * gb(cb) + 2];
        const double ap_dd = bo[6 * gb(pb) + 5], ac_dd = bo[6 * gb(cb) + 5];
        const double thp = ZQ(pb, 2), thc = ZQ(cb, 2), dwp = ZV(pb, 2), dwc = ZV(cb, 2);
        // grad h M^-1 u (E a = (-a_y, a_x))
        double bx = (y[3 * pb] - y[3 * pb + 2] * apy) - (y[3 * cb] - y[3 * cb + 2] * acy);
        double by = (y[3 * pb + 1] + y[3 * pb + 2] * apx) - (y[3 * cb + 1] + y[3 * cb + 2] * acx);
        // dgrad_h v': -dth_p w'_p a_p + dth_c w'_c a_c
        bx += -thp * ap_dd * apx + thc * ac_dd * acx;
        by += -thp * ap_dd * apy + thc * ac_dd * acy;
        // dc: -2 w_p dw_p a_p - w_p^2 dth_p E a_p + 2 w_c dw_c a_c + w_c^2 dth_c E a_c
        bx += -2.0 * wp * dwp * apx + wp * wp * thp * apy + 2.0 * wc * dwc * acx - wc * wc * thc * acy;
        by += -2.0 * wp * dwp * apy - wp * wp * thp * apx + 2.0 * wc * dwc * acy + wc * wc * thc * acx;
        bl[2 * (lb - 1)] = bx;
        bl[2 * (lb - 1) + 1] = by;
    }
    // ---- exchange 2: b of every joint ----
    double* xb2 = xch + L * 64;
    if constexpr (L > 1) {
#pragma unroll
        for (int e = 0; e < 2 * D; ++e) xb2[(leg * 2 * D + e) * 64 + lane] = bl[e];
        __syncthreads();
    }
    // ---- dv' = M^-1 u - Wm b on the local rows ----
    double kv[3 * LB];
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* wr = sr + R::WM + (3 * gb(lb) + q) * NJ2;
            double acc = y[3 * lb + q];
#pragma unroll
            for (int e = 0; e < NJ2; ++e) {
                double be;
                if constexpr (L > 1) be = xb2[e * 64 + lane];
                else be = bl[e];
                acc = fma(-wr[e], be, acc);
            }
            kv[3 * lb + q] = s * acc + fsel * bo[6 * gb(lb) + 3 + q];
        }
    // ---- the leg's integral rows and its share of the violation row ----
    double ky[5];
    {
        constexpr int lb = D;
        const double dPx = ZQ(lb, 0) - co[P_AY] * ZQ(lb, 2);
        const double dPy = ZQ(lb, 1) + co[P_AX] * ZQ(lb, 2);
        // d(J v) = dv_b + dw E a - w dth a
        const double wb = bo[6 * gb(lb) + 2];
        const double djx = ZV(lb, 0) - ZV(lb, 2) * co[P_AY] - wb * ZQ(lb, 2) * co[P_AX];
        const double djy = ZV(lb, 1) + ZV(lb, 2) * co[P_AX] - wb * ZQ(lb, 2) * co[P_AY];
        double dlc = (co[P_DTX] * co[P_JVX] + co[P_DTY] * co[P_JVY]) * dPx +
                     co[P_TX] * djx + co[P_TY] * djy;
        double dct = co[P_CCS] * (co[P_GSX] * dPx + co[P_GSY] * dPy);
        double dpn = 0.0, dgm = 0.0, drc = 0.0;
        const int i0 = NJ + 3 * leg;
        const double wt = ctrl == i0 ? w : 0.0, wn = ctrl == i0 + 1 ? w : 0.0;
        const double wg = ctrl == i0 + 2 ? w : 0.0;
        dpn += wn;
        dgm += wg;
        dlc += co[P_LCT] * wt + co[P_LCG] * wg;
        drc += co[P_RCN] * wn + co[P_RCT] * wt;
        dct += co[P_CCN] * wn + co[P_CCG] * wg + co[P_CCR] * (co[P_RCN] * wn + co[P_RCT] * wt);
        ky[0] = s * dpn + fsel * co[P_OPN];
        ky[1] = s * dlc + fsel * co[P_OLC];
        ky[2] = s * dgm + fsel * co[P_OGM];
        ky[3] = s * drc + fsel * co[P_ORC];
        ky[4] = s * dct + (leg == 0 ? fsel * sr[R::CT] : 0.0);
    }
    // ---- classical RK4 combination ----
    const double wk = (st == 0 || st == 3) ? 1.0 : 2.0;
    const double an = (st == 2) ? h : 0.5 * h;
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int r = 3 * lb + q;
            const double kq = s * z.zs[3 * LB + r] + fsel * bo[6 * gb(lb) + q];
            z.za[r] = st == 0 ? kq : z.za[r] + wk * kq;
            if (st < 3) z.zs[r] = z.zb[r] + an * kq;
        }
#pragma unroll
    for (int r = 0; r < 3 * LB; ++r) {
        z.za[3 * LB + r] = st == 0 ? kv[r] : z.za[3 * LB + r] + wk * kv[r];
        if (st < 3) z.zs[3 * LB + r] = z.zb[3 * LB + r] + an * kv[r];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) z.yc[q] += (h6 * wk) * ky[q];
    if (st == 3) {
#pragma unroll
        for (int r = 0; r < 6 * LB; ++r) {
            z.zb[r] += h6 * z.za[r];
            z.zs[r] = z.zb[r];
        }
    }
    if constexpr (L > 1) __syncthreads();   // the exchange areas are reused next stage
#undef ZQ
#undef ZV
}

template <class TP>
__global__ void __launch_bounds__(64 * TP::L) __attribute__((amdgpu_waves_per_eu(2)))
    k_paper_tan(PaperArgs a) {
    constexpr int N6 = TP::N6, NQ = TP::NQ, M = TP::M, D = TP::D, L = TP::L, LB = TP::LB;
    constexpr int NX = TP::NX, NC = TP::NC;
    using R = PRec<TP>;
    __shared__ double xch[(TP::L + 2 * TP::NJ) * 64];
    __shared__ double sink[PWarm<TP>::PW * PWarm<TP>::NT];
    int k, cb;
    unit_item(xcd_slot(blockIdx.x, gridDim.x), a.N, TP::NBLK, k, cb);
    const int tid = threadIdx.x, lane = tid & 63;
    const int leg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = cb * 64 + lane;
    const bool active = col < TP::NCOL;
    auto gb = [&](int lb) { return lb == 0 ? 0 : 1 + leg * D + lb - 1; };
    double wbm = 0.0, wbp = 0.0, fsel = 0.0;
    int ctrl = -1;
    if (col >= N6 && col < N6 + M) { wbm = 1.0; ctrl = col - N6; }
    else if (col >= N6 + M && col < N6 + 2 * M) { wbp = 1.0; ctrl = col - N6 - M; }
    else if (col == N6 + 2 * M) fsel = 1.0;
    PLane<TP> z;
#pragma unroll
    for (int lb = 0; lb < LB; ++lb)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int g = 3 * gb(lb) + q;
            z.zb[3 * lb + q] = (g == col) ? 1.0 : 0.0;
            z.zb[3 * LB + 3 * lb + q] = (NQ + g == col) ? 1.0 : 0.0;
        }
#pragma unroll
    for (int r = 0; r < 6 * LB; ++r) {
        z.zs[r] = z.zb[r];
        z.za[r] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) z.yc[q] = 0.0;
    const double* hd = a.rec + (int64_t)k * R::per_interval(a.K);
    const double h = 1.0 / double(a.K);
    for (int t = 0; t < 4 * a.K; ++t) {
        const int st = t & 3, j = t >> 2;
        const double tau = (double(j) + (st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5))) * h;
        const double* sr = hd + R::HDR + (int64_t)t * R::STAGE;
        paper_tangent_stage<TP>(z, hd, sr, xch, leg, lane, st, tau, wbm, wbp, ctrl, fsel,
                                t + 1 < 4 * a.K ? sr + R::STAGE : sr, sink);
    }
    // the warm-up copies are never read; a read on a path that never runs
    // (K >= 1 is checked on the host) keeps their stores
    if (a.K <= 0) xch[tid] = sink[tid];
    // violation row: the legs' shares in leg order
    double yct = z.yc[4];
    if constexpr (L > 1) {
        xch[leg * 64 + lane] = yct;
        __syncthreads();
        yct = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) yct += xch[l * 64 + lane];
    }
    if (!active) return;
    const int64_t ldi = a.ldi;
    double* out;
    int64_t cstride, c0;   // element (row, column) at out[(row * cstride + c0) * ldi + k]
    if (col < N6) { out = a.A; cstride = NX; c0 = col; }
    else if (col < N6 + M) { out = a.Bm; cstride = M; c0 = col - N6; }
    else if (col < N6 + 2 * M) { out = a.Bp; cstride = M; c0 = col - N6 - M; }
    else { out = a.S; cstride = 1; c0 = 0; }
#pragma unroll
    for (int lb = 0; lb < LB; ++lb) {
        if (lb == 0 && leg != 0) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int g = 3 * gb(lb) + q;
            out[((int64_t)g * cstride + c0) * ldi + k] = z.zb[3 * lb + q];
            out[((int64_t)(NQ + g) * cstride + c0) * ldi + k] = z.zb[3 * LB + 3 * lb + q];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) out[((int64_t)(N6 + 4 * leg + q) * cstride + c0) * ldi + k] = z.yc[q];
    if (leg == 0) out[((int64_t)(N6 + 4 * NC) * cstride + c0) * ldi + k] = yct;
}

template <int L, int D>
static cis_status launch_paper_t(const cis_model* m, const PaperArgs& a, hipStream_t stream) {
    if constexpr (L >= 1 && D >= 1) {
        using TP = PTopo<L, D>;
        const auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
        hipLaunchKernelGGL(k_paper_rec<TP>, dim3(a.N), dim3(64), 0, stream, a, mc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_paper_rec launch: %s", hipGetErrorString(e));
        hipLaunchKernelGGL(k_paper_tan<TP>, dim3(a.N * TP::NBLK), dim3(64 * TP::L), 0, stream, a);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(CIS_ERR_HIP, "k_paper_tan launch: %s", hipGetErrorString(e));
        return CIS_OK;
    } else {
        return fail(CIS_ERR_UNSUPPORTED, "the paper-dynamics form needs legs with links");
    }
}

template <int L, int D>
static int64_t paper_elems_t(int K) {
    if constexpr (L >= 1 && D >= 1) return PRec<PTopo<L, D>>::per_interval(K);
    else return -1;
}

static int64_t paper_elems(const cis_model* m, int K) {
#define CIS_PAPER_SZ(LL, DD) \
    if (m->L == LL && m->D == DD) return paper_elems_t<LL, DD>(K);
    CIS_TOPOLOGIES(CIS_PAPER_SZ)
#undef CIS_PAPER_SZ
    return -1;
}

}  // namespace cis

using namespace cis;

extern "C" cis_status cis_paper_dims(const cis_model* model, int32_t* nx, int32_t* m) {
    if (!model) return fail(CIS_ERR_NULL, "cis_paper_dims: model is required");
    if (nx) *nx = 6 * model->nb + 4 * model->nc + 1;
    if (m) *m = model->nj + 3 * model->nc;
    return CIS_OK;
}

extern "C" cis_status cis_paper_workspace_size(const cis_model* m, const cis_shape* sh,
                                               size_t* bytes) {
    if (!m || !sh || !bytes) return fail(CIS_ERR_NULL, "cis_paper_workspace_size: null argument");
    if (sh->N < 1 || sh->substeps < 1 || sh->substeps > 4096)
        return fail(CIS_ERR_DIM, "cis_paper_workspace_size: N=%d, K=%d out of range", sh->N,
                    sh->substeps);
    if (sh->dtype != CIS_F64)
        return fail(CIS_ERR_DTYPE, "cis_paper_workspace_size: the paper-dynamics form is FP64 only");
    const int64_t per = paper_elems(m, sh->substeps);
    if (per < 0) return fail(CIS_ERR_UNSUPPORTED, "paper-dynamics form: the model has no legs with links");
    *bytes = (size_t)per * (size_t)sh->N * sizeof(double);
    return CIS_OK;
}

static cis_status discretize_paper_impl(const cis_model* model, const cis_shape* shape,
                                        const void* X, const void* U, const void* s,
                                        const void* params, void* A, void* Bm, void* Bp,
                                        void* S, void* defect, void* xprop, void* ws,
                                        size_t ws_bytes, void* stream) {
    cis_status st = check_common(model, shape, X, U, s, params);
    if (st != CIS_OK) return st;
    if (shape->dtype != CIS_F64)
        return fail(CIS_ERR_DTYPE, "cis_discretize_paper: FP64 only");
    if (!A || !Bm || !Bp || !S || !defect)
        return fail(CIS_ERR_NULL, "cis_discretize_paper: A, Bm, Bp, S and defect are required");
    if (!aligned(A, 8) || !aligned(S, 8) || !aligned(defect, 8) || !aligned(xprop, 8) ||
        !aligned(Bm, 8) || !aligned(Bp, 8) || !aligned(ws, 8))
        return fail(CIS_ERR_LAYOUT, "cis_discretize_paper: pointer not aligned to 8 bytes");
    size_t need = 0;
    st = cis_paper_workspace_size(model, shape, &need);
    if (st != CIS_OK) return st;
    if (!ws || ws_bytes < need)
        return fail(CIS_ERR_WORKSPACE, "cis_discretize_paper: workspace of %zu bytes needed", need);
    PaperArgs a;
    a.X = (const double*)X;
    a.U = (const double*)U;
    a.s = (const double*)s;
    a.prm = (const double*)params;
    a.A = (double*)A;
    a.Bm = (double*)Bm;
    a.Bp = (double*)Bp;
    a.S = (double*)S;
    a.defect = (double*)defect;
    a.xprop = (double*)xprop;
    a.rec = (double*)ws;
    a.ldn = shape->ld_node;
    a.ldi = shape->ld_int;
    a.N = shape->N;
    a.K = shape->substeps;
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_PAPER(LL, DD) \
    if (model->L == LL && model->D == DD) return launch_paper_t<LL, DD>(model, a, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_PAPER)
#undef CIS_DISPATCH_PAPER
    return fail(CIS_ERR_UNSUPPORTED, "cis_discretize_paper: topology has no compiled kernel");
}

extern "C" cis_status cis_discretize_paper(const cis_model* model, const cis_shape* shape,
                                           const void* X, const void* U, const void* s,
                                           const void* params, void* A, void* Bm, void* Bp,
                                           void* S, void* defect, void* xprop, void* ws,
                                           size_t ws_bytes, void* stream) {
    cis_status st = discretize_paper_impl(model, shape, X, U, s, params, A, Bm, Bp, S, defect,
                                          xprop, ws, ws_bytes, stream);
    if (st != CIS_OK || !debug_finite_enabled()) return st;
    int32_t nx = 0, nu = 0;
    st = cis_paper_dims(model, &nx, &nu);
    if (st != CIS_OK) return st;
    return debug_scan_forward("cis_discretize_paper", model, shape, nx, nu, X, U, s, params, A,
                              Bm, Bp, S, defect, xprop, nullptr, stream);
}
