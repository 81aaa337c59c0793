// Node-level impact map and impact conditions of the transcribed problem, with
// their Jacobians (arxiv 2604.09993, Sec. II-B eq. impulse-dynamics and the
// elimination of the joint impulse that follows it; Sec. IV-C eq. FB-relax,
// eq. cito-impulse and the constraint families Theta^delta and Psi^{delta,eps}).
//
// One wave per node.  Per node the joint-impulse system
//     A Lambda = -grad h M^-1 (M v- + J^T R Phi),   A = grad h M^-1 grad h^T,
// is solved once by Gauss-Jordan elimination with one lane per column of the
// augmented matrix [A | grad h M^-1 | grad h f]: the pivot column is broadcast
// with lane reads, so the elimination runs in registers.  It leaves
// X = A^-1 grad h M^-1 (whose transpose is W = M^-1 grad h^T A^-1) and Lambda.
// Every Jacobian column of the velocity jump then follows from the identity
//     dv* = du - W (dgrad_h v* + grad h du),
// where du = df + d(M^-1) grad h^T Lambda + M^-1 dgrad_h^T Lambda lives on the
// one body a direction touches and dgrad_h on the joints at that body, so a
// lane forms its column from at most max(L, 2) joint columns of W.  The
// impact conditions of a contact depend on 14 node variables; one lane per
// (contact, variable) evaluates them in dual numbers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/cis.h"
#include "cis_host.hpp"
#include "cis_model.hpp"

namespace cis {

template <int L_, int D_>
struct ImpTopo {
    static constexpr int L = L_, D = D_;
    static constexpr int NB = 1 + L * D, NJ = L * D, NC = L;
    static constexpr int NQ = 3 * NB, NY = NC + 1, NXT = 6 * NB + NY;
    static constexpr int NJ2 = 2 * NJ, P = NB + 2;
    static constexpr int NCV = 2 * NQ + 2 * NC + NB;   // columns of JGv
    static constexpr int NTH = 10 * NC;                // rows of Theta
    static constexpr int NCT = 14;                     // columns of JTc
    static constexpr int NQP = NQ + (NQ & 1);          // row stride of X in LDS
    static constexpr int ADJ = L > 2 ? L : 2;          // joints at one body, at most
    static constexpr int NIN = 2 * NXT + 3 * NC;       // node inputs (x+, x-, Phi, Gamma)
    static_assert(NJ2 + NQ + 1 <= 64, "one lane per column of the augmented system");
    static_assert(NCT * NC <= 64, "one lane per (contact, variable)");
    static_assert(32 + 5 * NC <= 64, "one lane per (contact, wrench direction)");
    __host__ __device__ static constexpr int parent(int j) {
        return D == 0 ? 0 : ((j % D == 0) ? 0 : j);
    }
    __host__ __device__ static constexpr int cbody(int i) { return D * (i + 1); }
    // contact carried by body b, or -1
    __host__ __device__ static constexpr int contact_at(int b) {
        if (NC == 0) return -1;
        if (D == 0) return b == 0 ? 0 : -1;
        return (b >= 1 && (b - 1) % D == D - 1) ? (b - 1) / D : -1;
    }
    // slot s of the joints at body b: the joint index, whether b is its parent
    __host__ __device__ static constexpr int slot_joint(int b, int s, bool& b_is_parent) {
        b_is_parent = false;
        if (NJ == 0) return -1;
        if (b == 0) {
            b_is_parent = true;
            return s < L ? s * D : -1;
        }
        if (s == 0) return b - 1;                             // the joint above b
        b_is_parent = true;
        return (s == 1 && (b - 1) % D != D - 1) ? b : -1;     // the joint below b
    }
};

// ---------------------------------------------------------------------------
// Dual numbers (value, directional derivative) for the contact terms.
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual dn(double v, double d = 0.0) { return Dual{v, d}; }
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
    return {a.v * b.v, fma(a.d, b.v, a.v * b.d)};
}
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {   // a.v > 0 wherever it is used
    const double s = sqrt(a.v);
    return {s, a.d / (2.0 * s)};
}
__device__ __forceinline__ void dsincos(Dual a, Dual& s, Dual& c) {
    double sv, cv;
    sincos_t(a.v, &sv, &cv);
    s = {sv, cv * a.d};
    c = {cv, -sv * a.d};
}
// pseudo-Huber absolute value sqrt(a^2+1) - 1, written a^2 / (sqrt(a^2+1) + 1)
__device__ __forceinline__ Dual dsabs(Dual a) {
    const Dual r = dsqrt(a * a + dn(1.0));
    return (a * a) / (r + dn(1.0));
}
// Fischer-Burmeister relaxation a + b - sqrt(a^2 + b^2 + delta), delta > 0
__device__ __forceinline__ Dual dfb(Dual a, Dual b, double delta) {
    return a + b - dsqrt(a * a + b * b + dn(delta));
}

// Contact frame at P (Sec. II; terrain h = P_y - A sin(kappa P_x), signed
// distance h / ||grad h|| as in Sec. VI-B): sd, normal n, tangent t = (n_y, -n_x).
template <class MC>
__device__ __forceinline__ void frame_d(const MC& mc, Dual Px, Dual Py, Dual& sd, Dual& nx,
                                        Dual& ny, Dual& tx, Dual& ty) {
    Dual sw, cw;
    dsincos(mc.kappa * Px, sw, cw);
    const Dual H = Py - mc.A * sw;
    const Dual Hx = (-mc.A * mc.kappa) * cw;
    const Dual G = dsqrt(dn(1.0) + Hx * Hx);
    sd = H / G;
    nx = Hx / G;
    ny = dn(1.0) / G;
    tx = ny;
    ty = -nx;
}

// World-frame contact impulse R Phi = t Phi_t + n Phi_n at contact i of a body
// at (x, y, th), and its generalized force on that body (force, moment of the
// force about the body origin).
template <class MC>
__device__ __forceinline__ void contact_wrench(const MC& mc, int i, Dual x, Dual y, Dual th,
                                               Dual pt, Dual pn, Dual& Fx, Dual& Fy, Dual& Tq) {
    Dual s, c;
    dsincos(th, s, c);
    const double rx = mc.cr[i][0], ry = mc.cr[i][1];
    const Dual ax = rx * c - ry * s, ay = rx * s + ry * c;
    Dual sd, nx, ny, tx, ty;
    frame_d(mc, x + ax, y + ay, sd, nx, ny, tx, ty);
    Fx = tx * pt + nx * pn;
    Fy = ty * pt + ny * pn;
    Tq = ax * Fy - ay * Fx;
}

template <class TP>
struct ImpShared {
    double z[TP::NIN];                  // x+ | x- | Phi | Gamma of the node
    double ynext[TP::NY];               // integral states of x- at the next node
    double prm[TP::P];
    double cs[TP::NB][2];               // cos, sin of the post-impact angles
    double minv[TP::NQ];                // diagonal of M^-1
    double arm[cmax(TP::NJ, 1)][4];     // world-frame joint arms a_p, a_c
    double cw[cmax(TP::NC, 1)][3];      // generalized contact force on the contact body
    double f[TP::NQ];                   // v- + M^-1 J^T R Phi
    double vs[TP::NQ];                  // v*
    double lam[cmax(TP::NJ2, 1)];       // Lambda
    double X[cmax(TP::NJ2, 1)][TP::NQP];   // A^-1 grad h M^-1
    double dw[cmax(TP::NC, 1)][5][3];   // d(contact wrench)/d(x_b, y_b, th_b, Phi_t, Phi_n)
};

// value of v in lane `src` (wave-uniform), in every lane
__device__ __forceinline__ double bcast(double v, int src) {
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(w.x, src),
                                                __builtin_amdgcn_readlane(w.y, src)));
}

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct ImpactArgs {
    const double* Xp;      // [nx][ld]
    const double* Xm;      // [nx][ld]
    const double* Phi;     // [2 nc][ld]
    const double* Gam;     // [nc][ld]
    const double* prm;     // [P]
    double* G;             // [n][nx]
    double* Theta;         // [n][10 nc]
    double* JGv;           // [n][3 nb][NCV]
    double* JTc;           // [n][10 nc][14]
    double* Psi;           // [n-1][ny] or null
    int64_t ld;
    int n;
    double delta, eps;
};

template <class TP>
__global__ void __launch_bounds__(64) k_impact(ImpactArgs a, MConst<TP::NB, TP::NJ, TP::NC> mc) {
    constexpr int NB = TP::NB, NJ = TP::NJ, NC = TP::NC, NQ = TP::NQ, NY = TP::NY;
    constexpr int NXT = TP::NXT, NJ2 = TP::NJ2, NCV = TP::NCV, NIN = TP::NIN;
    __shared__ ImpShared<TP> sh;
    const int lane = threadIdx.x;
    const int k = xcd_slot(blockIdx.x, gridDim.x);
    if (k >= a.n) return;   // whole wave
    const int64_t ld = a.ld;

    // ---- node inputs -------------------------------------------------------
    for (int r = lane; r < NIN; r += 64) {
        const double* src = r < NXT ? a.Xp + (int64_t)r * ld
                          : r < 2 * NXT ? a.Xm + (int64_t)(r - NXT) * ld
                          : r < 2 * NXT + 2 * NC ? a.Phi + (int64_t)(r - 2 * NXT) * ld
                                                 : a.Gam + (int64_t)(r - 2 * NXT - 2 * NC) * ld;
        sh.z[r] = src[k];
    }
    if (lane < TP::P) sh.prm[lane] = a.prm[lane];
    if (a.Psi && lane < NY && k + 1 < a.n) sh.ynext[lane] = a.Xm[(int64_t)(6 * NB + lane) * ld + k + 1];
    lds_sync();
    const double* qp = sh.z;              // post-impact pose
    const double* vp = sh.z + NQ;         // post-impact velocity
    const double* qm = sh.z + NXT;
    const double* vm = sh.z + NXT + NQ;
    const double* phi = sh.z + 2 * NXT;
    const double* gam = sh.z + 2 * NXT + 2 * NC;

    // ---- rotations, M^-1 ---------------------------------------------------
    if (lane < NB) {
        double sn, cn;
        sincos_t(qp[3 * lane + 2], &sn, &cn);
        sh.cs[lane][0] = cn;
        sh.cs[lane][1] = sn;
        const double m = sh.prm[2 + lane];
        sh.minv[3 * lane] = 1.0 / m;
        sh.minv[3 * lane + 1] = 1.0 / m;
        sh.minv[3 * lane + 2] = 1.0 / (m * mc.ipm[lane]);
    }
    lds_sync();
    // ---- joint arms, contact wrenches --------------------------------------
    if constexpr (NJ > 0) {
        if (lane < NJ) {
            const int p = TP::parent(lane), c = lane + 1;
            const double cp = sh.cs[p][0], sp = sh.cs[p][1], cc = sh.cs[c][0], sc = sh.cs[c][1];
            sh.arm[lane][0] = cp * mc.rp[lane][0] - sp * mc.rp[lane][1];
            sh.arm[lane][1] = sp * mc.rp[lane][0] + cp * mc.rp[lane][1];
            sh.arm[lane][2] = cc * mc.rc[lane][0] - sc * mc.rc[lane][1];
            sh.arm[lane][3] = sc * mc.rc[lane][0] + cc * mc.rc[lane][1];
        }
    }
    if constexpr (NC > 0) {
        // lane 32 + 5 i + d: the wrench of contact i and its derivative along
        // direction d of (x_b, y_b, th_b, Phi_t, Phi_n)
        if (lane >= 32 && lane < 32 + 5 * NC) {
            const int i = (lane - 32) / 5, d = lane - 32 - 5 * i, b = TP::cbody(i);
            Dual Fx, Fy, Tq;
            contact_wrench(mc, i, dn(qp[3 * b], d == 0), dn(qp[3 * b + 1], d == 1),
                           dn(qp[3 * b + 2], d == 2), dn(phi[2 * i], d == 3),
                           dn(phi[2 * i + 1], d == 4), Fx, Fy, Tq);
            if (d == 0) {
                sh.cw[i][0] = Fx.v;
                sh.cw[i][1] = Fy.v;
                sh.cw[i][2] = Tq.v;
            }
            sh.dw[i][d][0] = Fx.d;
            sh.dw[i][d][1] = Fy.d;
            sh.dw[i][d][2] = Tq.d;
        }
    }
    lds_sync();
    if (lane < NQ) {
        const int b = lane / 3, q = lane - 3 * b, i = TP::contact_at(b);
        const double gen = i >= 0 ? sh.cw[i < 0 ? 0 : i][q] : 0.0;
        sh.f[lane] = vm[lane] + sh.minv[lane] * gen;
    }
    lds_sync();

    // ---- joint impulse: Gauss-Jordan on [A | grad h M^-1 | grad h f] --------
    if constexpr (NJ > 0) {
        // grad h row l (joint l/2, component l&1) restricted to body coordinate r
        double y[NQ];
        {
            const int jl = (lane < NJ2 ? lane : 0) >> 1, cl = lane & 1;
            const int pl = TP::parent(jl), chl = jl + 1;
            // (E a)_c with E a = (-a_y, a_x)
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
                                       : sh.f[r];
            }
        }
        double col[NJ2];
#pragma unroll
        for (int i = 0; i < NJ2; ++i) {
            const int j = i >> 1, c = i & 1, p = TP::parent(j), ch = j + 1;
            const double eap = c == 0 ? -sh.arm[j][1] : sh.arm[j][0];
            const double eac = c == 0 ? -sh.arm[j][3] : sh.arm[j][2];
            col[i] = (y[3 * p + c] + y[3 * p + 2] * eap) - (y[3 * ch + c] + y[3 * ch + 2] * eac);
        }
#pragma unroll
        for (int kk = 0; kk < NJ2; ++kk) {
            double piv[NJ2];
#pragma unroll
            for (int i = 0; i < NJ2; ++i) piv[i] = bcast(col[i], kk);
            const double t = col[kk] / piv[kk];
#pragma unroll
            for (int i = 0; i < NJ2; ++i) col[i] = i == kk ? t : fma(-piv[i], t, col[i]);
        }
        if (lane >= NJ2 && lane < NJ2 + NQ) {
#pragma unroll
            for (int i = 0; i < NJ2; ++i) sh.X[i][lane - NJ2] = col[i];
        }
        if (lane == NJ2 + NQ) {
#pragma unroll
            for (int i = 0; i < NJ2; ++i) sh.lam[i] = -col[i];
        }
        lds_sync();
    }

    // ---- v* = f + M^-1 grad h^T Lambda; node residual G~ --------------------
    if (lane < NQ) {
        const int b = lane / 3, q = lane - 3 * b;
        double jt = 0.0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int p = TP::parent(j), ch = j + 1;
            const double lx = sh.lam[2 * j], ly = sh.lam[2 * j + 1];
            const double tp = sh.arm[j][0] * ly - sh.arm[j][1] * lx;   // a_p x Lambda_j
            const double tc = sh.arm[j][2] * ly - sh.arm[j][3] * lx;
            const double vpar = q == 0 ? lx : (q == 1 ? ly : tp);
            const double vch = q == 0 ? lx : (q == 1 ? ly : tc);
            if (b == p) jt += vpar;
            if (b == ch) jt -= vch;
        }
        sh.vs[lane] = sh.f[lane] + sh.minv[lane] * jt;
    }
    lds_sync();
    {
        double* Gk = a.G + (int64_t)k * NXT;
        for (int r = lane; r < NXT; r += 64) {
            double g;
            if (r < NQ) g = qp[r] - qm[r];
            else if (r < 2 * NQ) g = vp[r - NQ] - sh.vs[r - NQ];
            else g = sh.z[r] - sh.z[NXT + r];
            Gk[r] = g;
        }
        if (a.Psi && lane < NY && k + 1 < a.n)
            a.Psi[(int64_t)k * NY + lane] =
                (sh.ynext[lane] - sh.z[6 * NB + lane]) - (lane < NC ? a.delta : a.eps);
    }

    // ---- JGv: columns of dG~_v / d(q+, v-, Phi, masses) ---------------------
    double* Jk = a.JGv + (int64_t)k * NQ * NCV;
#pragma unroll 1
    for (int c0 = 0; c0 < NCV; c0 += 64) {
        const int cj = c0 + lane;
        if (cj >= NCV) break;
        int b, kind, comp;   // kind 0: q+, 1: v-, 2: Phi, 3: mass
        if (cj < NQ) { kind = 0; b = cj / 3; comp = cj % 3; }
        else if (cj < 2 * NQ) { kind = 1; b = (cj - NQ) / 3; comp = (cj - NQ) % 3; }
        else if (cj < 2 * NQ + 2 * NC) { kind = 2; comp = cj - 2 * NQ; b = TP::cbody(comp >> 1); }
        else { kind = 3; b = cj - 2 * NQ - 2 * NC; comp = 0; }
        double du[3] = {0.0, 0.0, 0.0};
        if constexpr (NC > 0) {
            const int i = TP::contact_at(b);
            if (i >= 0 && (kind == 0 || kind == 2)) {
                const int d = kind == 0 ? comp : 3 + (comp & 1);
#pragma unroll
                for (int q = 0; q < 3; ++q) du[q] = sh.minv[3 * b + q] * sh.dw[i][d][q];
            }
        }
        if (kind == 1) du[comp] = 1.0;
        if (kind == 3) {
            const double rm = 1.0 / sh.prm[2 + b];
#pragma unroll
            for (int q = 0; q < 3; ++q) du[q] = -(sh.vs[3 * b + q] - vm[3 * b + q]) * rm;
        }
        const bool thdir = kind == 0 && comp == 2;
        // joints at b: d(grad h)^T Lambda (angle direction) and the columns of W
        int js[TP::ADJ];
        double bx[TP::ADJ], by[TP::ADJ];
        if constexpr (NJ > 0) {
            double dtq = 0.0;
#pragma unroll
            for (int s = 0; s < TP::ADJ; ++s) {
                bool par;
                const int j = TP::slot_joint(b, s, par);
                js[s] = j < 0 ? 0 : j;
                if (j >= 0 && thdir) {
                    // d(E a)/dth = -a: parent side -a_p, child side +a_c
                    const double ax = par ? -sh.arm[j][0] : sh.arm[j][2];
                    const double ay = par ? -sh.arm[j][1] : sh.arm[j][3];
                    dtq += ax * sh.lam[2 * j] + ay * sh.lam[2 * j + 1];
                }
            }
            du[2] += sh.minv[3 * b + 2] * dtq;
            const double om = sh.vs[3 * b + 2];
#pragma unroll
            for (int s = 0; s < TP::ADJ; ++s) {
                bool par;
                const int j = TP::slot_joint(b, s, par);
                double vx = 0.0, vy = 0.0;
                if (j >= 0) {
                    const double ax = par ? sh.arm[j][0] : sh.arm[j][2];
                    const double ay = par ? sh.arm[j][1] : sh.arm[j][3];
                    const double sg = par ? 1.0 : -1.0;
                    // grad h_j du  (+ d(grad h_j) v* for the angle direction)
                    vx = sg * (du[0] - du[2] * ay);
                    vy = sg * (du[1] + du[2] * ax);
                    if (thdir) {
                        vx -= sg * ax * om;
                        vy -= sg * ay * om;
                    }
                }
                bx[s] = vx;
                by[s] = vy;
            }
        }
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            double acc = (r / 3 == b) ? -du[r % 3] : 0.0;
            if constexpr (NJ > 0) {
#pragma unroll
                for (int s = 0; s < TP::ADJ; ++s)
                    acc = fma(sh.X[2 * js[s]][r], bx[s], fma(sh.X[2 * js[s] + 1][r], by[s], acc));
            }
            Jk[(int64_t)r * NCV + cj] = acc;
        }
    }

    // ---- Theta and JTc: one lane per (contact, variable) --------------------
    if constexpr (NC > 0) {
        if (lane < TP::NCT * NC) {
            const int i = lane / TP::NCT, c = lane - TP::NCT * i, b = TP::cbody(i);
            auto in = [&](double v, int idx) { return dn(v, c == idx ? 1.0 : 0.0); };
            const Dual x = in(qp[3 * b], 0), y = in(qp[3 * b + 1], 1), th = in(qp[3 * b + 2], 2);
            const Dual ux = in(vp[3 * b], 3), uy = in(vp[3 * b + 1], 4), uo = in(vp[3 * b + 2], 5);
            const Dual wx = in(vm[3 * b], 6), wy = in(vm[3 * b + 1], 7), wo = in(vm[3 * b + 2], 8);
            const Dual pt = in(phi[2 * i], 9), pn = in(phi[2 * i + 1], 10);
            const Dual g = in(gam[i], 11), mu = in(sh.prm[0], 12), e = in(sh.prm[1], 13);
            Dual s, co;
            dsincos(th, s, co);
            const double rx = mc.cr[i][0], ry = mc.cr[i][1];
            const Dual ax = rx * co - ry * s, ay = rx * s + ry * co;
            Dual sd, nx, ny, tx, ty;
            frame_d(mc, x + ax, y + ay, sd, nx, ny, tx, ty);
            // contact-point velocities J v+ and J v- (E a = (-a_y, a_x))
            const Dual px = ux - uo * ay, py = uy + uo * ax;
            const Dual mx = wx - wo * ay, my = wy + wo * ax;
            const Dual w = nx * (px + e * mx) + ny * (py + e * my);
            const Dual vt = tx * px + ty * py;
            const Dual lam = vt + g * pt / dsqrt(pt * pt + dn(1.0));
            const Dual rho = dsabs(mu * pn) - dsabs(pt);
            const double dl = a.delta;
            const Dual rows[10] = {dfb(pn, sd, dl), dfb(pn, w, dl), pn * lam - dn(dl),
                                   -(pn * lam) - dn(dl), dfb(g, rho, dl), -pn, -sd, -w, -g, -rho};
            double* Tk = a.JTc + ((int64_t)k * TP::NTH + 10 * i) * TP::NCT + c;
#pragma unroll
            for (int q = 0; q < 10; ++q) Tk[q * TP::NCT] = rows[q].d;
            if (c == 0) {
                double* th_out = a.Theta + (int64_t)k * TP::NTH + 10 * i;
#pragma unroll
                for (int q = 0; q < 10; ++q) th_out[q] = rows[q].v;
            }
        }
    }
}

template <int L, int D>
cis_status launch_impact(const cis_model* m, const ImpactArgs& args, hipStream_t stream) {
    using TP = ImpTopo<L, D>;
    const auto mc = make_const<TP::NB, TP::NJ, TP::NC>(m);
    hipLaunchKernelGGL(k_impact<TP>, dim3(args.n), dim3(64), 0, stream, args, mc);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CIS_OK
                           : fail(CIS_ERR_HIP, "cis_impact_linearize: launch failed: %s",
                                  hipGetErrorString(e));
}

}  // namespace cis

using namespace cis;

extern "C" cis_status cis_impact_dims(const cis_model* model, int32_t* n_theta, int32_t* n_jgv_cols,
                                      int32_t* n_jtc_cols) {
    if (!model) return fail(CIS_ERR_NULL, "cis_impact_dims: model is required");
    if (n_theta) *n_theta = 10 * model->nc;
    if (n_jgv_cols) *n_jgv_cols = 6 * model->nb + 2 * model->nc + model->nb;
    if (n_jtc_cols) *n_jtc_cols = 14;
    return CIS_OK;
}

extern "C" cis_status cis_impact_linearize(const cis_model* model, int32_t n_nodes, int64_t ld_node,
                                           const double* Xp, const double* Xm, const double* Phi,
                                           const double* Gamma, const double* params, double delta,
                                           double eps, double* G, double* Theta, double* JGv,
                                           double* JTc, double* Psi, void* stream) {
    if (!model) return fail(CIS_ERR_NULL, "cis_impact_linearize: model is required");
    if (n_nodes < 0 || n_nodes > (1 << 30))
        return fail(CIS_ERR_DIM, "cis_impact_linearize: n_nodes=%d out of range", n_nodes);
    if (ld_node < n_nodes || ld_node < 1)
        return fail(CIS_ERR_DIM, "cis_impact_linearize: ld_node=%lld < max(n_nodes, 1)",
                    (long long)ld_node);
    if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(eps))
        return fail(CIS_ERR_DIM, "cis_impact_linearize: delta must be finite and > 0, eps finite");
    if (n_nodes == 0) return CIS_OK;
    const bool hc = model->nc > 0;
    if (!Xp || !Xm || !params || !G || !JGv || (hc && (!Phi || !Gamma || !Theta || !JTc)))
        return fail(CIS_ERR_NULL,
                    "cis_impact_linearize: Xp, Xm, params, G, JGv (and Phi, Gamma, Theta, JTc "
                    "when the model has contacts) are required");
    const void* ptrs[] = {Xp, Xm, Phi, Gamma, params, G, Theta, JGv, JTc, Psi};
    for (const void* p : ptrs)
        if (!aligned(p, 8))
            return fail(CIS_ERR_LAYOUT, "cis_impact_linearize: pointer not aligned to 8 bytes");
    ImpactArgs a;
    a.Xp = Xp;
    a.Xm = Xm;
    a.Phi = Phi;
    a.Gam = Gamma;
    a.prm = params;
    a.G = G;
    a.Theta = Theta;
    a.JGv = JGv;
    a.JTc = JTc;
    a.Psi = Psi;
    a.ld = ld_node;
    a.n = n_nodes;
    a.delta = delta;
    a.eps = eps;
    hipStream_t hs = (hipStream_t)stream;
#define CIS_DISPATCH_IMPACT(LL, DD) \
    if (model->L == LL && model->D == DD) return launch_impact<LL, DD>(model, a, hs);
    CIS_TOPOLOGIES(CIS_DISPATCH_IMPACT)
#undef CIS_DISPATCH_IMPACT
    return fail(CIS_ERR_UNSUPPORTED, "cis_impact_linearize: topology has no compiled kernel");
}
