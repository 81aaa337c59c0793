// Body-lane evaluation of the nominal stages (state recursion and Jacobian
// coefficients) for the discretize kernel.
//
// Lane b < NB of a wave owns body b: its six state rows (x, y, th, xd, yd, w)
// and the joint whose child it is (joint b-1, for b >= 1) and the contact it
// carries (the tip of a leg's last link).  Per stage the only cross-lane
// traffic goes through DPP row shifts and lane reads (all bodies sit in the
// first row of 16 lanes): a body's parent is the previous lane, or the torso
// (lane 0) for the first link of a leg; an interior link's child is the next
// lane, and the torso collects the first links of all legs.  Right-hand side
// as in Sec. II-A (eq. ct-dynamics),
// Sec. III (integrands) and Sec. IV-B (dilation, FOH); Jacobian nonzeros in
// the layout of Coef<TP>.
#pragma once
#include "cis_model.hpp"

namespace cis {

template <class TP>
__device__ __forceinline__ int parent_body(int b) {
    // body b >= 1 is the child of joint b-1; the torso has no parent (0 = itself)
    if (b == 0 || TP::D == 0) return 0;
    return ((b - 1) % TP::D) == 0 ? 0 : b - 1;
}
template <class TP>
__device__ __forceinline__ bool has_contact(int b) {
    if constexpr (TP::D == 0) return b == 0 && TP::L >= 1;
    else return b >= 1 && ((b - 1) % TP::D) == TP::D - 1;
}
template <class TP>
__device__ __forceinline__ int contact_of(int b) {
    return TP::D == 0 ? 0 : (b - 1) / TP::D;
}

// DPP row shifts by one lane: prev_lane(v) in lane b is v of lane b-1, next_lane(v) that
// of lane b+1 (within rows of 16 lanes; the value at a row edge is unspecified).
template <int CTRL>
__device__ __forceinline__ int dpp_row(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(dpp_row<CTRL>(w.x), dpp_row<CTRL>(w.y)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
    return __builtin_bit_cast(float, dpp_row<CTRL>(__builtin_bit_cast(int, v)));
}
template <class T>
__device__ __forceinline__ T prev_lane(T v) { return dpp_row<0x111>(v); }   // row_shr:1
template <class T>
__device__ __forceinline__ T next_lane(T v) { return dpp_row<0x101>(v); }   // row_shl:1

// value of v in lane `src` (a wave-uniform lane index), in every lane
__device__ __forceinline__ double lane_value(double v, int src) {
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(w.x, src),
                                                __builtin_amdgcn_readlane(w.y, src)));
}
__device__ __forceinline__ float lane_value(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// value of v at the parent body of this lane's body (lane 0 gets its own value)
template <class TP, class T>
__device__ __forceinline__ T from_parent(T v, bool parent_is_torso) {
    const T t = lane_value(v, 0);
    const T q = prev_lane(v);
    return parent_is_torso ? t : q;
}

// sum, in the parent lane, of a value held by the child lanes of the joints:
// interior links take it from the next lane, the torso from the first link of
// every leg (in leg order).  Lanes without children get 0.
template <class TP, class T>
__device__ __forceinline__ T from_children(T v, int b) {
    if constexpr (TP::D == 0) {
        return T(0);
    } else {
        const T q = next_lane(v);
        T t = T(0);
#pragma unroll
        for (int l = 0; l < TP::L; ++l) t += lane_value(v, 1 + l * TP::D);
        const bool interior = b >= 1 && (b % TP::D) != 0;   // not a leg tip
        return b == 0 ? t : (interior ? q : T(0));
    }
}

// Constants a body lane keeps in registers for the whole interval.
template <class T, class TP>
struct BodyConst {
    static_assert(TP::NB <= 16, "the bodies must fit one DPP row");
    int b, p;                 // own and parent body
    bool joint, contact;      // has a parent joint, carries a contact
    int j, i;                 // joint and contact index
    T rpx, rpy, rcx, rcy;     // joint anchors (parent frame, own frame)
    T kj, dj;                 // stiffness, damping of the parent joint
    T rx, ry;                 // contact point
    T mi, ii;                 // 1/m, 1/I
    T uk[3], uk1[3];          // joint controls tau, lambda_x, lambda_y at the two nodes
    T ck[3], ck1[3];          // contact controls lambda_n, lambda_t+, lambda_t-
};

template <class T, class TP>
__device__ __forceinline__ BodyConst<T, TP> body_const(const Interval<T, TP>& iv,
                                                       const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                                       int lane) {
    constexpr int NB = TP::NB, NJ = TP::NJ;
    BodyConst<T, TP> c;
    c.b = lane < NB ? lane : 0;
    c.p = parent_body<TP>(c.b);
    c.joint = TP::D >= 1 && lane < NB && c.b >= 1;
    c.contact = lane < NB && has_contact<TP>(c.b);
    c.j = c.joint ? c.b - 1 : 0;
    c.i = c.contact ? contact_of<TP>(c.b) : 0;
    c.rpx = c.rpy = c.rcx = c.rcy = c.kj = c.dj = c.rx = c.ry = T(0);
    for (int q = 0; q < 3; ++q) c.uk[q] = c.uk1[q] = c.ck[q] = c.ck1[q] = T(0);
    if constexpr (NJ > 0) {
        if (c.joint) {
            c.rpx = T(mc.rp[c.j][0]);
            c.rpy = T(mc.rp[c.j][1]);
            c.rcx = T(mc.rc[c.j][0]);
            c.rcy = T(mc.rc[c.j][1]);
            c.kj = T(mc.ks[c.j]);
            c.dj = T(mc.ds[c.j]);
            const int us[3] = {c.j, NJ + 2 * c.j, NJ + 2 * c.j + 1};
            for (int q = 0; q < 3; ++q) {
                c.uk[q] = iv.uk[us[q]];
                c.uk1[q] = iv.uk1[us[q]];
            }
        }
    }
    if constexpr (TP::NC > 0) {
        if (c.contact) {
            c.rx = T(mc.cr[c.i][0]);
            c.ry = T(mc.cr[c.i][1]);
            for (int q = 0; q < 3; ++q) {
                c.ck[q] = iv.uk[3 * NJ + 3 * c.i + q];
                c.ck1[q] = iv.uk1[3 * NJ + 3 * c.i + q];
            }
        }
    }
    c.mi = iv.minv[c.b];
    c.ii = iv.iinv[c.b];
    return c;
}

// RK4 state of a body lane: base, accumulator, stage input of its six rows
template <class T>
struct BodyRK {
    T xb[6], xa[6], xs[6];
};

// Terrain frame at the contact point (flat ground when A == 0).
template <class T>
struct Frame {
    T sd, nx, ny, tx, ty, dsd_px, dsd_py, dnx, dny;
};
template <class T, class MC>
__device__ __forceinline__ Frame<T> terrain(const MC& mc, T Px, T Py) {
    Frame<T> f;
    if (mc.A == 0.0) {
        f.sd = Py;
        f.nx = T(0);
        f.ny = T(1);
        f.tx = T(1);
        f.ty = T(0);
        f.dsd_px = T(0);
        f.dsd_py = T(1);
        f.dnx = T(0);
        f.dny = T(0);
    } else {
        // Sec. II contact frame; Sec. VI-B sd = h / ||grad h||
        const T A = T(mc.A), kap = T(mc.kappa);
        T sw, cw;
        sincos_t(kap * Px, &sw, &cw);
        const T H = Py - A * sw;
        const T Hx = -A * kap * cw;
        const T Hxx = A * kap * kap * sw;
        const T G = sqrt_t(T(1) + Hx * Hx);
        const T rG = T(1) / G;
        const T rG3 = rG * rG * rG;
        f.sd = H * rG;
        f.nx = Hx * rG;
        f.ny = rG;
        f.tx = f.ny;
        f.ty = -f.nx;
        f.dsd_px = Hx * rG - H * Hx * Hxx * rG3;
        f.dsd_py = rG;
        f.dnx = Hxx * rG3;
        f.dny = -Hx * Hxx * rG3;
    }
    return f;
}

// Accelerations fv (x, y, theta) of the lane's body at the stage input xs
// (its six rows; the parent's and children's rows come through DPP and lane
// reads) at stage time tau, and the body rotation (cb, sb).
template <class T, class TP>
__device__ __forceinline__ void body_accel(const Interval<T, TP>& iv,
                                           const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                           const BodyConst<T, TP>& c, const T (&xs)[6], T tau,
                                           T (&fv)[3], T& cb, T& sb) {
    const T omt = T(1) - tau;
    sincos_t(xs[2], &sb, &cb);
    const bool pt = c.p == 0;
    const T thp = from_parent<TP>(xs[2], pt), omp = from_parent<TP>(xs[5], pt);
    const T sp = from_parent<TP>(sb, pt), cp = from_parent<TP>(cb, pt);
    T Fx = T(0), Fy = T(0), Tq = T(0);
    T wx = T(0), wy = T(0), wt = T(0);   // parent-side wrench of the own joint
    if (c.joint) {
        const T apx = cp * c.rpx - sp * c.rpy, apy = sp * c.rpx + cp * c.rpy;
        const T acx = cb * c.rcx - sb * c.rcy, acy = sb * c.rcx + cb * c.rcy;
        const T tq = omt * c.uk[0] + tau * c.uk1[0];
        const T lx = omt * c.uk[1] + tau * c.uk1[1];
        const T ly = omt * c.uk[2] + tau * c.uk1[2];
        const T tt = tq - c.kj * (xs[2] - thp) - c.dj * (xs[5] - omp);
        Fx -= lx;
        Fy -= ly;
        Tq += -(acx * ly - acy * lx) + tt;
        wx = lx;
        wy = ly;
        wt = (apx * ly - apy * lx) - tt;
    }
    if (c.contact) {
        const T ax = cb * c.rx - sb * c.ry, ay = sb * c.rx + cb * c.ry;
        const Frame<T> f = terrain<T>(mc, xs[0] + ax, xs[1] + ay);
        const T ln = omt * c.ck[0] + tau * c.ck1[0];
        const T ft = (omt * c.ck[1] + tau * c.ck1[1]) - (omt * c.ck[2] + tau * c.ck1[2]);
        const T fx = f.tx * ft + f.nx * ln, fy = f.ty * ft + f.ny * ln;
        Fx += fx;
        Fy += fy;
        Tq += ax * fy - ay * fx;
    }
    // parent-side wrenches of the children's joints
    Fx += from_children<TP>(wx, c.b);
    Fy += from_children<TP>(wy, c.b);
    Tq += from_children<TP>(wt, c.b);
    fv[0] = Fx * c.mi;
    fv[1] = Fy * c.mi - T(mc.g);
    fv[2] = Tq * c.ii;
}

// ---------------------------------------------------------------------------
// State wave: one stage.  bs.xs holds the stage input of the lane's body.
// Writes the next stage input (or the new substep state after stage 3) into
// bs.xs and into ring[NX], the body rotation into cs_out[NB][2] and the
// accelerations into fv_out[3 NB].
template <class T, class TP, int ST>
__device__ __forceinline__ void state_stage(const Interval<T, TP>& iv,
                                            const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                            const BodyConst<T, TP>& c, BodyRK<T>& bs, T tau,
                                            T* ring, T (*cs_out)[2], T* fv_out, int lane) {
    constexpr int st = ST;   // RK stage, known at compile time
    constexpr int NB = TP::NB, NQ = TP::NQ;
    T fv[3], cb, sb;
    body_accel<T, TP>(iv, mc, c, bs.xs, tau, fv, cb, sb);
    const T s = iv.s, h = iv.h;
    const T an = (st == 2) ? h : T(0.5) * h;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const T kk = s * (k < 3 ? bs.xs[3 + k] : fv[k - 3]);
        if constexpr (st == 0) bs.xa[k] = kk;
        else if constexpr (st == 3) bs.xa[k] += kk;
        else bs.xa[k] += T(2) * kk;
    }
    if (lane < NB) {
#pragma unroll
        for (int k = 0; k < 3; ++k) fv_out[3 * c.b + k] = fv[k];
        cs_out[c.b][0] = cb;
        cs_out[c.b][1] = sb;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if constexpr (st < 3) {
            const T kk = s * (k < 3 ? bs.xs[3 + k] : fv[k - 3]);
            bs.xs[k] = bs.xb[k] + an * kk;
        } else {
            bs.xb[k] += iv.h6 * bs.xa[k];
            bs.xs[k] = bs.xb[k];
        }
    }
    if (lane < NB) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ring[3 * c.b + k] = bs.xs[k];
            ring[NQ + 3 * c.b + k] = bs.xs[3 + k];
        }
    }
}

// ---------------------------------------------------------------------------
// Coefficient wave: Jacobian nonzeros and F~ of one stage, given its input
// state xs[NX], the body rotations cs[NB][2] and accelerations fv[3NB] from
// the state wave.  Writes cf (layout Coef<TP>) and returns, in the lanes that
// own them, the integral-row right-hand sides (cc_i on contact lanes, the
// violation row on lane 0) through ycc / yct.  With SPLIT the call contains
// one workgroup barrier; without WRITE only the integral-row integrands are
// formed (nothing is stored).
// ---------------------------------------------------------------------------
// STORES: 0 = values gathered, stored at the end in the compiler's order
// (FP32 default); 1 = the same with a scheduling fence before the stores
// (FP64 default); 2 = each value stored as soon as it is formed (fewest
// registers).
template <class T, class TP, bool SPLIT = false, bool WRITE = true, class LY = CoefDense<TP>,
          int STORES = (sizeof(T) == 8 ? 1 : 0)>
__device__ __forceinline__ void coef_stage(const Interval<T, TP>& iv,
                                           const MConst<TP::NB, TP::NJ, TP::NC>& mc,
                                           const BodyConst<T, TP>& c, const T* xs,
                                           const T (*cs)[2], const T* fv, T tau, T* cf, T& ycc,
                                           T& yct, int lane) {
    constexpr int NB = TP::NB, NQ = TP::NQ, NX = TP::NX;
    const T s = iv.s, omt = T(1) - tau;
    const int b = c.b, p = c.p;
    const T cb = cs[b][0], sb = cs[b][1];
    const T xb = xs[3 * b], yb = xs[3 * b + 1];
    const bool pt = p == 0;
    const T cp = from_parent<TP>(cb, pt), sp = from_parent<TP>(sb, pt);
    const T xp = from_parent<TP>(xb, pt), yp = from_parent<TP>(yb, pt);
    // Every lane evaluates both the joint and the contact terms (finite values
    // from zero constants where it has none) and selects; stores of lanes
    // without the datum go to the lane's TRASH slot, so the stage has no branches.
    const bool jl = c.joint, cl = c.contact;
    // joint: arms, h_x, h_y
    const T apx = cp * c.rpx - sp * c.rpy, apy = sp * c.rpx + cp * c.rpy;
    const T acx = cb * c.rcx - sb * c.rcy, acy = sb * c.rcx + cb * c.rcy;
    const T lx = omt * c.uk[1] + tau * c.uk1[1];
    const T ly = omt * c.uk[2] + tau * c.uk1[2];
    const T a0 = xp + apx - xb - acx;
    const T a1 = yp + apy - yb - acy;
    // contact: point, velocity, terrain frame, v_t, -sd
    const T ax = cb * c.rx - sb * c.ry, ay = sb * c.rx + cb * c.ry;
    const T om = xs[NQ + 3 * b + 2];
    const T Pdx = xs[NQ + 3 * b] - om * ay;
    const T Pdy = xs[NQ + 3 * b + 1] + om * ax;
    const Frame<T> f = terrain<T>(mc, xb + ax, yb + ay);
    const T ln = omt * c.ck[0] + tau * c.ck1[0];
    const T ft = (omt * c.ck[1] + tau * c.ck1[1]) - (omt * c.ck[2] + tau * c.ck1[2]);
    const T a2 = f.tx * Pdx + f.ty * Pdy;
    const T a3 = -f.sd;
    T v0, d0, v1, d1, v2, d2, v3, d3;
    sabs_d(a0, v0, d0);
    sabs_d(a1, v1, d1);
    sabs_d(a2, v2, d2);
    sabs_d(a3, v3, d3);
    // SPLIT: the stage spans two pipeline steps, split by one workgroup
    // barrier where the two halves balance best as measured: FP32 here,
    // between the smooth functions and the integrands; FP64 after the
    // integrands, before the Jacobian terms.
    if constexpr (SPLIT && sizeof(T) == 4) __syncthreads();
    // integrands (Sec. III pairs; violation: |h|_s of joints, ramp_s(-sd))
    const T lnb = T(0.5) * (c.ck[0] + c.ck1[0]);
    const T ltpb = T(0.5) * (c.ck[1] + c.ck1[1]);
    const T ltmb = T(0.5) * (c.ck[2] + c.ck1[2]);
    const T vt = a2, av = v2, dav = d2;
    const T rp = vt > T(0) ? av : T(0);
    const T rm = vt < T(0) ? av : T(0);
    const T mu = iv.prm[0];
    const T slack = mu * lnb - ltpb - ltmb;
    const bool pen = -f.sd > T(0);
    ycc = cl ? lnb * f.sd + ltpb * rp + ltmb * rm + slack * av : T(0);
    const T ctp = (jl ? v0 + v1 : T(0)) + (cl && pen ? v3 : T(0));
    if constexpr (SPLIT && sizeof(T) == 8) __syncthreads();
    // dT_b/dth_b parts: child side of the own joint, contact, parent side
    const T fx = f.tx * ft + f.nx * ln, fy = f.ty * ft + f.ny * ln;
    const T dTown = (jl ? acx * lx + acy * ly : T(0)) + (cl ? -(ax * fx + ay * fy) : T(0));
    const T dTpar = jl ? -(apx * lx + apy * ly) : T(0);
    const T dT = dTown + from_children<TP>(dTpar, b);
    // contact derivative terms
    const T gv = ltpb * (vt > T(0) ? dav : T(0)) + ltmb * (vt < T(0) ? dav : T(0)) + slack * dav;
    const T Dg = -(pen ? d3 : T(0));
    const T dtx = f.dny, dty = -f.dnx;
    const T dfx = dtx * ft + f.dnx * ln, dfy = dty * ft + f.dny * ln;
    const T dvt_px = dtx * Pdx + dty * Pdy;
    const T im = s * c.mi, ii = s * c.ii;
    // what the stores need from LDS (read after the split barrier; the rings
    // hold this stage's entries until the state wave's step t+3, after both
    // steps of the stage)
    const T ip = s * iv.iinv[p];
    T fq[3], fa[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fq[k] = xs[NQ + 3 * b + k];
        fa[k] = fv[3 * b + k];
    }
    if constexpr (WRITE) {
        // STORES = 1 (FP64 by default): all values and addresses are formed
        // first and stored in one burst, since a register overwritten right
        // after an LDS store waits until the LDS unit has read it (measured
        // faster); FP32 keeps the compiler's interleaved order (measured faster
        // there); STORES = 2 stores at once (throughput kernels).
        constexpr int NV = STORES < 2 ? 42 + LY::TORSO_COPIES : 1;
        T val[NV];
        T* ptr[NV];
        int e = 0;
        const int j = c.j, i = c.i;
        // one sink slot per lane: stores of many lanes to one LDS address serialize
        T* tr = cf + LY::TRASH + lane;
        auto put = [&](bool ok, int off, T v, int t = 0) {
            T* const a = ok ? cf + off : tr + t;
            if constexpr (STORES < 2) {
                ptr[e] = a;
                val[e] = v;
                ++e;
            } else {
                *a = v;
            }
        };
        // joint rows of the violation integrand and the joint-force torques
        put(jl, LY::jh(j, 0), s * d0);
        put(jl, LY::jh(j, 1), s * d1);
        put(jl, LY::jh(j, 2), s * (d1 * apx - d0 * apy));
        put(jl, LY::jh(j, 3), s * (d0 * acy - d1 * acx));
        put(jl, LY::gv_joint(j, 0, p, b, 0), -apy * ip);
        put(jl, LY::gv_joint(j, 0, p, b, 1), apx * ip);
        put(jl, LY::gv_joint(j, 1, p, b, 0), acy * ii);
        put(jl, LY::gv_joint(j, 1, p, b, 1), -acx * ii);
        // contact terms
        put(cl, LY::ct(i, C_AX), ax, C_AX);
        put(cl, LY::ct(i, C_AY), ay, C_AY);
        put(cl, LY::ct(i, C_FXP), dfx * im, C_FXP);
        put(cl, LY::ct(i, C_FYP), dfy * im, C_FYP);
        put(cl, LY::ct(i, C_TP), (ax * dfy - ay * dfx) * ii, C_TP);
        put(cl, LY::ct(i, C_EPX), s * (lnb * f.dsd_px + gv * dvt_px), C_EPX);
        put(cl, LY::ct(i, C_EPY), s * (lnb * f.dsd_py), C_EPY);
        put(cl, LY::ct(i, C_EXD), s * (gv * f.tx), C_EXD);
        put(cl, LY::ct(i, C_EYD), s * (gv * f.ty), C_EYD);
        put(cl, LY::ct(i, C_EOM), s * (gv * (f.ty * ax - f.tx * ay)), C_EOM);
        put(cl, LY::ct(i, C_ETH), s * (-gv * om * (f.tx * ax + f.ty * ay)), C_ETH);
        put(cl, LY::ct(i, C_ZPX), s * (Dg * f.dsd_px), C_ZPX);
        put(cl, LY::ct(i, C_ZPY), s * (Dg * f.dsd_py), C_ZPY);
        put(cl, LY::ct(i, C_JMU), s * (lnb * av), C_JMU);
        put(cl, LY::gv_contact(i, b, 0, 0), f.nx * im);
        put(cl, LY::gv_contact(i, b, 1, 0), f.ny * im);
        put(cl, LY::gv_contact(i, b, 2, 0), (ax * f.ny - ay * f.nx) * ii);
        put(cl, LY::gv_contact(i, b, 0, 1), f.tx * im);
        put(cl, LY::gv_contact(i, b, 1, 1), f.ty * im);
        put(cl, LY::gv_contact(i, b, 2, 1), (ax * f.ty - ay * f.tx) * ii);
        put(cl, LY::gv_contact(i, b, 0, 2), -f.tx * im);
        put(cl, LY::gv_contact(i, b, 1, 2), -f.ty * im);
        put(cl, LY::gv_contact(i, b, 2, 2), -(ax * f.ty - ay * f.tx) * ii);
        put(cl, LY::gc(i, 0), s * T(0.5) * (f.sd + mu * av));
        put(cl, LY::gc(i, 1), s * T(0.5) * (rp - av));
        put(cl, LY::gc(i, 2), s * T(0.5) * (rm - av));
        put(cl, LY::f(NX + i), ycc);
        // F~ (q rows: stage velocities; v rows: the state wave's accelerations),
        // dT/dth and the violation part of the lane's body
        const bool bl = lane < NB;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            put(bl, LY::f(3 * b + k), fq[k], k);
            put(bl, LY::f(NQ + 3 * b + k), fa[k], k);
        }
        const T cth = s * dT * c.ii;
        put(bl, LY::cth(b, 0), cth);
        // further copies of the torso entry (compact record: one per leg block)
#pragma unroll
        for (int q = 1; q < LY::TORSO_COPIES; ++q) put(lane == 0, LY::cth(0, q), cth, q);
        put(bl, LY::ctp(b), ctp);
        if constexpr (STORES < 2) {
            if constexpr (STORES == 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < NV; ++q) *ptr[q] = val[q];
        }
        (void)e;
    }
    // the lane's body's part of the violation row (summed by the consumers)
    yct = lane < NB ? ctp : T(0);
}

// The dilation column S on body lanes (its own column group in the latency
// layout): lane b < NB holds the six rows of body b; a foot lane holds the
// cross-complementarity row of its contact (the torso lane all of them when
// the legs have no links); every body lane integrates its part of the
// violation row.  The Jacobian product is that of the tangent lanes with the
// joint terms exchanged between parent and child lanes, plus the F~ forcing.
template <class T, class TP>
struct SLane {
    static constexpr int NCL = TP::D == 0 ? (TP::L > 0 ? TP::L : 1) : 1;   // cc rows per lane
    T zs[6], zb[6], za[6];
    T ycc[NCL], yct;
};

// Derivative of the S column on the lane's body at the stage input zs: the
// velocity rows kv, the lane's cross-complementarity rows kcc and its part of
// the violation row kct (the pose rows are s zs_v + F~, formed by the caller).
template <class T, class TP, class LY>
__device__ __forceinline__ void s_rhs(const Interval<T, TP>& iv, const BodyConst<T, TP>& c,
                                      const T (&zs)[6], const T* __restrict__ cf, int lane,
                                      T (&kv)[3], T (&kcc)[SLane<T, TP>::NCL], T& kct) {
    constexpr int NB = TP::NB, NQ = TP::NQ, NX = TP::NX, D = TP::D, L = TP::L;
    constexpr int NCL = SLane<T, TP>::NCL;
    const int b = c.b;
    const T x = zs[0], y = zs[1], th = zs[2];
    const T vx = zs[3], vy = zs[4], om = zs[5];
    kv[0] = cf[LY::f(NQ + 3 * b)];
    kv[1] = cf[LY::f(NQ + 3 * b + 1)];
    kv[2] = cf[LY::f(NQ + 3 * b + 2)] + cf[LY::cth(b)] * th;
    kct = lane < NB ? cf[LY::ctp(b)] : T(0);
#pragma unroll
    for (int l = 0; l < NCL; ++l) kcc[l] = T(0);
    if constexpr (D >= 1) {
        // own joint (this body is its child): stiffness and damping, and the
        // joint rows of the violation integrand; the parent's share of the
        // stiffness and damping torque goes back to the parent lane
        const bool pt = c.p == 0;
        const T thp = from_parent<TP>(th, pt), omp = from_parent<TP>(om, pt);
        const T xp = from_parent<TP>(x, pt), yp = from_parent<TP>(y, pt);
        T tp = T(0);
        if (c.joint) {
            const int j = c.j;
            const T dth = th - thp, dom = om - omp;
            kv[2] -= iv.kc[j][2] * dth + iv.kc[j][3] * dom;
            tp = iv.kc[j][0] * dth + iv.kc[j][1] * dom;
            kct += cf[LY::jh(j, 0)] * (xp - x) + cf[LY::jh(j, 1)] * (yp - y) +
                   cf[LY::jh(j, 2)] * thp + cf[LY::jh(j, 3)] * th;
        }
        kv[2] += from_children<TP>(tp, b);
    }
    if constexpr (L >= 1) {
#pragma unroll
        for (int l = 0; l < NCL; ++l) {
            const bool on = D >= 1 ? c.contact : (lane == 0);
            const int i = D >= 1 ? c.i : l;
            if (on) {
                auto ct = [&](int q) { return cf[LY::ct(i, q)]; };
                const T dPx = x - ct(C_AY) * th;
                const T dPy = y + ct(C_AX) * th;
                kv[0] += ct(C_FXP) * dPx;
                kv[1] += ct(C_FYP) * dPx;
                kv[2] += ct(C_TP) * dPx;
                kcc[l] = ct(C_EPX) * dPx + ct(C_EPY) * dPy + ct(C_EXD) * vx + ct(C_EYD) * vy +
                         ct(C_EOM) * om + ct(C_ETH) * th + cf[LY::f(NX + i)];
                kct += ct(C_ZPX) * dPx + ct(C_ZPY) * dPy;
            }
        }
    }
}

template <class T, class TP, int ST, class LY = CoefDense<TP>>
__device__ __forceinline__ void s_stage(const Interval<T, TP>& iv, const BodyConst<T, TP>& c,
                                        SLane<T, TP>& z, const T* __restrict__ cf, int lane) {
    constexpr int NCL = SLane<T, TP>::NCL;
    const T s = iv.s, h = iv.h;
    const int b = c.b;
    T kv[3], kcc[NCL], kct;
    s_rhs<T, TP, LY>(iv, c, z.zs, cf, lane, kv, kcc, kct);
    // classical RK4 combination (stage ST known at compile time)
    constexpr int WK = (ST == 0 || ST == 3) ? 1 : 2;
    const T an = (ST == 2) ? h : T(0.5) * h;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T kq = s * z.zs[3 + k] + cf[LY::f(3 * b + k)];
        if (ST == 0) z.za[k] = kq;
        else z.za[k] += T(WK) * kq;
        if (ST < 3) z.zs[k] = z.zb[k] + an * kq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (ST == 0) z.za[3 + k] = kv[k];
        else z.za[3 + k] += T(WK) * kv[k];
        if (ST < 3) z.zs[3 + k] = z.zb[3 + k] + an * kv[k];
    }
    const T h6 = iv.h6;
#pragma unroll
    for (int l = 0; l < NCL; ++l) z.ycc[l] += (h6 * T(WK)) * kcc[l];
    z.yct += (h6 * T(WK)) * kct;
    if (ST == 3) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            z.zb[r] += h6 * z.za[r];
            z.zs[r] = z.zb[r];
        }
    }
}

}  // namespace cis
