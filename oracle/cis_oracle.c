/*
 * CPU FP64 oracle for the CI-SCvx interval linearize-and-discretize step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * Plain, slow and dense on purpose: the right-hand side, its Jacobians (filled
 * entry by entry from hand-derived formulas), classical RK4 with the
 * variational equations on dense matrices, the same for any explicit
 * Runge-Kutta tableau (the Fehlberg 4(5) pair of the paper's transcription),
 * the reverse sweep of the discrete map, and forward parameter
 * sensitivities.  Every quantity is double.
 *
 * What it follows (arxiv 2604.09993):
 *  - planar maximal-coordinate dynamics  q' = v,  M v' = W + J^T R phi + grad h^T lambda
 *    (Sec. II-A, eq. ct-dynamics), M = diag(m, m, I) per body;
 *  - contact frame R = [t n], n the unit surface normal, sd the signed distance,
 *    approximated on a sinusoid by h/||grad h|| (Sec. II, Sec. VI-B);
 *  - pseudo-Huber smooth abs and ramp with unit steepness (Sec. II notation);
 *  - integral cross-complementarity states and the continuous-time constraint
 *    violation state (Sec. III, Prop. 1 and eq. aux-dynamics; Sec. IV-A);
 *  - time-dilated augmented system x~' = s (f, Omega) on tau in [0, 1]
 *    (Sec. IV-B, eq. aug-dynamics) with first-order-hold controls and its
 *    integral form (eq. intg-aug-sys-param);
 *  - internal numerical differentiation: the sensitivities are the exact
 *    derivatives of the discrete integrator (Sec. VI, transcription).
 *
 * Readings where the paper is silent (each documented with the design notes):
 *  joint forces and split friction [lam_n, lam_t+, lam_t-] are controls; one
 *  cross-complementarity state per contact whose integrand multiplies the
 *  interval-mean forces with the state functions sd, ramp_s(+-v_t), abs_s(v_t);
 *  one constraint-violation state summing ramp_s(-sd) and abs_s(h) over joints;
 *  classical RK4 with K uniform substeps; I_b = m_b L_b^2 / 12; +tau on the
 *  child, -tau on the parent; stage times (j + c_i)/K.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nb, nj, nc;
    const double *len;        /* [nb] link length (inertia of a slender rod) */
    const int *jp, *jc;       /* [nj] parent / child body of each revolute joint */
    const double *rp, *rc;    /* [nj][2] joint anchor in parent / child body frame */
    const double *kst, *dmp;  /* [nj] joint stiffness and damping */
    const int *cb;            /* [nc] body carrying contact i */
    const double *cr;         /* [nc][2] contact point in that body's frame */
    double g, A, kappa;       /* gravity; terrain h(P) = P_y - A sin(kappa P_x) */
} omodel;

/* ---- sizes and index maps (state x~ = (q, v, y_cc, y_ctcs)) ---------------- */
static int o_n(const omodel *M) { return 6 * M->nb; }
static int o_nx(const omodel *M) { return 6 * M->nb + M->nc + 1; }
static int o_m(const omodel *M) { return 3 * M->nj + 3 * M->nc; }
static int o_np(const omodel *M) { return M->nb + 2; }
static int IQ(const omodel *M, int b, int k) { (void)M; return 3 * b + k; }
static int IV(const omodel *M, int b, int k) { return 3 * M->nb + 3 * b + k; }
static int ICC(const omodel *M, int i) { return 6 * M->nb + i; }
static int ICT(const omodel *M) { return 6 * M->nb + M->nc; }
static int UTAU(const omodel *M, int j) { (void)M; return j; }
static int ULAM(const omodel *M, int j, int a) { return M->nj + 2 * j + a; }
static int UCN(const omodel *M, int i) { return 3 * M->nj + 3 * i; }
static int UCP(const omodel *M, int i) { return 3 * M->nj + 3 * i + 1; }
static int UCM(const omodel *M, int i) { return 3 * M->nj + 3 * i + 2; }

int oracle_dims(const omodel *M, int *n, int *nx, int *m, int *np) {
    *n = o_n(M); *nx = o_nx(M); *m = o_m(M); *np = o_np(M);
    return 0;
}

/* ---- pseudo-Huber functions with unit steepness (Sec. II notation) --------
 * |a|_s = sqrt(a^2 + 1) - 1, written in the cancellation-free form
 * a^2 / (sqrt(a^2 + 1) + 1);  ramp_s(a) = |a|_s for a > 0, else 0.          */
static double sabs(double a) { return a * a / (sqrt(a * a + 1.0) + 1.0); }
static double dsabs(double a) { return a / sqrt(a * a + 1.0); }
static double sramp(double a) { return a > 0.0 ? sabs(a) : 0.0; }
static double dsramp(double a) { return a > 0.0 ? dsabs(a) : 0.0; }

static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

/* Per-contact terrain quantities at the contact point P (Sec. II contact frame,
 * Sec. VI-B signed-distance approximation sd = h / ||grad h||).             */
typedef struct {
    double sd, nx, ny, tx, ty;         /* signed distance, normal, tangent   */
    double dsd_px, dsd_py;             /* d sd / d P                          */
    double dnx_px, dny_px, dtx_px, dty_px;  /* d n / d P_x, d t / d P_x       */
} terrain_t;

static void terrain_eval(const omodel *M, double px, double py, terrain_t *T) {
    double w = M->kappa * px;
    double H = py - M->A * sin(w);
    double Hx = -M->A * M->kappa * cos(w);           /* d h / d P_x          */
    double Hxx = M->A * M->kappa * M->kappa * sin(w); /* d^2 h / d P_x^2     */
    double G = sqrt(1.0 + Hx * Hx);
    double G3 = G * G * G;
    T->sd = H / G;
    T->nx = Hx / G;
    T->ny = 1.0 / G;
    T->tx = T->ny;             /* t = (n_y, -n_x): [t n] is right-handed     */
    T->ty = -T->nx;
    T->dsd_px = Hx / G - H * Hx * Hxx / G3;
    T->dsd_py = 1.0 / G;
    T->dnx_px = Hxx / G3;
    T->dny_px = -Hx * Hxx / G3;
    T->dtx_px = T->dny_px;
    T->dty_px = -T->dnx_px;
}

/*
 * Right-hand side F~(x~, u, ubar; p) of the augmented system before dilation:
 * F~ = (v, M^{-1}(W + contact + joint forces), Omega_cc, Omega_ctcs).
 * u is the control at the stage time, ubar the interval mean of the FOH
 * control (used by the cross-complementarity integrand).
 * If Jx / Ju / Jub / Jp are non-NULL they receive the dense Jacobians
 * dF~/dx~ [nx][nx], dF~/du [nx][m], dF~/dubar [nx][m], dF~/dp [nx][np]
 * (row-major), derived by hand term by term.
 */
void oracle_rhs_jac(const omodel *M, const double *x, const double *u, const double *ub,
                    const double *p, double *F, double *Jx, double *Ju, double *Jub,
                    double *Jp) {
    const int nb = M->nb, nj = M->nj, nc = M->nc;
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
    const double mu = p[0];
    double *Fx = calloc(nb, sizeof(double)), *Fy = calloc(nb, sizeof(double));
    double *Tq = calloc(nb, sizeof(double));
    /* generalized force Jacobians (force / torque on each body) */
    double *dF = NULL, *dFu = NULL;   /* [3 nb][nx], [3 nb][m]: (Fx, Fy, T) rows */
    if (Jx) dF = calloc((size_t)3 * nb * nx, sizeof(double));
    if (Ju) dFu = calloc((size_t)3 * nb * m, sizeof(double));
#define DF(b, k, col) dF[(size_t)(3 * (b) + (k)) * nx + (col)]
#define DFU(b, k, col) dFu[(size_t)(3 * (b) + (k)) * m + (col)]
#define JX(r, c) Jx[(size_t)(r) * nx + (c)]
#define JU(r, c) Ju[(size_t)(r) * m + (c)]
#define JUB(r, c) Jub[(size_t)(r) * m + (c)]
#define JP(r, c) Jp[(size_t)(r) * np + (c)]
    if (Jx) memset(Jx, 0, sizeof(double) * nx * nx);
    if (Ju) memset(Ju, 0, sizeof(double) * nx * m);
    if (Jub) memset(Jub, 0, sizeof(double) * nx * m);
    if (Jp) memset(Jp, 0, sizeof(double) * nx * np);
    double ctcs = 0.0;

    /* kinematic rates q' = v */
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k) {
            F[IQ(M, b, k)] = x[IV(M, b, k)];
            if (Jx) JX(IQ(M, b, k), IV(M, b, k)) = 1.0;
        }

    /* revolute joints: world-frame reaction force lam applied +lam to the
     * parent at its anchor and -lam to the child at its anchor (grad h^T lam);
     * actuation plus stiffness/damping torque +1x child, -1x parent.        */
    for (int j = 0; j < nj; ++j) {
        int pb = M->jp[j], cbd = M->jc[j];
        double thp = x[IQ(M, pb, 2)], thc = x[IQ(M, cbd, 2)];
        double cp = cos(thp), sp = sin(thp), cc = cos(thc), sc = sin(thc);
        double apx = cp * M->rp[2 * j] - sp * M->rp[2 * j + 1];
        double apy = sp * M->rp[2 * j] + cp * M->rp[2 * j + 1];
        double acx = cc * M->rc[2 * j] - sc * M->rc[2 * j + 1];
        double acy = sc * M->rc[2 * j] + cc * M->rc[2 * j + 1];
        double hx = x[IQ(M, pb, 0)] + apx - x[IQ(M, cbd, 0)] - acx;
        double hy = x[IQ(M, pb, 1)] + apy - x[IQ(M, cbd, 1)] - acy;
        double lx = u[ULAM(M, j, 0)], ly = u[ULAM(M, j, 1)];
        double k = M->kst[j], d = M->dmp[j];
        double tsd = -k * (thc - thp) - d * (x[IV(M, cbd, 2)] - x[IV(M, pb, 2)]);
        double tt = u[UTAU(M, j)] + tsd;
        Fx[pb] += lx; Fy[pb] += ly;
        Tq[pb] += cross2(apx, apy, lx, ly) - tt;
        Fx[cbd] -= lx; Fy[cbd] -= ly;
        Tq[cbd] += -cross2(acx, acy, lx, ly) + tt;
        ctcs += sabs(hx) + sabs(hy);
        if (Jx) {
            /* d(a x lam)/d theta = (E a) x lam = -(a . lam) */
            DF(pb, 2, IQ(M, pb, 2)) += -(apx * lx + apy * ly);
            DF(cbd, 2, IQ(M, cbd, 2)) += (acx * lx + acy * ly);
            /* stiffness / damping: -tt on parent, +tt on child */
            DF(pb, 2, IQ(M, cbd, 2)) += k;   DF(pb, 2, IQ(M, pb, 2)) += -k;
            DF(pb, 2, IV(M, cbd, 2)) += d;   DF(pb, 2, IV(M, pb, 2)) += -d;
            DF(cbd, 2, IQ(M, cbd, 2)) += -k; DF(cbd, 2, IQ(M, pb, 2)) += k;
            DF(cbd, 2, IV(M, cbd, 2)) += -d; DF(cbd, 2, IV(M, pb, 2)) += d;
            /* constraint-violation integrand |h_x|_s + |h_y|_s */
            double gx = dsabs(hx), gy = dsabs(hy);
            int r = ICT(M);
            JX(r, IQ(M, pb, 0)) += gx;  JX(r, IQ(M, cbd, 0)) -= gx;
            JX(r, IQ(M, pb, 1)) += gy;  JX(r, IQ(M, cbd, 1)) -= gy;
            JX(r, IQ(M, pb, 2)) += gx * (-apy) + gy * apx;
            JX(r, IQ(M, cbd, 2)) += gx * acy + gy * (-acx);
        }
        if (Ju) {
            DFU(pb, 0, ULAM(M, j, 0)) += 1.0;  DFU(pb, 1, ULAM(M, j, 1)) += 1.0;
            DFU(cbd, 0, ULAM(M, j, 0)) -= 1.0; DFU(cbd, 1, ULAM(M, j, 1)) -= 1.0;
            DFU(pb, 2, ULAM(M, j, 0)) += -apy; DFU(pb, 2, ULAM(M, j, 1)) += apx;
            DFU(cbd, 2, ULAM(M, j, 0)) += acy; DFU(cbd, 2, ULAM(M, j, 1)) += -acx;
            DFU(pb, 2, UTAU(M, j)) += -1.0;    DFU(cbd, 2, UTAU(M, j)) += 1.0;
        }
    }

    /* contacts: force F = t (lam_t+ - lam_t-) + n lam_n applied at P_i */
    for (int i = 0; i < nc; ++i) {
        int b = M->cb[i];
        double th = x[IQ(M, b, 2)], c = cos(th), s = sin(th);
        double ax = c * M->cr[2 * i] - s * M->cr[2 * i + 1];
        double ay = s * M->cr[2 * i] + c * M->cr[2 * i + 1];
        double Px = x[IQ(M, b, 0)] + ax, Py = x[IQ(M, b, 1)] + ay;
        double om = x[IV(M, b, 2)];
        double Pdx = x[IV(M, b, 0)] - om * ay, Pdy = x[IV(M, b, 1)] + om * ax;
        terrain_t T;
        terrain_eval(M, Px, Py, &T);
        double ln = u[UCN(M, i)], ltp = u[UCP(M, i)], ltm = u[UCM(M, i)];
        double ft = ltp - ltm;
        double fx = T.tx * ft + T.nx * ln, fy = T.ty * ft + T.ny * ln;
        Fx[b] += fx; Fy[b] += fy;
        Tq[b] += cross2(ax, ay, fx, fy);
        double vt = T.tx * Pdx + T.ty * Pdy;
        double lnb = ub[UCN(M, i)], ltpb = ub[UCP(M, i)], ltmb = ub[UCM(M, i)];
        double slack = mu * lnb - ltpb - ltmb;
        F[ICC(M, i)] = lnb * T.sd + ltpb * sramp(vt) + ltmb * sramp(-vt) + slack * sabs(vt);
        ctcs += sramp(-T.sd);
        /* partial derivatives of P, Pdot w.r.t. the body state */
        /* dP/dx = (1,0), dP/dy = (0,1), dP/dth = (-ay, ax)
         * dPdot/dxd = (1,0), dPdot/dyd = (0,1), dPdot/dom = (-ay, ax),
         * dPdot/dth = om (-ax, -ay)                                          */
        double dfx_px = T.dtx_px * ft + T.dnx_px * ln;
        double dfy_px = T.dty_px * ft + T.dny_px * ln;
        double dvt_px = T.dtx_px * Pdx + T.dty_px * Pdy;
        if (Jx) {
            int cx = IQ(M, b, 0), cy = IQ(M, b, 1), cth = IQ(M, b, 2);
            int cxd = IV(M, b, 0), cyd = IV(M, b, 1), com = IV(M, b, 2);
            /* force on body b via P_x (terrain frame rotates with P_x) */
            DF(b, 0, cx) += dfx_px;          DF(b, 1, cx) += dfy_px;
            DF(b, 0, cth) += dfx_px * (-ay); DF(b, 1, cth) += dfy_px * (-ay);
            /* torque a x F */
            double dT_px = cross2(ax, ay, dfx_px, dfy_px);
            DF(b, 2, cx) += dT_px;
            DF(b, 2, cth) += -(ax * fx + ay * fy) + dT_px * (-ay);
            /* v_t = t(P_x) . Pdot */
            double dvt_x = dvt_px, dvt_th = dvt_px * (-ay) + om * (T.tx * (-ax) + T.ty * (-ay));
            double dvt_xd = T.tx, dvt_yd = T.ty, dvt_om = T.tx * (-ay) + T.ty * ax;
            /* sd(P) */
            double dsd_x = T.dsd_px, dsd_y = T.dsd_py, dsd_th = T.dsd_px * (-ay) + T.dsd_py * ax;
            double gv = ltpb * dsramp(vt) - ltmb * dsramp(-vt) + slack * dsabs(vt);
            int r = ICC(M, i);
            JX(r, cx) += lnb * dsd_x + gv * dvt_x;
            JX(r, cy) += lnb * dsd_y;
            JX(r, cth) += lnb * dsd_th + gv * dvt_th;
            JX(r, cxd) += gv * dvt_xd;
            JX(r, cyd) += gv * dvt_yd;
            JX(r, com) += gv * dvt_om;
            /* d ramp_s(-sd)/d sd = -ramp_s'(-sd) */
            double gs = -dsramp(-T.sd);
            int rc = ICT(M);
            JX(rc, cx) += gs * dsd_x;
            JX(rc, cy) += gs * dsd_y;
            JX(rc, cth) += gs * dsd_th;
        }
        if (Ju) {
            DFU(b, 0, UCN(M, i)) += T.nx;  DFU(b, 1, UCN(M, i)) += T.ny;
            DFU(b, 0, UCP(M, i)) += T.tx;  DFU(b, 1, UCP(M, i)) += T.ty;
            DFU(b, 0, UCM(M, i)) -= T.tx;  DFU(b, 1, UCM(M, i)) -= T.ty;
            DFU(b, 2, UCN(M, i)) += cross2(ax, ay, T.nx, T.ny);
            DFU(b, 2, UCP(M, i)) += cross2(ax, ay, T.tx, T.ty);
            DFU(b, 2, UCM(M, i)) -= cross2(ax, ay, T.tx, T.ty);
        }
        if (Jub) {
            int r = ICC(M, i);
            JUB(r, UCN(M, i)) += T.sd + mu * sabs(vt);
            JUB(r, UCP(M, i)) += sramp(vt) - sabs(vt);
            JUB(r, UCM(M, i)) += sramp(-vt) - sabs(vt);
        }
        if (Jp) JP(ICC(M, i), 0) += lnb * sabs(vt);
    }
    F[ICT(M)] = ctcs;

    /* accelerations v' = M^{-1} (forces) - g e_y, M = diag(m, m, I) */
    for (int b = 0; b < nb; ++b) {
        double mb = p[2 + b];
        double Ib = mb * M->len[b] * M->len[b] / 12.0;
        F[IV(M, b, 0)] = Fx[b] / mb;
        F[IV(M, b, 1)] = Fy[b] / mb - M->g;
        F[IV(M, b, 2)] = Tq[b] / Ib;
        if (Jx)
            for (int col = 0; col < nx; ++col) {
                JX(IV(M, b, 0), col) += DF(b, 0, col) / mb;
                JX(IV(M, b, 1), col) += DF(b, 1, col) / mb;
                JX(IV(M, b, 2), col) += DF(b, 2, col) / Ib;
            }
        if (Ju)
            for (int col = 0; col < m; ++col) {
                JU(IV(M, b, 0), col) += DFU(b, 0, col) / mb;
                JU(IV(M, b, 1), col) += DFU(b, 1, col) / mb;
                JU(IV(M, b, 2), col) += DFU(b, 2, col) / Ib;
            }
        if (Jp) {
            /* d/dm (F/m) = -F/m^2 ; d/dm (T/I) = -T/(I m) since I is linear in m */
            JP(IV(M, b, 0), 2 + b) += -Fx[b] / (mb * mb);
            JP(IV(M, b, 1), 2 + b) += -Fy[b] / (mb * mb);
            JP(IV(M, b, 2), 2 + b) += -Tq[b] / (Ib * mb);
        }
    }
    free(Fx); free(Fy); free(Tq); free(dF); free(dFu);
#undef DF
#undef DFU
#undef JX
#undef JU
#undef JUB
#undef JP
}

/* C = A (r x k) * B (k x c), row-major, plain triple loop */
static void matmul(int r, int k, int c, const double *A, const double *B, double *C) {
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double acc = 0.0;
            for (int l = 0; l < k; ++l) acc += A[(size_t)i * k + l] * B[(size_t)l * c + j];
            C[(size_t)i * c + j] = acc;
        }
}

static const double RK_C[4] = {0.0, 0.5, 0.5, 1.0};   /* stage nodes            */
static const double RK_A[4] = {0.0, 0.5, 0.5, 1.0};   /* stage-input multipliers */
static const double RK_W[4] = {1.0, 2.0, 2.0, 1.0};   /* weights (times h/6)     */

/*
 * Classical RK4 of the time-dilated augmented system on [tau0, tau1] with K
 * uniform steps, together with the variational equations (IND, Sec. VI):
 *   Phi' = s J_x Phi,  Phi(tau0) = I                         (full nx x nx)
 *   Bm'  = s J_x Bm + s (J_u (1 - tau) + J_ubar / 2)
 *   Bp'  = s J_x Bp + s (J_u tau + J_ubar / 2)
 *   Sv'  = s J_x Sv + F~
 *   Pi'  = s J_x Pi + s J_p                                   (if Pi != NULL)
 * where u(tau) = (1 - tau) Uk + tau Uk1 and ubar = (Uk + Uk1)/2 (FOH, Sec. IV-B)
 * and every Jacobian is evaluated at the stage state, so the sensitivities
 * are the exact derivatives of the discrete RK4 map.
 * Outputs may be NULL except xf.
 */
void oracle_integrate(const omodel *M, const double *x0, const double *Uk, const double *Uk1,
                      double s, const double *p, double tau0, double tau1, int K,
                      double *xf, double *Phi, double *Bm, double *Bp, double *Sv, double *Pi) {
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
    /* tangent matrix Z = [Phi | Bm | Bp | Sv | Pi], nx rows, nz columns */
    const int nz = nx + 2 * m + 1 + np;
    const int oB = nx, oP = nx + m, oS = nx + 2 * m, oPi = nx + 2 * m + 1;
    const double h = (tau1 - tau0) / K;
    double *x = malloc(sizeof(double) * nx), *xs = malloc(sizeof(double) * nx);
    double *xacc = malloc(sizeof(double) * nx), *kx = malloc(sizeof(double) * nx);
    double *Z = calloc((size_t)nx * nz, sizeof(double)), *Zs = malloc(sizeof(double) * nx * nz);
    double *Zacc = malloc(sizeof(double) * nx * nz), *KZ = malloc(sizeof(double) * nx * nz);
    double *Jx = malloc(sizeof(double) * nx * nx), *Ju = malloc(sizeof(double) * nx * m);
    double *Jub = malloc(sizeof(double) * nx * m), *Jp = malloc(sizeof(double) * nx * np);
    double *u = malloc(sizeof(double) * (m + 1)), *ub = malloc(sizeof(double) * (m + 1));
    for (int r = 0; r < nx; ++r) { x[r] = x0[r]; Z[(size_t)r * nz + r] = 1.0; }
    for (int c = 0; c < m; ++c) ub[c] = 0.5 * (Uk[c] + Uk1[c]);
    for (int j = 0; j < K; ++j) {
        memcpy(xs, x, sizeof(double) * nx);
        memcpy(Zs, Z, sizeof(double) * nx * nz);
        memset(xacc, 0, sizeof(double) * nx);
        memset(Zacc, 0, sizeof(double) * nx * nz);
        for (int st = 0; st < 4; ++st) {
            double tau = tau0 + (j + RK_C[st]) * (tau1 - tau0) / K;
            if (st > 0) {
                for (int r = 0; r < nx; ++r) xs[r] = x[r] + h * RK_A[st] * kx[r];
                for (size_t e = 0; e < (size_t)nx * nz; ++e) Zs[e] = Z[e] + h * RK_A[st] * KZ[e];
            }
            for (int c = 0; c < m; ++c) u[c] = (1.0 - tau) * Uk[c] + tau * Uk1[c];
            double *Fv = kx;  /* reuse: F~ at the stage */
            oracle_rhs_jac(M, xs, u, ub, p, Fv, Jx, Ju, Jub, Jp);
            /* tangent derivative: KZ = s Jx Zs + forcing */
            matmul(nx, nx, nz, Jx, Zs, KZ);
            for (size_t e = 0; e < (size_t)nx * nz; ++e) KZ[e] *= s;
            for (int r = 0; r < nx; ++r) {
                for (int c = 0; c < m; ++c) {
                    KZ[(size_t)r * nz + oB + c] += s * (Ju[(size_t)r * m + c] * (1.0 - tau) + 0.5 * Jub[(size_t)r * m + c]);
                    KZ[(size_t)r * nz + oP + c] += s * (Ju[(size_t)r * m + c] * tau + 0.5 * Jub[(size_t)r * m + c]);
                }
                KZ[(size_t)r * nz + oS] += Fv[r];
                for (int c = 0; c < np; ++c) KZ[(size_t)r * nz + oPi + c] += s * Jp[(size_t)r * np + c];
            }
            for (int r = 0; r < nx; ++r) kx[r] = s * Fv[r];
            for (int r = 0; r < nx; ++r) xacc[r] += RK_W[st] * kx[r];
            for (size_t e = 0; e < (size_t)nx * nz; ++e) Zacc[e] += RK_W[st] * KZ[e];
        }
        for (int r = 0; r < nx; ++r) x[r] += h / 6.0 * xacc[r];
        for (size_t e = 0; e < (size_t)nx * nz; ++e) Z[e] += h / 6.0 * Zacc[e];
    }
    memcpy(xf, x, sizeof(double) * nx);
    for (int r = 0; r < nx; ++r) {
        if (Phi) for (int c = 0; c < nx; ++c) Phi[(size_t)r * nx + c] = Z[(size_t)r * nz + c];
        if (Bm) for (int c = 0; c < m; ++c) Bm[(size_t)r * m + c] = Z[(size_t)r * nz + oB + c];
        if (Bp) for (int c = 0; c < m; ++c) Bp[(size_t)r * m + c] = Z[(size_t)r * nz + oP + c];
        if (Sv) Sv[r] = Z[(size_t)r * nz + oS];
        if (Pi) for (int c = 0; c < np; ++c) Pi[(size_t)r * np + c] = Z[(size_t)r * nz + oPi + c];
    }
    free(x); free(xs); free(xacc); free(kx); free(Z); free(Zs); free(Zacc); free(KZ);
    free(Jx); free(Ju); free(Jub); free(Jp); free(u); free(ub);
}

/*
 * Multiple shooting over N intervals (Sec. VI: intervals are independent given
 * the node variables).  Node-major arrays: X[N+1][nx], U[N+1][m], s[N].
 * Outputs per interval k (any may be NULL): A[N][nx][nx], Bm/Bp[N][nx][m],
 * S[N][nx], defect d_k = F~_k - X_{k+1} [N][nx], xprop F~_k [N][nx],
 * Pi (parameter sensitivities) [N][nx][np].
 */
int oracle_discretize(const omodel *M, int N, int K, const double *X, const double *U,
                      const double *s, const double *p, double *A, double *Bm, double *Bp,
                      double *S, double *defect, double *xprop, double *Pi, int nthreads) {
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int k = 0; k < N; ++k) {
        double *xf = malloc(sizeof(double) * nx);
        oracle_integrate(M, X + (size_t)k * nx, U + (size_t)k * m, U + (size_t)(k + 1) * m, s[k], p,
                         0.0, 1.0, K, xf,
                         A ? A + (size_t)k * nx * nx : NULL,
                         Bm ? Bm + (size_t)k * nx * m : NULL,
                         Bp ? Bp + (size_t)k * nx * m : NULL,
                         S ? S + (size_t)k * nx : NULL,
                         Pi ? Pi + (size_t)k * nx * np : NULL);
        for (int r = 0; r < nx; ++r) {
            if (xprop) xprop[(size_t)k * nx + r] = xf[r];
            if (defect) defect[(size_t)k * nx + r] = xf[r] - X[(size_t)(k + 1) * nx + r];
        }
        free(xf);
    }
    return 0;
}

/* Forward pass without sensitivities: xprop and defects only. */
int oracle_defects(const omodel *M, int N, int K, const double *X, const double *U,
                   const double *s, const double *p, double *defect, double *xprop, int nthreads) {
    const int nx = o_nx(M), m = o_m(M);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int k = 0; k < N; ++k) {
        double *xf = malloc(sizeof(double) * nx);
        oracle_integrate(M, X + (size_t)k * nx, U + (size_t)k * m, U + (size_t)(k + 1) * m, s[k], p,
                         0.0, 1.0, K, xf, NULL, NULL, NULL, NULL, NULL);
        for (int r = 0; r < nx; ++r) {
            if (xprop) xprop[(size_t)k * nx + r] = xf[r];
            if (defect) defect[(size_t)k * nx + r] = xf[r] - X[(size_t)(k + 1) * nx + r];
        }
        free(xf);
    }
    return 0;
}

/*
 * Reverse sweep (vector-Jacobian product) of the discrete RK4 map of one
 * interval on [0, 1]: given lam = dJ/dF~_k, returns
 *   xbar = (dF~_k/dx0)^T lam, ukbar / uk1bar = (dF~_k/dU_k)^T lam, (dF~_k/dU_k+1)^T lam,
 *   sbar = (dF~_k/ds)^T lam, pbar += (dF~_k/dp)^T lam.
 * Stage states are stored for the whole interval (no checkpointing here).
 */
static void adjoint_interval(const omodel *M, const double *x0, const double *Uk,
                             const double *Uk1, double s, const double *p, int K,
                             const double *lam, double *xbar, double *ukbar, double *uk1bar,
                             double *sbar, double *pbar) {
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
    const double h = 1.0 / K;
    double *stage = malloc(sizeof(double) * (size_t)K * 4 * nx);  /* stage states */
    double *kst = malloc(sizeof(double) * (size_t)4 * nx);
    double *x = malloc(sizeof(double) * nx), *xs = malloc(sizeof(double) * nx);
    double *F = malloc(sizeof(double) * nx);
    double *Jx = malloc(sizeof(double) * nx * nx), *Ju = malloc(sizeof(double) * nx * m);
    double *Jub = malloc(sizeof(double) * nx * m), *Jp = malloc(sizeof(double) * nx * np);
    double *u = malloc(sizeof(double) * (m + 1)), *ub = malloc(sizeof(double) * (m + 1));
    double *xb = malloc(sizeof(double) * nx), *kb = malloc(sizeof(double) * nx);
    double *Xb = malloc(sizeof(double) * nx), *Xsum = malloc(sizeof(double) * nx);
    for (int c = 0; c < m; ++c) ub[c] = 0.5 * (Uk[c] + Uk1[c]);
    /* forward: record the 4 stage states of every step */
    memcpy(x, x0, sizeof(double) * nx);
    for (int j = 0; j < K; ++j) {
        for (int st = 0; st < 4; ++st) {
            double tau = (j + RK_C[st]) / K;
            for (int r = 0; r < nx; ++r)
                xs[r] = st == 0 ? x[r] : x[r] + h * RK_A[st] * kst[(size_t)(st - 1) * nx + r];
            memcpy(stage + ((size_t)j * 4 + st) * nx, xs, sizeof(double) * nx);
            for (int c = 0; c < m; ++c) u[c] = (1.0 - tau) * Uk[c] + tau * Uk1[c];
            oracle_rhs_jac(M, xs, u, ub, p, F, NULL, NULL, NULL, NULL);
            for (int r = 0; r < nx; ++r) kst[(size_t)st * nx + r] = s * F[r];
        }
        for (int r = 0; r < nx; ++r)
            x[r] += h / 6.0 * (kst[r] + 2.0 * kst[nx + r] + 2.0 * kst[2 * nx + r] + kst[3 * nx + r]);
    }
    /* reverse */
    for (int r = 0; r < nx; ++r) xb[r] = lam[r];
    for (int c = 0; c < m; ++c) { ukbar[c] = 0.0; uk1bar[c] = 0.0; }
    *sbar = 0.0;
    for (int j = K - 1; j >= 0; --j) {
        memset(Xsum, 0, sizeof(double) * nx);
        memset(Xb, 0, sizeof(double) * nx);   /* adjoint of the later stage's input */
        for (int st = 3; st >= 0; --st) {
            double tau = (j + RK_C[st]) / K;
            /* kbar_st = h/6 w_st xbar_{j+1} + h a_{st+1} Xbar_{st+1} */
            for (int r = 0; r < nx; ++r)
                kb[r] = h / 6.0 * RK_W[st] * xb[r] + (st < 3 ? h * RK_A[st + 1] * Xb[r] : 0.0);
            const double *xsr = stage + ((size_t)j * 4 + st) * nx;
            for (int c = 0; c < m; ++c) u[c] = (1.0 - tau) * Uk[c] + tau * Uk1[c];
            oracle_rhs_jac(M, xsr, u, ub, p, F, Jx, Ju, Jub, Jp);
            /* Xbar_st = s Jx^T kbar */
            for (int c = 0; c < nx; ++c) {
                double acc = 0.0;
                for (int r = 0; r < nx; ++r) acc += Jx[(size_t)r * nx + c] * kb[r];
                Xb[c] = s * acc;
            }
            for (int c = 0; c < m; ++c) {
                double au = 0.0, aub = 0.0;
                for (int r = 0; r < nx; ++r) {
                    au += Ju[(size_t)r * m + c] * kb[r];
                    aub += Jub[(size_t)r * m + c] * kb[r];
                }
                ukbar[c] += s * (au * (1.0 - tau) + 0.5 * aub);
                uk1bar[c] += s * (au * tau + 0.5 * aub);
            }
            double sf = 0.0;
            for (int r = 0; r < nx; ++r) sf += F[r] * kb[r];
            *sbar += sf;
            for (int c = 0; c < np; ++c) {
                double acc = 0.0;
                for (int r = 0; r < nx; ++r) acc += Jp[(size_t)r * np + c] * kb[r];
                pbar[c] += s * acc;
            }
            for (int r = 0; r < nx; ++r) Xsum[r] += Xb[r];
        }
        for (int r = 0; r < nx; ++r) xb[r] += Xsum[r];
    }
    memcpy(xbar, xb, sizeof(double) * nx);
    free(stage); free(kst); free(x); free(xs); free(F); free(Jx); free(Ju); free(Jub); free(Jp);
    free(u); free(ub); free(xb); free(kb); free(Xb); free(Xsum);
}

/*
 * Gradients of J with seed lam_k = dJ/dF~_k [N][nx] (node-major):
 *   gX_k = (dF~_k/dX_k)^T lam_k for k < N, gX_N = 0;
 *   gU_k = (dF~_k/dU_k)^T lam_k + (dF~_{k-1}/dU_k)^T lam_{k-1};
 *   gs_k = (dF~_k/ds_k)^T lam_k;  gp = sum_k (dF~_k/dp)^T lam_k (summed in k order).
 */
int oracle_adjoint(const omodel *M, int N, int K, const double *X, const double *U,
                   const double *s, const double *p, const double *lam, double *gX, double *gU,
                   double *gs, double *gp, int nthreads) {
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
    double *ukb = calloc((size_t)N * m + 1, sizeof(double));
    double *uk1b = calloc((size_t)N * m + 1, sizeof(double));
    double *pb = calloc((size_t)N * np, sizeof(double));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int k = 0; k < N; ++k) {
        adjoint_interval(M, X + (size_t)k * nx, U + (size_t)k * m, U + (size_t)(k + 1) * m, s[k], p, K,
                         lam + (size_t)k * nx, gX + (size_t)k * nx, ukb + (size_t)k * m,
                         uk1b + (size_t)k * m, gs + k, pb + (size_t)k * np);
    }
    for (int r = 0; r < nx; ++r) gX[(size_t)N * nx + r] = 0.0;
    for (int k = 0; k <= N; ++k)
        for (int c = 0; c < m; ++c)
            gU[(size_t)k * m + c] = (k < N ? ukb[(size_t)k * m + c] : 0.0) +
                                    (k > 0 ? uk1b[(size_t)(k - 1) * m + c] : 0.0);
    for (int c = 0; c < np; ++c) {
        double acc = 0.0;
        for (int k = 0; k < N; ++k) acc += pb[(size_t)k * np + c];
        gp[c] = acc;
    }
    free(ukb); free(uk1b); free(pb);
    return 0;
}

/* ==========================================================================
 * Runge-Kutta-Fehlberg transcription (Sec. VI: the custom Runge-Kutta-Fehlberg
 * integrator with internal numerical differentiation, a fixed number of steps
 * per interval).
 *
 * Any explicit Runge-Kutta method with a strictly lower-triangular tableau
 * (stage nodes c_i, coefficients a_ij, weights b_i and, optionally, embedded
 * weights bh_i):
 *     K_i = h F~(tau_j + c_i h, x_j + h sum_{l<i} a_il K_l)   (here h = 1/K on tau)
 *     x_{j+1} = x_j + sum_i b_i K_i,   e_j = sum_i (bh_i - b_i) K_i
 * with the same stages applied to the variational equations (every Jacobian
 * at the stage state), so the sensitivities are the exact derivatives of the
 * discrete map.  The tableau used by oracle_discretize_rkf is the 4(5) pair of
 * Fehlberg (1969): the fourth-order solution is propagated and the
 * fifth-order one gives the embedded error estimate; every interval reports
 * max_j max_r |e_j[r]| over its steps and all augmented rows.
 * ========================================================================== */
#define RKF_S 6
static const double RKF_C[RKF_S] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double RKF_A[RKF_S][RKF_S] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0}};
static const double RKF_B4[RKF_S] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0,
                                     -1.0 / 5.0, 0.0};
static const double RKF_B5[RKF_S] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                                     -9.0 / 50.0, 2.0 / 55.0};

/* The Fehlberg tableau as used (c[6], a[6][6] row-major, b[6], bh[6]). */
void oracle_rkf_tableau(double *c, double *a, double *b, double *bh) {
    for (int i = 0; i < RKF_S; ++i) {
        c[i] = RKF_C[i];
        b[i] = RKF_B4[i];
        bh[i] = RKF_B5[i];
        for (int l = 0; l < RKF_S; ++l) a[i * RKF_S + l] = RKF_A[i][l];
    }
}

/*
 * One interval [tau0, tau1] with K steps of the explicit method (S stages,
 * tableau c, a (S x S row-major), b, bh (may be NULL)), with the variational
 * equations of oracle_integrate for Z = [Phi | Bm | Bp | Sv]; *err receives
 * the largest |e| (0 when bh is NULL).  Outputs other than xf may be NULL.
 */
void oracle_integrate_erk(const omodel *M, const double *x0, const double *Uk, const double *Uk1,
                          double s, const double *p, double tau0, double tau1, int K, int S,
                          const double *c, const double *a, const double *b, const double *bh,
                          double *xf, double *Phi, double *Bm, double *Bp, double *Sv,
                          double *err) {
    const int nx = o_nx(M), m = o_m(M), np = o_np(M);
    const int nz = nx + 2 * m + 1;
    const int oB = nx, oP = nx + m, oS = nx + 2 * m;
    const size_t NZ = (size_t)nx * nz;
    const double h = (tau1 - tau0) / K;
    double *x = malloc(sizeof(double) * nx), *xs = malloc(sizeof(double) * nx);
    double *kx = malloc(sizeof(double) * nx * S);          /* K_i of the state, [S][nx] */
    double *Z = calloc(NZ, sizeof(double)), *Zs = malloc(sizeof(double) * NZ);
    double *KZ = malloc(sizeof(double) * NZ * S);          /* K_i of Z, [S][nx][nz] */
    double *Fv = malloc(sizeof(double) * nx), *Jx = malloc(sizeof(double) * nx * nx);
    double *Ju = malloc(sizeof(double) * nx * (m + 1)), *Jub = malloc(sizeof(double) * nx * (m + 1));
    double *Jp = malloc(sizeof(double) * nx * np);
    double *u = malloc(sizeof(double) * (m + 1)), *ub = malloc(sizeof(double) * (m + 1));
    double emax = 0.0;
    for (int r = 0; r < nx; ++r) { x[r] = x0[r]; Z[(size_t)r * nz + r] = 1.0; }
    for (int q = 0; q < m; ++q) ub[q] = 0.5 * (Uk[q] + Uk1[q]);
    for (int j = 0; j < K; ++j) {
        for (int i = 0; i < S; ++i) {
            const double tau = tau0 + (j + c[i]) * h;
            /* stage input */
            for (int r = 0; r < nx; ++r) {
                double acc = 0.0;
                for (int l = 0; l < i; ++l) acc += a[i * S + l] * kx[(size_t)l * nx + r];
                xs[r] = x[r] + acc;
            }
            for (size_t e = 0; e < NZ; ++e) {
                double acc = 0.0;
                for (int l = 0; l < i; ++l) acc += a[i * S + l] * KZ[(size_t)l * NZ + e];
                Zs[e] = Z[e] + acc;
            }
            for (int q = 0; q < m; ++q) u[q] = (1.0 - tau) * Uk[q] + tau * Uk1[q];
            oracle_rhs_jac(M, xs, u, ub, p, Fv, Jx, Ju, Jub, Jp);
            /* K_i = h (s Jx Zs + forcing), forcing as in oracle_integrate */
            double *KZi = KZ + (size_t)i * NZ;
            matmul(nx, nx, nz, Jx, Zs, KZi);
            for (size_t e = 0; e < NZ; ++e) KZi[e] *= s;
            for (int r = 0; r < nx; ++r) {
                for (int q = 0; q < m; ++q) {
                    KZi[(size_t)r * nz + oB + q] += s * (Ju[(size_t)r * m + q] * (1.0 - tau) + 0.5 * Jub[(size_t)r * m + q]);
                    KZi[(size_t)r * nz + oP + q] += s * (Ju[(size_t)r * m + q] * tau + 0.5 * Jub[(size_t)r * m + q]);
                }
                KZi[(size_t)r * nz + oS] += Fv[r];
            }
            for (size_t e = 0; e < NZ; ++e) KZi[e] *= h;
            for (int r = 0; r < nx; ++r) kx[(size_t)i * nx + r] = h * s * Fv[r];
        }
        if (bh) {
            for (int r = 0; r < nx; ++r) {
                double e = 0.0;
                for (int i = 0; i < S; ++i) e += (bh[i] - b[i]) * kx[(size_t)i * nx + r];
                if (fabs(e) > emax) emax = fabs(e);
            }
        }
        for (int r = 0; r < nx; ++r) {
            double acc = 0.0;
            for (int i = 0; i < S; ++i) acc += b[i] * kx[(size_t)i * nx + r];
            x[r] += acc;
        }
        for (size_t e = 0; e < NZ; ++e) {
            double acc = 0.0;
            for (int i = 0; i < S; ++i) acc += b[i] * KZ[(size_t)i * NZ + e];
            Z[e] += acc;
        }
    }
    memcpy(xf, x, sizeof(double) * nx);
    for (int r = 0; r < nx; ++r) {
        if (Phi) for (int q = 0; q < nx; ++q) Phi[(size_t)r * nx + q] = Z[(size_t)r * nz + q];
        if (Bm) for (int q = 0; q < m; ++q) Bm[(size_t)r * m + q] = Z[(size_t)r * nz + oB + q];
        if (Bp) for (int q = 0; q < m; ++q) Bp[(size_t)r * m + q] = Z[(size_t)r * nz + oP + q];
        if (Sv) Sv[r] = Z[(size_t)r * nz + oS];
    }
    if (err) *err = emax;
    free(x); free(xs); free(kx); free(Z); free(Zs); free(KZ); free(Fv); free(Jx); free(Ju);
    free(Jub); free(Jp); free(u); free(ub);
}

/* Multiple shooting with the Fehlberg pair: outputs of oracle_discretize
 * (without Pi) plus err[N], the embedded estimate of each interval. */
int oracle_discretize_rkf(const omodel *M, int N, int K, const double *X, const double *U,
                          const double *s, const double *p, double *A, double *Bm, double *Bp,
                          double *S, double *defect, double *xprop, double *err, int nthreads) {
    const int nx = o_nx(M), m = o_m(M);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int k = 0; k < N; ++k) {
        double *xf = malloc(sizeof(double) * nx);
        oracle_integrate_erk(M, X + (size_t)k * nx, U + (size_t)k * m, U + (size_t)(k + 1) * m,
                             s[k], p, 0.0, 1.0, K, RKF_S, RKF_C, &RKF_A[0][0], RKF_B4, RKF_B5, xf,
                             A ? A + (size_t)k * nx * nx : NULL,
                             Bm ? Bm + (size_t)k * nx * m : NULL,
                             Bp ? Bp + (size_t)k * nx * m : NULL,
                             S ? S + (size_t)k * nx : NULL, err ? err + k : NULL);
        for (int r = 0; r < nx; ++r) {
            if (xprop) xprop[(size_t)k * nx + r] = xf[r];
            if (defect) defect[(size_t)k * nx + r] = xf[r] - X[(size_t)(k + 1) * nx + r];
        }
        free(xf);
    }
    return 0;
}
