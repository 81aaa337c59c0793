// Sparse LDL^T factorization of symmetric quasi-definite matrices: the
// reduced KKT systems that the interior-point QP solver of the SCP driver
// factors once per iteration (the convex subproblems of arxiv 2604.09993,
// Sec. V; canonical-form solve of Sec. VI).  Host code.
//
// The matrix is given by its upper triangle (diagonal included) in
// compressed sparse columns, already in the elimination order.  Symbolic
// step: the elimination tree and the number of entries of every column of
// L, from the row subtrees of the matrix.  Numeric step: up-looking
// factorization, row k of L from a sparse triangular solve with the rows
// above it, whose pattern is the reach of column k's entries in the tree.
// Quasi-definite matrices (positive definite block, negative definite
// block) have an LDL^T factorization in every symmetric order, so no
// pivoting is done.  Far into an interior-point solve the diagonal spans
// many orders of magnitude and rounding can leave a pivot of the wrong sign
// or near zero: with the expected sign of every pivot given, such a pivot is
// replaced by sign * delta (dynamic regularization; the solver's iterative
// refinement against the unregularized matrix restores the accuracy).
#include <stdint.h>

#include "../../include/cis.h"

extern "C" int64_t cis_ldl_symbolic(int32_t n, const int32_t* Ap, const int32_t* Ai,
                                    int32_t* parent, int32_t* Lnz, int32_t* work) {
    if (n < 0 || !Ap) return -1;
    if (n == 0) return 0;
    if (!Ai || !parent || !Lnz || !work) return -1;
    int32_t* mark = work;
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        parent[k] = -1;
        mark[k] = k;
        Lnz[k] = 0;
        for (int32_t p = Ap[k]; p < Ap[k + 1]; ++p) {
            int32_t i = Ai[p];
            if (i < 0 || i > k) return -2;   // only the upper triangle
            // climb from i towards k: every node passed gets an entry in row k
            while (mark[i] != k) {
                if (parent[i] == -1) parent[i] = k;
                ++Lnz[i];
                mark[i] = k;
                i = parent[i];
            }
        }
    }
    for (int32_t k = 0; k < n; ++k) total += Lnz[k];
    return total;
}

extern "C" int32_t cis_ldl_numeric(int32_t n, const int32_t* Ap, const int32_t* Ai,
                                   const double* Ax, const int32_t* parent, const int32_t* Lnz,
                                   const int8_t* sign, double eps, double delta, int32_t* Lp,
                                   int32_t* Li, double* Lx, double* D, int32_t* iwork,
                                   double* y) {
    if (n < 0 || !Ap) return -1;
    if (n == 0) return 0;
    if (!Ai || !Ax || !parent || !Lnz || !Lp || !Li || !Lx || !D || !iwork || !y) return -1;
    int32_t* mark = iwork;           // [n] last row that visited a node
    int32_t* stack = iwork + n;      // [n] pattern of the current row
    int32_t* fill = iwork + 2 * n;   // [n] entries of each column written so far
    Lp[0] = 0;
    for (int32_t k = 0; k < n; ++k) {
        Lp[k + 1] = Lp[k] + Lnz[k];
        y[k] = 0.0;
        fill[k] = 0;
    }
    int32_t replaced = 0;
    for (int32_t k = 0; k < n; ++k) {
        int32_t top = n;
        mark[k] = k;
        for (int32_t p = Ap[k]; p < Ap[k + 1]; ++p) {
            int32_t i = Ai[p];
            y[i] += Ax[p];
            // the path from i up to the first visited node, pushed so that
            // every node comes before its ancestors
            int32_t len = 0;
            for (; mark[i] != k; i = parent[i]) {
                stack[len++] = i;
                mark[i] = k;
            }
            while (len > 0) stack[--top] = stack[--len];
        }
        double dk = y[k];
        y[k] = 0.0;
        for (; top < n; ++top) {
            const int32_t i = stack[top];
            const double yi = y[i];
            y[i] = 0.0;
            const int32_t end = Lp[i] + fill[i];
            for (int32_t p = Lp[i]; p < end; ++p) y[Li[p]] -= Lx[p] * yi;
            const double lki = yi / D[i];
            dk -= lki * yi;
            Li[end] = k;
            Lx[end] = lki;
            ++fill[i];
        }
        if (dk != dk) return -2;
        if (sign) {
            if (sign[k] * dk <= eps) {
                dk = sign[k] * delta;
                ++replaced;
            }
        } else if (dk == 0.0) {
            return -2;
        }
        D[k] = dk;
    }
    return replaced;
}

extern "C" void cis_ldl_solve(int32_t n, const int32_t* Lp, const int32_t* Li, const double* Lx,
                              const double* D, double* x) {
    for (int32_t j = 0; j < n; ++j) {
        const double xj = x[j];
        for (int32_t p = Lp[j]; p < Lp[j + 1]; ++p) x[Li[p]] -= Lx[p] * xj;
    }
    for (int32_t j = 0; j < n; ++j) x[j] /= D[j];
    for (int32_t j = n - 1; j >= 0; --j) {
        double xj = x[j];
        for (int32_t p = Lp[j]; p < Lp[j + 1]; ++p) xj -= Lx[p] * x[Li[p]];
        x[j] = xj;
    }
}
