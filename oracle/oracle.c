/*
 * Plain CPU oracle for the tile Householder QR path. TEST INFRASTRUCTURE ONLY:
 * nothing in the product library calls, links or loads this file; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark do.
 *
 * What it computes. Section 2.1 of the paper factorizes a dense matrix as
 * A = QR, with Q a product of Householder reflectors, by a DAG of tile tasks
 * (DGEQRT, DTSQRT, DLARFB, DSSRFB). Up to rounding order and the choice of
 * reflector signs, every tiling and inner blocking reaches the result of the
 * plain, unblocked Householder QR (LAPACK xGEQR2 semantics). That plain
 * definition is what this file writes out, in FP64, with no blocking, no
 * fusion and no reordering. The paper defers the kernels' formulas to its
 * reference on PLASMA tile algorithms, so the textbook definition is used:
 *
 *   for j = 0 .. K-1 (K = min(M, N)):
 *     alpha = A[j][j], x = A[j+1:M][j], xi = ||x||_2
 *     xi == 0  -> tau_j = 0 (H_j = I, A[j][j] keeps its sign)
 *     else        beta = -sign(alpha) sqrt(alpha^2 + xi^2), sign(0) = +1,
 *                 tau_j = (beta - alpha) / beta, v = [1; x / (alpha - beta)],
 *                 A[j][j] = beta, A[j+1:M][j] = v[1:]
 *     A[j:M][j+1:N] -= tau_j v (v^T A[j:M][j+1:N])
 *
 * Norms are a plain sum of squares followed by a square root (the inputs are
 * O(1); no LAPACK-style rescaling). All matrices are column-major with an
 * explicit leading dimension. The only parallelism is OpenMP over the
 * independent trailing columns of the rank-1 update, which changes no result.
 *
 * Also here: Q^T B and Q B by applying the reflectors one at a time, the
 * compact-WY factor T of a run of reflectors (its defining recurrence), a
 * Gram entry (A^T A)_ij, and the FP64 forward/backward of the small MLP cost
 * model (5 -> 64 -> 64 -> 64 -> 1, ReLU) used to pin the GPU training
 * kernels.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(a, i, j, ld) ((a)[(int64_t)(j) * (ld) + (i)])

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One Householder step on column j (reflector generation). Returns tau. */
static double make_reflector(int64_t m, double *a, int64_t lda, int64_t j) {
    double alpha = IDX(a, j, j, lda);
    double ss = 0.0;
    for (int64_t r = j + 1; r < m; ++r) {
        double x = IDX(a, r, j, lda);
        ss += x * x;
    }
    if (ss == 0.0) return 0.0;
    double xi = sqrt(ss);
    double nrm = sqrt(alpha * alpha + xi * xi);
    double beta = (alpha >= 0.0) ? -nrm : nrm; /* sign(0) = +1 */
    double tau = (beta - alpha) / beta;
    double scale = 1.0 / (alpha - beta);
    for (int64_t r = j + 1; r < m; ++r) IDX(a, r, j, lda) *= scale;
    IDX(a, j, j, lda) = beta;
    return tau;
}

/* Apply H = I - tau v v^T (v = [1; V[j+1:m][j]]) to columns c0..c1-1 of B,
 * rows j..m-1. */
static void apply_reflector(int64_t m, const double *v, int64_t ldv, int64_t j,
                            double tau, double *b, int64_t ldb, int64_t c0,
                            int64_t c1) {
    if (tau == 0.0) return;
#pragma omp parallel for schedule(static) if ((c1 - c0) * (m - j) > 65536)
    for (int64_t c = c0; c < c1; ++c) {
        double w = IDX(b, j, c, ldb);
        for (int64_t r = j + 1; r < m; ++r) w += IDX(v, r, j, ldv) * IDX(b, r, c, ldb);
        w *= tau;
        IDX(b, j, c, ldb) -= w;
        for (int64_t r = j + 1; r < m; ++r) IDX(b, r, c, ldb) -= w * IDX(v, r, j, ldv);
    }
}

/* The first `steps` Householder steps of the unblocked QR (all K = min(m, n)
 * of them when steps >= K): column j's reflector is generated, then applied
 * to every column to its right. A bounded number of steps is the sample the
 * benchmark times on large inputs; the full factorization below is the same
 * loop run to the end, so both share one code path. */
void oracle_geqr2_steps(int64_t m, int64_t n, double *a, int64_t lda,
                        double *tau, int64_t steps) {
    int64_t k = m < n ? m : n;
    if (steps < k) k = steps;
    for (int64_t j = 0; j < k; ++j) {
        tau[j] = make_reflector(m, a, lda, j);
        apply_reflector(m, a, lda, j, tau[j], a, lda, j + 1, n);
    }
}

/* Unblocked Householder QR: on exit R is in the upper triangle/trapezoid of
 * A, the reflectors' tails below the diagonal, tau[0..K-1] the scalars. */
void oracle_geqr2(int64_t m, int64_t n, double *a, int64_t lda, double *tau) {
    oracle_geqr2_steps(m, n, a, lda, tau, m < n ? m : n);
}

/* B <- Q^T B = H_{K-1} ... H_0 B: reflectors applied in ascending order. */
void oracle_apply_qt(int64_t m, int64_t k, const double *v, int64_t ldv,
                     const double *tau, int64_t nrhs, double *b, int64_t ldb) {
    for (int64_t j = 0; j < k; ++j)
        apply_reflector(m, v, ldv, j, tau[j], b, ldb, 0, nrhs);
}

/* B <- Q B = H_0 ... H_{K-1} B: reflectors applied in descending order. */
void oracle_apply_q(int64_t m, int64_t k, const double *v, int64_t ldv,
                    const double *tau, int64_t nrhs, double *b, int64_t ldb) {
    for (int64_t j = k - 1; j >= 0; --j)
        apply_reflector(m, v, ldv, j, tau[j], b, ldb, 0, nrhs);
}

/* Back substitution: X = R^{-1} B for the upper triangle of the n x n block
 * R, in place in B (n x nrhs), row n-1 first:
 * x_i = (b_i - sum_{c>i} R[i][c] x_c) / R[i][i]. */
void oracle_trsv_upper(int64_t n, const double *r, int64_t ldr, int64_t nrhs, double *b,
                       int64_t ldb) {
    for (int64_t q = 0; q < nrhs; ++q)
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = IDX(b, i, q, ldb);
            for (int64_t c = i + 1; c < n; ++c) s -= IDX(r, i, c, ldr) * IDX(b, c, q, ldb);
            IDX(b, i, q, ldb) = s / IDX(r, i, i, ldr);
        }
}

/* Compact-WY factor of the reflectors j0 .. j0+k-1 stored in V (unit entry
 * at row j, tail below it): H_{j0} ... H_{j0+k-1} = I - Vb T Vb^T with T
 * k-by-k upper triangular, T[c][c] = tau_c and
 * T[0:c][c] = -tau_c T[0:c][0:c] (Vb[:,0:c]^T vb_c). */
void oracle_larft(int64_t m, int64_t j0, int64_t k, const double *v,
                  int64_t ldv, const double *tau, double *t, int64_t ldt) {
    for (int64_t c = 0; c < k; ++c)
        for (int64_t r = 0; r < k; ++r) IDX(t, r, c, ldt) = 0.0;
    double *z = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int64_t c = 0; c < k; ++c) {
        int64_t jc = j0 + c;
        /* z_p = vb_p^T vb_c for p < c, with the implicit unit entries. */
        for (int64_t p = 0; p < c; ++p) {
            int64_t jp = j0 + p;
            double s = IDX(v, jc, jp, ldv); /* vb_p[jc] * vb_c[jc] (= 1) */
            for (int64_t r = jc + 1; r < m; ++r)
                s += IDX(v, r, jp, ldv) * IDX(v, r, jc, ldv);
            z[p] = s;
        }
        for (int64_t a = 0; a < c; ++a) {
            double s = 0.0;
            for (int64_t p = a; p < c; ++p) s += IDX(t, a, p, ldt) * z[p];
            IDX(t, a, c, ldt) = -tau[jc] * s;
        }
        IDX(t, c, c, ldt) = tau[jc];
    }
    free(z);
}

/* (A^T A)_ij: a plain dot product of two columns. */
double oracle_gram_entry(int64_t m, const double *a, int64_t lda, int64_t i,
                         int64_t j) {
    double s = 0.0;
    for (int64_t r = 0; r < m; ++r) s += IDX(a, r, i, lda) * IDX(a, r, j, lda);
    return s;
}

/* ------------------------------------------------------------------------
 * MLP cost model, FP64. Parameter vector layout (8769 entries), each weight
 * matrix row-major [out][in]:
 *   W1[64][5] @0, b1[64] @320, W2[64][64] @384, b2[64] @4480,
 *   W3[64][64] @4544, b3[64] @8640, W4[1][64] @8704, b4[1] @8768.
 * yhat = W4 h3 + b4, h_l = relu(W_l h_{l-1} + b_l), h_0 = x.
 * Loss over a batch of n rows: L = (1 / (2n)) sum_r (yhat_r - y_r)^2.
 * ---------------------------------------------------------------------- */
#define MLP_IN 5
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 320
#define OFF_W2 384
#define OFF_B2 4480
#define OFF_W3 4544
#define OFF_B3 8640
#define OFF_W4 8704
#define OFF_B4 8768
#define MLP_NPARAM 8769

int oracle_mlp_nparam(void) { return MLP_NPARAM; }

static void mlp_fwd_one(const double *p, const double *x, double *z1, double *h1,
                        double *z2, double *h2, double *z3, double *h3,
                        double *yhat) {
    for (int o = 0; o < MLP_H; ++o) {
        double s = p[OFF_B1 + o];
        for (int i = 0; i < MLP_IN; ++i) s += p[OFF_W1 + o * MLP_IN + i] * x[i];
        z1[o] = s;
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = p[OFF_B2 + o];
        for (int i = 0; i < MLP_H; ++i) s += p[OFF_W2 + o * MLP_H + i] * h1[i];
        z2[o] = s;
        h2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = p[OFF_B3 + o];
        for (int i = 0; i < MLP_H; ++i) s += p[OFF_W3 + o * MLP_H + i] * h2[i];
        z3[o] = s;
        h3[o] = s > 0.0 ? s : 0.0;
    }
    double s = p[OFF_B4];
    for (int i = 0; i < MLP_H; ++i) s += p[OFF_W4 + i] * h3[i];
    *yhat = s;
}

void oracle_mlp_forward(const double *p, const double *x, int64_t n, double *y) {
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], z3[MLP_H], h3[MLP_H];
    for (int64_t r = 0; r < n; ++r)
        mlp_fwd_one(p, x + r * MLP_IN, z1, h1, z2, h2, z3, h3, &y[r]);
}

/* Loss and its gradient w.r.t. every parameter, by the chain rule. The ReLU
 * derivative at exactly 0 is taken as 0. */
double oracle_mlp_grad(const double *p, const double *x, const double *y,
                       int64_t n, double *g) {
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], z3[MLP_H], h3[MLP_H];
    double d1[MLP_H], d2[MLP_H], d3[MLP_H];
    double loss = 0.0;
    memset(g, 0, sizeof(double) * MLP_NPARAM);
    for (int64_t r = 0; r < n; ++r) {
        const double *xr = x + r * MLP_IN;
        double yhat;
        mlp_fwd_one(p, xr, z1, h1, z2, h2, z3, h3, &yhat);
        double e = yhat - y[r];
        loss += 0.5 * e * e;
        double dy = e / (double)n;
        g[OFF_B4] += dy;
        for (int i = 0; i < MLP_H; ++i) {
            g[OFF_W4 + i] += dy * h3[i];
            d3[i] = (z3[i] > 0.0) ? dy * p[OFF_W4 + i] : 0.0;
        }
        for (int o = 0; o < MLP_H; ++o) {
            g[OFF_B3 + o] += d3[o];
            for (int i = 0; i < MLP_H; ++i) g[OFF_W3 + o * MLP_H + i] += d3[o] * h2[i];
        }
        for (int i = 0; i < MLP_H; ++i) {
            double s = 0.0;
            for (int o = 0; o < MLP_H; ++o) s += p[OFF_W3 + o * MLP_H + i] * d3[o];
            d2[i] = (z2[i] > 0.0) ? s : 0.0;
        }
        for (int o = 0; o < MLP_H; ++o) {
            g[OFF_B2 + o] += d2[o];
            for (int i = 0; i < MLP_H; ++i) g[OFF_W2 + o * MLP_H + i] += d2[o] * h1[i];
        }
        for (int i = 0; i < MLP_H; ++i) {
            double s = 0.0;
            for (int o = 0; o < MLP_H; ++o) s += p[OFF_W2 + o * MLP_H + i] * d2[o];
            d1[i] = (z1[i] > 0.0) ? s : 0.0;
        }
        for (int o = 0; o < MLP_H; ++o) {
            g[OFF_B1 + o] += d1[o];
            for (int i = 0; i < MLP_IN; ++i) g[OFF_W1 + o * MLP_IN + i] += d1[o] * xr[i];
        }
    }
    return loss / (double)n;
}
