/*
 * Plain FP64 CPU oracle for Greedy Frank-Wolfe (GFW) multiclass graph segmentation
 * (Faccio, Porcelli, Rinaldi, Stoll, "Fast and Simple Multiclass Data Segmentation:
 * An Eigendecomposition and Projection-Free Approach", arXiv 2508.09738).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU path is checked against.  Nothing in the product path may link,
 * load or call it; only the tests, the smoke check and the CPU leg of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * Conventions: every floating-point quantity is double; rows and neighbours are
 * visited in index order; no blocking, fusion or reordering beyond the
 * definitions cited at each function.  Compiled with -ffp-contract=off so that
 * a*b+c is two roundings, as written.
 *
 * Timing build.  Compiled with -fopenmp -DORC_OPENMP, the loops marked ROW_LOOP
 * (loops over rows whose iterations write disjoint outputs and read nothing another
 * iteration writes) are split over threads.  Every sum that crosses rows stays a
 * serial loop in index order, so the timing build returns bit for bit what the
 * serial build returns; the serial build is the one the parity tests use.
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *  - argmin/argmax ties are broken towards the lowest class index;
 *  - d_i = 0 (isolated node) gives d_i^{-1/2} = 0, so row i of L_s is e_i;
 *  - the stop test g_k <= tol sits after the GLMO and before the update
 *    (Alg. 3, step 4); a negative tol disables it; `iters` counts updates;
 *  - the update is written U_{k+1} = (1-a) U_k + a S_k, the second form the paper
 *    gives for step 6, so that a = 1 lands exactly on S_k; rows whose direction
 *    d_i = s_i - u_i is zero (binary rows kept by the GLMO) are not touched, which
 *    keeps them exact for step sizes that are not powers of two;
 *  - "binary row" means every entry is exactly 0 or 1; supp(u_i) = {j : u_ij != 0}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gfw_oracle.h"

#ifdef ORC_OPENMP
#include <omp.h>
#define ROW_LOOP _Pragma("omp parallel for schedule(static)")
int orc_threads(void) { return omp_get_max_threads(); }
#else
#define ROW_LOOP
int orc_threads(void) { return 1; }
#endif

/* ------------------------------------------------------------------------- */
/* Graph quantities (Section 1: degrees, L = D - W, L_s = I - D^-1/2 W D^-1/2) */
/* ------------------------------------------------------------------------- */

/* Degrees d_i = sum_j w_ij (row sums of W, self-loops included). */
int orc_degrees(int64_t n, const int64_t *rp, const int32_t *ci, const double *w, double *d)
{
    (void)ci;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += w[p];
        d[i] = s;
    }
    return 0;
}

/*
 * Fully connected Gaussian graph (the Gaussian similarity of Section 1 on every pair, the
 * image setting of Section 5.1), evaluated from the features x (n x d, row-major) without
 * storing W: w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) for i != j, w_ii = 0.
 */
static double gauss_w(const double *x, int64_t d, int64_t i, int64_t j, double sigma)
{
    double r2 = 0.0;
    for (int64_t q = 0; q < d; ++q) {
        const double df = x[i * d + q] - x[j * d + q];
        r2 += df * df;
    }
    return exp(-r2 / (2.0 * sigma * sigma));
}

/* Degrees d_i = sum_{j != i} w_ij of the fully connected Gaussian graph (j increasing). */
int orc_gaussian_degrees(int64_t n, int64_t d, const double *x, double sigma, double *deg)
{
    ROW_LOOP
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) s += gauss_w(x, d, i, j, sigma);
        deg[i] = s;
    }
    return 0;
}

/*
 * Rows rows[0..m) of L_s U for the fully connected Gaussian graph, given its degrees:
 * (L_s U)_i = U_i - d_i^{-1/2} sum_{j != i} w_ij d_j^{-1/2} U_j (j increasing; a node of
 * degree 0 has d^{-1/2} = 0).  U is n x K, out is m x K.
 */
int orc_gaussian_rows(int64_t n, int64_t d, const double *x, double sigma, const double *deg, int32_t K,
                      const double *U, int64_t m, const int64_t *rows, double *out)
{
    ROW_LOOP
    for (int64_t r = 0; r < m; ++r) {
        const int64_t i = rows[r];
        const double di = deg[i] > 0.0 ? 1.0 / sqrt(deg[i]) : 0.0;
        double *o = out + r * K;
        for (int32_t c = 0; c < K; ++c) o[c] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double dj = deg[j] > 0.0 ? 1.0 / sqrt(deg[j]) : 0.0;
            const double w = gauss_w(x, d, i, j, sigma) * dj;
            for (int32_t c = 0; c < K; ++c) o[c] += w * U[j * K + c];
        }
        for (int32_t c = 0; c < K; ++c) o[c] = U[i * K + c] - di * o[c];
    }
    return 0;
}

/*
 * Symmetric normalised Laplacian L_s = I - D^{-1/2} W D^{-1/2} as an explicit CSR
 * matrix whose pattern is that of W plus the diagonal (inserted in sorted position
 * when W has no self-loop on that row).  Output buffers must hold nnz(W) + n
 * entries; the number written is returned (negative on malformed input).
 */
int64_t orc_build_sym_laplacian(int64_t n, const int64_t *rp, const int32_t *ci, const double *w,
                                int64_t *lrp, int32_t *lci, double *lv)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *dm = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!d || !dm) { free(d); free(dm); return -1; }
    orc_degrees(n, rp, ci, w, d);
    for (int64_t i = 0; i < n; ++i) dm[i] = d[i] > 0.0 ? 1.0 / sqrt(d[i]) : 0.0;

    int64_t out = 0;
    lrp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int diag_done = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t j = ci[p];
            if (!diag_done && j > i) {           /* diagonal comes before any larger column */
                lci[out] = (int32_t)i;
                lv[out] = 1.0;
                ++out;
                diag_done = 1;
            }
            if (j == i) {
                lci[out] = (int32_t)i;
                lv[out] = 1.0 - dm[i] * w[p] * dm[i];
                ++out;
                diag_done = 1;
            } else {
                lci[out] = j;
                lv[out] = -(dm[i] * w[p] * dm[j]);
                ++out;
            }
        }
        if (!diag_done) {
            lci[out] = (int32_t)i;
            lv[out] = 1.0;
            ++out;
        }
        lrp[i + 1] = out;
    }
    free(d);
    free(dm);
    return out;
}

/* P = L U for a CSR matrix L (n x n) and a row-major U (n x K). */
int orc_spmm(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
             const double *U, double *P)
{
    ROW_LOOP
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t c = 0; c < K; ++c) {
            double s = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * U[(int64_t)ci[p] * K + c];
            P[i * K + c] = s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Objective and gradient (eqs. gl_vv2 / gradgl_vv2 and gradgl_vv2g)          */
/* ------------------------------------------------------------------------- */

/*
 * E(U) = 1/2 tr(U^T L U) + (1/eps) tr(U (1 - U^T)) + 1/2 || D_w^{1/2} (Uhat - U) ||_F^2
 * with the all-ones 1, omega_i = omega0 on labelled rows and 0 elsewhere.
 * inv_eps = 1/eps (0 when eps = +inf).  Uhat rows of unlabelled nodes are never read.
 */
double orc_objective(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
                     const double *U, const double *Uhat, const double *omega, double inv_eps)
{
    double *P = (double *)malloc(sizeof(double) * (size_t)(n * K > 0 ? n * K : 1));
    if (!P) return NAN;
    orc_spmm(n, K, rp, ci, v, U, P);
    double quad = 0.0, pen = 0.0, fid = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t c = 0; c < K; ++c) {
            double u = U[i * K + c];
            quad += u * P[i * K + c];
            pen += u * (1.0 - u);
        }
        if (omega[i] != 0.0) {
            double r = 0.0;
            for (int32_t c = 0; c < K; ++c) {
                double e = Uhat[i * K + c] - U[i * K + c];
                r += e * e;
            }
            fid += omega[i] * r;
        }
    }
    free(P);
    return 0.5 * quad + inv_eps * pen + 0.5 * fid;
}

/* grad E(U) = L U + (1/eps)(1 - 2U) - D_w (Uhat - U); P = L U is passed in. */
int orc_gradient_from_P(int64_t n, int32_t K, const double *P, const double *U, const double *Uhat,
                        const double *omega, double inv_eps, double *G)
{
    ROW_LOOP
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t c = 0; c < K; ++c) {
            double u = U[i * K + c];
            double fid = omega[i] != 0.0 ? omega[i] * (Uhat[i * K + c] - u) : 0.0;
            G[i * K + c] = P[i * K + c] + inv_eps * (1.0 - 2.0 * u) - fid;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Linear minimisation oracles (Section 4)                                   */
/* ------------------------------------------------------------------------- */

static int row_is_binary(const double *u, int32_t K)
{
    for (int32_t c = 0; c < K; ++c)
        if (!(u[c] == 0.0 || u[c] == 1.0)) return 0;
    return 1;
}

/*
 * Vertex index s_i of row i of the oracle's output (the output is one-hot in every
 * row, so the vertex index describes it fully).
 *  GREEDY (GLMO): a row with u_i in {0,1}^K keeps u_i (its 1 is at s_i); any other
 *                 row takes the lowest index minimising G_ij over supp(u_i).
 *  FULL (LMO):    every row takes the lowest index minimising G_ij over all j.
 * A binary row of the simplex has exactly one 1; for the GREEDY case a binary row
 * with no 1 (off the simplex) keeps its first largest entry.
 * Returns the number of non-binary rows.
 */
int64_t orc_lmo(int64_t n, int32_t K, const double *U, const double *G, int mode, int32_t *s)
{
    int64_t nonbinary = 0;
#ifdef ORC_OPENMP
#pragma omp parallel for schedule(static) reduction(+ : nonbinary)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const double *u = U + i * K;
        const double *g = G + i * K;
        int bin = row_is_binary(u, K);
        if (!bin) ++nonbinary;
        if (mode == ORC_LMO_GREEDY && bin) {
            int32_t at = 0;
            for (int32_t c = 1; c < K; ++c)
                if (u[c] > u[at]) at = c;
            s[i] = at;
            continue;
        }
        int32_t best = -1;
        for (int32_t c = 0; c < K; ++c) {
            if (mode == ORC_LMO_GREEDY && u[c] == 0.0) continue; /* outside supp(u_i) */
            if (best < 0 || g[c] < g[best]) best = c;
        }
        s[i] = best < 0 ? 0 : best;
    }
    return nonbinary;
}

/* ------------------------------------------------------------------------- */
/* The GFW loop (Alg. 3), its FW (Alg. 2) and one-shot (Alg. 4) variants      */
/* ------------------------------------------------------------------------- */

static void set_hist(double *h, int64_t stride, int64_t k, double E, double g, double q, double a, double nb)
{
    if (!h) return;
    h[0 * stride + k] = E;
    h[1 * stride + k] = g;
    h[2 * stride + k] = q;
    h[3 * stride + k] = a;
    h[4 * stride + k] = nb;
}

/*
 * Runs the method on the CSR operator L (already L_s, or a user-supplied L).
 * U (n x K, row-major) holds U_0 on entry and the last iterate on exit.
 * Uhat/omega define the fidelity term.  hist (5 x (max_iter+1), may be NULL)
 * receives per evaluated iterate k: E(U_k), g_k, q_k = <D_k, Hess D_k>, alpha_k,
 * and the number of non-binary rows (NaN where a quantity was not formed).
 * s_hist (max_iter+1 rows of n, may be NULL) receives the vertex indices used.
 * s_first (n entries, may be NULL) replaces the (G)LMO's vertices of the first iteration:
 * the tests use it to follow another implementation's choice among tied minimisers
 * (the caller checks that the given vertices are minimisers up to its tolerance).
 */
int orc_solve(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
              const double *Uhat, const double *omega, const orc_params_t *prm,
              double *U, int32_t *labels, orc_stats_t *st, double *hist, int32_t *s_hist,
              const int32_t *s_first)
{
    if (n < 0 || K < 1 || !prm || !U) return -1;
    const int64_t nK = n * K;
    const int64_t hs = (int64_t)prm->max_iter + 1;
    double inv_eps = isinf(prm->eps) ? 0.0 : 1.0 / prm->eps;
    double *P = (double *)malloc(sizeof(double) * (size_t)(nK > 0 ? nK : 1));
    double *G = (double *)malloc(sizeof(double) * (size_t)(nK > 0 ? nK : 1));
    double *Dm = (double *)malloc(sizeof(double) * (size_t)(nK > 0 ? nK : 1));
    double *LD = (double *)malloc(sizeof(double) * (size_t)(nK > 0 ? nK : 1));
    double *Ut = (double *)malloc(sizeof(double) * (size_t)(nK > 0 ? nK : 1));
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!P || !G || !Dm || !LD || !Ut || !s) {
        free(P); free(G); free(Dm); free(LD); free(Ut); free(s);
        return -2;
    }
    if (hist)
        for (int64_t t = 0; t < 5 * hs; ++t) hist[t] = NAN;

    orc_stats_t out;
    memset(&out, 0, sizeof(out));
    out.stop_reason = ORC_STOP_MAXITER;
    out.alpha_last = NAN;
    out.gap = NAN;
    int32_t k = 0;
    for (k = 0; k < prm->max_iter; ++k) {
        /* gradient at U_k */
        orc_spmm(n, K, rp, ci, v, U, P);
        orc_gradient_from_P(n, K, P, U, Uhat, omega, inv_eps, G);
        /* E(U_k) from its definition, reusing P = L U_k */
        double quad = 0.0, pen = 0.0, fid = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t c = 0; c < K; ++c) {
                double u = U[i * K + c];
                quad += u * P[i * K + c];
                pen += u * (1.0 - u);
            }
            if (omega[i] != 0.0) {
                double r = 0.0;
                for (int32_t c = 0; c < K; ++c) {
                    double e = Uhat[i * K + c] - U[i * K + c];
                    r += e * e;
                }
                fid += omega[i] * r;
            }
        }
        double Ek = 0.5 * quad + inv_eps * pen + 0.5 * fid;

        /* step 3: S_k from the (G)LMO */
        int64_t nonbin = orc_lmo(n, K, U, G, prm->lmo, s);
        if (k == 0 && s_first) memcpy(s, s_first, sizeof(int32_t) * (size_t)n);
        if (s_hist) memcpy(s_hist + (int64_t)k * n, s, sizeof(int32_t) * (size_t)n);

        /* D_k = S_k - U_k and the gap g_k = -<grad E(U_k), D_k> */
        ROW_LOOP
        for (int64_t i = 0; i < n; ++i)
            for (int32_t c = 0; c < K; ++c) Dm[i * K + c] = (c == s[i] ? 1.0 : 0.0) - U[i * K + c];
        double gd = 0.0;
        for (int64_t t = 0; t < nK; ++t) gd += G[t] * Dm[t];
        double g = -gd;
        out.gap = g;
        if (isnan(g) || isnan(Ek)) {
            set_hist(hist, hs, k, Ek, g, NAN, NAN, (double)nonbin);
            out.stop_reason = ORC_STOP_NUMERIC;
            break;
        }
        /* step 4: stopping condition */
        if (prm->tol >= 0.0 && g <= prm->tol) {
            set_hist(hist, hs, k, Ek, g, NAN, NAN, (double)nonbin);
            out.stop_reason = ORC_STOP_TOL;
            break;
        }

        /* curvature q = <D, Hess E D> = <D, L D> - (2/eps)||D||^2 + sum_i omega_i ||d_i||^2 */
        orc_spmm(n, K, rp, ci, v, Dm, LD);
        double dld = 0.0, dd = 0.0, wdd = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double r = 0.0;
            for (int32_t c = 0; c < K; ++c) {
                double d = Dm[i * K + c];
                dld += d * LD[i * K + c];
                r += d * d;
            }
            dd += r;
            wdd += omega[i] * r;
        }
        double q = dld - 2.0 * inv_eps * dd + wdd;

        /* step 6: step size */
        double alpha = 1.0;
        if (prm->osfw) {
            alpha = 1.0; /* Alg. 4: U_1 = S_0 */
        } else if (prm->ls == ORC_LS_ARMIJO) {
            /* eqs. (eta)/(Armijo): smallest j >= 0 with
             * E(U) - E(U + delta^j D) >= -gamma delta^j <grad E, D>.  E is quadratic, so
             * E(U) - E(U + a D) = a g - a^2 q / 2 exactly; with armijo_direct the trial
             * point is instead evaluated from the definition of E. */
            alpha = 1.0;
            for (int j = 0; j <= 1074; ++j) {
                double dec;
                if (prm->armijo_direct) {
                    for (int64_t t = 0; t < nK; ++t) Ut[t] = U[t] + alpha * Dm[t];
                    dec = Ek - orc_objective(n, K, rp, ci, v, Ut, Uhat, omega, inv_eps);
                } else {
                    dec = alpha * g - 0.5 * alpha * alpha * q;
                }
                if (dec >= prm->gamma * alpha * g) break;
                alpha *= prm->delta;
            }
        } else if (prm->ls == ORC_LS_EXACT) {
            /* minimiser of the quadratic E(U + a D) over a in [0, 1] */
            alpha = q <= 0.0 ? 1.0 : fmin(1.0, g / q);
        } else { /* ORC_LS_SHORT: a = min(1, g / (Lbar ||D||^2)), eq. (alphabound) */
            alpha = fmin(1.0, g / (prm->lipschitz * dd));
        }
        set_hist(hist, hs, k, Ek, g, q, alpha, (double)nonbin);
        out.alpha_last = alpha;

        /* step 6: U_{k+1} = (1 - a) U_k + a S_k; a row whose direction d_i is zero (a
         * binary row kept by the GLMO) is left exactly as it is */
        ROW_LOOP
        for (int64_t i = 0; i < n; ++i) {
            int zero_dir = 1;
            for (int32_t c = 0; c < K; ++c)
                if (Dm[i * K + c] != 0.0) zero_dir = 0;
            if (zero_dir) continue;
            for (int32_t c = 0; c < K; ++c) {
                double sv = c == s[i] ? 1.0 : 0.0;
                double u = (1.0 - alpha) * U[i * K + c] + alpha * sv;
                U[i * K + c] = prm->store_f32 ? (double)(float)u : u;
            }
        }
        if (prm->osfw) { ++k; break; }
    }
    out.iters = k;
    out.objective = orc_objective(n, K, rp, ci, v, U, Uhat, omega, inv_eps);
    if (labels) {
        for (int64_t i = 0; i < n; ++i) {
            int32_t at = 0;
            for (int32_t c = 1; c < K; ++c)
                if (U[i * K + c] > U[i * K + at]) at = c;
            labels[i] = at;
        }
    }
    if (st) *st = out;
    free(P); free(G); free(Dm); free(LD); free(Ut); free(s);
    return 0;
}
