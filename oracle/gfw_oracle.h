/*
 * Plain FP64 CPU oracle for Greedy Frank-Wolfe multiclass graph segmentation
 * (arXiv 2508.09738).  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the CPU leg of the benchmark; never by the product path.
 */
#ifndef GFW_ORACLE_H
#define GFW_ORACLE_H
#include <stdint.h>

enum { ORC_LMO_GREEDY = 0, ORC_LMO_FULL = 1 };
enum { ORC_LS_ARMIJO = 0, ORC_LS_EXACT = 1, ORC_LS_SHORT = 2 };
enum { ORC_STOP_MAXITER = 0, ORC_STOP_TOL = 1, ORC_STOP_NUMERIC = 2 };

typedef struct {
    double eps;          /* penalty parameter; +inf drops the penalty          */
    double omega0;       /* fidelity weight (informational; omega[] is passed) */
    int32_t max_iter;
    double tol;          /* stop when g_k <= tol; negative disables            */
    int32_t ls;          /* ORC_LS_*                                           */
    double delta, gamma; /* Armijo parameters                                  */
    int32_t lmo;         /* ORC_LMO_*                                          */
    int32_t osfw;        /* 1: one-shot FW (U_1 = S_0)                         */
    double lipschitz;    /* Lbar for the short step                            */
    int32_t armijo_direct; /* 1: evaluate E at Armijo trial points directly    */
    int32_t store_f32;   /* 1: round U to the nearest FP32 value after every
                            update (models FP32 storage of the iterate)        */
} orc_params_t;

typedef struct {
    int32_t iters, stop_reason;
    double gap, objective, alpha_last;
} orc_stats_t;

int orc_degrees(int64_t n, const int64_t *rp, const int32_t *ci, const double *w, double *d);
int orc_gaussian_degrees(int64_t n, int64_t d, const double *x, double sigma, double *deg);
int orc_gaussian_rows(int64_t n, int64_t d, const double *x, double sigma, const double *deg, int32_t K,
                      const double *U, int64_t m, const int64_t *rows, double *out);
int64_t orc_build_sym_laplacian(int64_t n, const int64_t *rp, const int32_t *ci, const double *w,
                                int64_t *lrp, int32_t *lci, double *lv);
int orc_spmm(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
             const double *U, double *P);
double orc_objective(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
                     const double *U, const double *Uhat, const double *omega, double inv_eps);
int orc_gradient_from_P(int64_t n, int32_t K, const double *P, const double *U, const double *Uhat,
                        const double *omega, double inv_eps, double *G);
int64_t orc_lmo(int64_t n, int32_t K, const double *U, const double *G, int mode, int32_t *s);
/* threads the row loops may use: 1 in the serial build, the OpenMP team size in
 * the timing build (compiled with -fopenmp -DORC_OPENMP) */
int orc_threads(void);
int orc_solve(int64_t n, int32_t K, const int64_t *rp, const int32_t *ci, const double *v,
              const double *Uhat, const double *omega, const orc_params_t *prm,
              double *U, int32_t *labels, orc_stats_t *st, double *hist, int32_t *s_hist,
              const int32_t *s_first);
#endif
