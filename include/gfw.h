/*
 * gfw.h -- C ABI of an MI355X (gfx950) implementation of Greedy Frank-Wolfe (GFW)
 * multiclass graph segmentation: Faccio, Porcelli, Rinaldi, Stoll, "Fast and Simple
 * Multiclass Data Segmentation: An Eigendecomposition and Projection-Free Approach"
 * (arXiv 2508.09738).
 *
 * The method (Section 2, eqs. gl_vv2 / penalty_form) finds U in Sigma, the product of n
 * unit simplices (eq. fs), minimising
 *     E(U) = 1/2 tr(U^T L_s U) + (1/eps) tr(U (1 - U^T)) + 1/2 ||D_w^{1/2} (Uhat - U)||_F^2
 * where L_s = I - D^{-1/2} W D^{-1/2} is the symmetric normalised graph Laplacian
 * (Section 1), Uhat holds the known one-hot labels and D_w = diag(omega), omega_i = omega0
 * on labelled nodes and 0 elsewhere.  Each iteration of Alg. 3 forms the gradient
 * (eq. gradgl_vv2g), the greedy linear minimisation oracle (GLMO, Section 4), the duality
 * gap g_k = -<grad E(U_k), D_k> and an Armijo step (eqs. eta, Armijo; Section 5.1 uses
 * delta = 0.5, gamma = 1e-6, at most 30 iterations or g_k <= 1e-6), then
 * U_{k+1} = (1 - alpha_k) U_k + alpha_k S_k.
 *
 * General conventions
 *  - Every call returns gfw_status_t; no C++ exception crosses this boundary.  On error
 *    gfw_last_error() returns a thread-local message.  Scalar and O(n) checks run on the
 *    host before any launch; the checks of the CSR entries (column range and order,
 *    values, symmetry) run as a kernel on the uploaded copy, before the operator is
 *    formed.  A failed call leaves nothing allocated.
 *  - Pointers are caller-owned.  Whether a problem's arrays live in host or device
 *    memory is stated by gfw_problem_t.location.  Output arrays of gfw_solve and
 *    gfw_objective are DEVICE pointers; the server's outputs are HOST pointers.
 *  - Calls taking a hipStream_t (passed as void*; NULL = the null stream) are ordered on
 *    that stream.  A context is not thread-safe; a server is internally synchronised.
 *  - Row-major layouts: U is n x K, element (i, c) at U[i*K + c], of the graph's dtype.
 *  - Indices: row_ptr is int64[n+1] (row_ptr[0] = 0), col_idx int32[nnz], sorted strictly
 *    increasing within each row.  nnz must be < 2^31.
 */
#ifndef GFW_H
#define GFW_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define GFW_API __attribute__((visibility("default")))
#else
#define GFW_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GFW_OK = 0,
    GFW_E_INVALID_ARG = -1, /* NULL pointer, K < 2, n < 1, eps <= 0 or NaN, bad enum ...  */
    GFW_E_GRAPH = -2,       /* CSR malformed: row_ptr not monotone, column out of range,
                               unsorted or duplicate columns, negative/NaN/inf weight,
                               nnz >= 2^31, asymmetric pattern or values                   */
    GFW_E_LABELS = -3,      /* labelled index out of range or repeated, label not in [0,K) */
    GFW_E_NOMEM = -4,       /* device allocation failed                                    */
    GFW_E_HIP = -5,         /* a HIP runtime call failed (no GPU, launch error, ...)        */
    GFW_E_UNSUPPORTED = -6, /* valid but not supported (e.g. K above GFW_MAX_K)             */
    GFW_E_BUDGET = -7,      /* a request does not fit the server's HBM budget               */
    GFW_E_NOT_READY = -8,   /* non-blocking poll: result not available yet                  */
    GFW_E_NUMERIC = -9      /* the iteration produced a NaN (poisoned input)                */
} gfw_status_t;

#define GFW_MAX_K 1024

typedef enum {
    GFW_GRAPH_W = 0, /* weights W >= 0 (symmetric); the library forms L_s (Section 1)      */
    GFW_GRAPH_L = 1  /* a symmetric operator L given as is (e.g. L = D - W); used as L_s   */
} gfw_graph_kind_t;

typedef enum { GFW_F32 = 0, GFW_F64 = 1 } gfw_dtype_t;

typedef enum { GFW_HOST = 0, GFW_DEVICE = 1 } gfw_location_t;

typedef enum {
    GFW_LS_ARMIJO = 0, /* alpha = delta^j, smallest j >= 0 meeting eq. Armijo               */
    GFW_LS_EXACT = 1,  /* minimiser of the quadratic E(U + a D) on [0, 1]                  */
    GFW_LS_SHORT = 2   /* a = min(1, g / (Lbar ||D||^2)), the bound of eq. alphabound       */
} gfw_linesearch_t;

typedef enum {
    GFW_LMO_GREEDY = 0, /* GLMO of Alg. 3: binary rows keep u_i, others argmin on supp(u_i) */
    GFW_LMO_FULL = 1    /* classic LMO of Alg. 2: argmin over all K classes in every row    */
} gfw_lmo_t;

typedef enum {
    GFW_STOP_MAXITER = 0, /* max_iter updates were made                                      */
    GFW_STOP_TOL = 1,     /* g_k <= tol (Alg. 3 step 4); iters = k                             */
    GFW_STOP_NUMERIC = 2  /* NaN met; U holds the last finite iterate                        */
} gfw_stop_t;

/* A segmentation problem: the graph, the labelled node set and its labels, K (Section 2). */
typedef struct {
    int64_t n;                 /* nodes, >= 1                                               */
    int64_t nnz;               /* stored entries of W (or L), < 2^31                        */
    int32_t K;                 /* classes, 2 <= K <= GFW_MAX_K                              */
    gfw_graph_kind_t kind;
    gfw_dtype_t dtype;         /* dtype of vals and of U                                    */
    gfw_location_t location;   /* where row_ptr, col_idx, vals, labelled_idx, labels live   */
    const int64_t *row_ptr;    /* int64[n+1]                                                */
    const int32_t *col_idx;    /* int32[nnz]                                                */
    const void *vals;          /* dtype[nnz]; NULL = unit weights (kind W only)            */
    int64_t n_labelled;        /* >= 0                                                      */
    const int32_t *labelled_idx; /* int32[n_labelled], distinct, in [0, n)                  */
    const int32_t *labels;     /* int32[n_labelled], in [0, K)                              */
} gfw_problem_t;

/* Solver settings (Alg. 3 and Section 5.1).  gfw_params_default fills the paper's values. */
typedef struct {
    double eps;          /* penalty parameter > 0; +INFINITY drops the penalty term        */
    double omega0;       /* fidelity weight >= 0 on labelled nodes                          */
    int32_t max_iter;    /* >= 0; the paper uses 30                                          */
    double tol;          /* stop when g_k <= tol (paper 1e-6); negative disables the test   */
    gfw_linesearch_t ls;
    double delta;        /* Armijo reduction factor in (0, 1); paper 0.5                     */
    double gamma;        /* Armijo slope in (0, 1/2); paper 1e-6                              */
    gfw_lmo_t lmo;
    int32_t one_shot;    /* 1: Alg. 4 (OSFW), U_1 = S_0                                      */
    double lipschitz;    /* Lbar for GFW_LS_SHORT; <= 0 selects rho_max + 2/eps + omega0    */
    const void *U0;      /* n x K of the graph's dtype, rows in Sigma (not checked); NULL =
                            U_0 = Uhat with unlabelled rows 1/K (Section 5.1).  A DEVICE
                            array for gfw_solve / gfw_solve_batched, a HOST array (copied at
                            submit) for gfw_server_submit.  Warm start for new nodes
                            (Section 4, closing remarks): rows of already segmented nodes
                            one-hot, new rows anywhere in Sigma; the GLMO keeps binary rows,
                            so only the new rows move.                                       */
    int32_t p_refresh;   /* recompute L_s U by a full SpMM every p_refresh iterations
                            (0 = only at the start); see gfw_solve                          */
    int32_t incremental; /* 1: inference for new nodes (Section 4, closing remarks): a warm
                            start from U0 that iterates only the rows of U0 that are not
                            binary.  The GLMO keeps binary rows, so their rows of U, of the
                            vertex matrix S and of the direction are fixed; each iteration
                            then touches only the moving rows and their CSR entries.  When
                            a history is asked for, E(U_k) is carried by the exact quadratic
                            update E_{k+1} = E_k - alpha g_k + alpha^2 q_k / 2 from E(U_0)
                            (one evaluation on the whole graph; without a history the
                            history's E is not formed).  The
                            iterates are those of the full iteration (sums in another
                            order).  Needs U0, the GLMO, p_refresh = 0, a CSR graph and
                            K <= 16 (GFW_E_INVALID_ARG / GFW_E_UNSUPPORTED otherwise); not
                            in batches or the server.  0: every row every iteration.        */
} gfw_params_t;

typedef struct {
    int32_t iters;       /* updates made                                                    */
    int32_t stop_reason; /* gfw_stop_t                                                      */
    double gap;          /* last g_k formed                                                 */
    double objective;    /* E(U_out) from its definition                                    */
    double alpha_last;   /* last step size (NaN if none)                                    */
} gfw_stats_t;

typedef struct gfw_context_s *gfw_context_t;
typedef struct gfw_graph_s *gfw_graph_t;
typedef struct gfw_server_s *gfw_server_t;

/* ---- errors and defaults ---------------------------------------------------------- */
GFW_API const char *gfw_status_string(gfw_status_t s);
GFW_API const char *gfw_last_error(void);
/* eps = 50, omega0 = 1000, max_iter = 30, tol = 1e-6, Armijo with delta = 0.5,
 * gamma = 1e-6, GLMO, no one-shot, lipschitz = 0, U0 = NULL, p_refresh = 0, incremental = 0. */
GFW_API void gfw_params_default(gfw_params_t *p);
/* Host-only checks (no GPU needed).  gfw_check_problem validates the scalar fields and,
 * for location == GFW_HOST, the whole CSR and label arrays (same codes as
 * gfw_graph_create).  gfw_check_params validates p for K classes. */
GFW_API gfw_status_t gfw_check_problem(const gfw_problem_t *p);
GFW_API gfw_status_t gfw_check_params(const gfw_params_t *p, int32_t K);

/* ---- context ------------------------------------------------------------------------ */
/* Binds HIP device `device` (must be gfx950).  GFW_E_HIP when no such device exists. */
GFW_API gfw_status_t gfw_context_create(gfw_context_t *ctx, int device);
GFW_API gfw_status_t gfw_context_destroy(gfw_context_t ctx);

/* ---- graphs ------------------------------------------------------------------------- */
/*
 * Validates the problem (GFW_E_GRAPH / GFW_E_LABELS: sizes, row pointers and labels of
 * host input on the host; the CSR entries - column range and order, finite non-negative
 * values, symmetry - by a kernel after the upload), copies it into library-owned device
 * memory and forms the operator (Section 1):
 * degrees d_i = sum_j w_ij, d_i^{-1/2} (0 for an isolated node, whose row of L_s is then
 * e_i) and the scaled values -d_i^{-1/2} w_ij d_j^{-1/2}.  Symmetry of W (or L) is
 * checked.  The caller's arrays may be freed when the call returns.
 */
GFW_API gfw_status_t gfw_graph_create(gfw_context_t ctx, const gfw_problem_t *p, gfw_graph_t *out, void *stream);

/*
 * Fully connected Gaussian graphs, the image setting of Section 5.1: node i carries a
 * feature vector x_i in R^d (e.g. the colour of a pixel) and w_ij = exp(-||x_i - x_j||^2 /
 * (2 sigma^2)) for i != j (the Gaussian similarity of Section 1; no self-loops), so W is
 * dense.  The library never forms it: each product with L_s = I - D^{-1/2} W D^{-1/2} sums
 * the weights from the features (the paper uses an NFFT-based fast summation for these
 * products, Section 5.1).  method: GFW_GAUSS_EXACT forms every weight (O(n^2 K) per product,
 * 1 <= d <= 8; each weight formed in the graph's dtype — an FP32 graph from its FP32 features
 * with the FP32 exponential, as an FP32 CSR graph stores FP32 values — and summed in FP64);
 * GFW_GAUSS_GRID, for 1 <= d <= 3, gathers the points onto a grid of
 * spacing sigma / 2 with a Gaussian window, convolves the grid with a Gaussian and
 * interpolates back, the widths chosen so that the composite kernel is the Gaussian of width
 * sigma (windows cut at 5 widths: a relative error of about 1e-7 per product, and about 7e-8
 * more for an FP32 graph, whose convolved grid is stored in FP32; O((n + cells) 14^d K) per
 * product, the cells spanning the range of the features in steps of sigma / 2;
 * GFW_E_UNSUPPORTED when the grid would exceed 2^26 / KP cells, KP = K rounded up to 4, 8 or
 * 16), and makes a node whose degree
 * is at most 1e-6 isolated;
 * GFW_GAUSS_AUTO takes the method of the smaller modelled time (the grid only when d <= 3 and
 * it fits): the grid at about 1.8 ps per unit of its work estimate (point and cell visits,
 * (n + cells) 14^d) plus 20 us, the exact sums at 0.8 ps (FP32 graph) or 1.3 ps (FP64) per
 * pair, rates measured on an MI355X.  The graph is then used by
 * gfw_solve, gfw_objective, gfw_objective_noalloc and gfw_spmm like any other (K <= 16);
 * gfw_solve_batched and the server return GFW_E_UNSUPPORTED for it.  features: n x d of dtype,
 * row-major, finite (GFW_E_GRAPH otherwise); sigma > 0 and finite.  Labels as in
 * gfw_problem_t.  All arrays are HOST or DEVICE as `location` says; copied at creation.
 */
typedef enum { GFW_GAUSS_AUTO = 0, GFW_GAUSS_EXACT = 1, GFW_GAUSS_GRID = 2 } gfw_gauss_method_t;
typedef struct {
    int64_t n;                   /* nodes, >= 1                                               */
    int32_t d;                   /* feature dimensions                                        */
    int32_t K;                   /* classes, 2 <= K <= 16                                     */
    gfw_dtype_t dtype;           /* dtype of the features and of U                            */
    gfw_location_t location;
    const void *features;        /* n x d                                                     */
    double sigma;                /* width of the Gaussian similarity                          */
    gfw_gauss_method_t method;
    int64_t n_labelled;
    const int32_t *labelled_idx; /* int32[n_labelled], distinct, in [0, n)                    */
    const int32_t *labels;       /* int32[n_labelled], in [0, K)                              */
} gfw_gaussian_problem_t;
GFW_API gfw_status_t gfw_graph_create_gaussian(gfw_context_t ctx, const gfw_gaussian_problem_t *p, gfw_graph_t *out,
                                       void *stream);
GFW_API gfw_status_t gfw_graph_destroy(gfw_graph_t g);
/* Device bytes held by a graph and by one solve on it (workspace). */
GFW_API gfw_status_t gfw_graph_footprint(gfw_graph_t g, size_t *graph_bytes, size_t *solve_bytes);
/* Implementation choices of a graph (results are identical whichever is chosen):
 *  GFW_TUNE_LABEL_PATH: 0 = automatic (chosen at gfw_graph_create from the graph's
 *    locality), 1 = plain label pass, 2 = column-sorted label pass (builds, once, a copy
 *    of the entries sorted by column within tiles of rows, 4 bytes per entry: the entry's
 *    offset in the tile and its column relative to an anchor column per 64 sorted entries;
 *    tiles are sized so that their count fills whole rounds of the device's compute units;
 *    GFW_E_UNSUPPORTED if a row has more than 131072 entries), 3 = measured: times both
 *    passes on this graph (5 launches each, on the default stream, synchronising it) and
 *    keeps the faster.  K > 16 has one pass.
 * gfw_graph_query returns the current value of a key: GFW_TUNE_LABEL_PATH 1 or 2;
 * GFW_TUNE_LABEL_PLAIN_NS / GFW_TUNE_LABEL_SORTED_NS the mean launch times measured by
 * the last value-3 tuning, in ns (0 if none); GFW_TUNE_SORTED_WIDE_CHUNKS (query only) the
 * number of 64-entry runs of the column-sorted copy whose columns span more than 32767, so
 * that their entries read the column from the CSR instead (0 before the copy is built);
 * GFW_TUNE_GAUSS_METHOD (query only) the method a fully connected Gaussian graph sums its
 * products with, GFW_GAUSS_EXACT or GFW_GAUSS_GRID (what GFW_GAUSS_AUTO chose), 0 for a graph
 * given by its entries. */
typedef enum {
    GFW_TUNE_LABEL_PATH = 0,
    GFW_TUNE_LABEL_PLAIN_NS = 1,
    GFW_TUNE_LABEL_SORTED_NS = 2,
    GFW_TUNE_SORTED_WIDE_CHUNKS = 3,
    GFW_TUNE_GAUSS_METHOD = 4
} gfw_tune_t;
GFW_API gfw_status_t gfw_graph_tune(gfw_graph_t g, gfw_tune_t key, int64_t value);
GFW_API gfw_status_t gfw_graph_query(gfw_graph_t g, gfw_tune_t key, int64_t *value);

/* ---- solving ------------------------------------------------------------------------ */
/*
 * Runs Alg. 3 (or Alg. 2 with GFW_LMO_FULL, Alg. 4 with one_shot) on graph g.
 *  U_out      DEVICE n x K (dtype of g): the last iterate.                 (may be NULL)
 *  labels_out DEVICE int32[n]: lowest-index argmax of each row of U_out.   (may be NULL)
 *  s_out      DEVICE int32[n]: vertex index of every row of the last GLMO
 *             output S (S is one-hot in every row).                        (may be NULL)
 *  stats      HOST; history HOST double[5 * (max_iter + 1)]: rows E(U_k), g_k,
 *             q_k = <D_k, Hess E D_k>, alpha_k, number of non-binary rows, for every
 *             evaluated iterate k (NaN where not formed).  Either may be NULL; when
 *             either is given the call synchronises `stream`.
 * Ties in the argmin are broken towards the lowest class index.  The stop test g_k <= tol
 * is made after the GLMO and before the update.  Implementation note: L_s U_{k+1} is
 * obtained as (1 - a) L_s U_k + a L_s S_k (exact in real arithmetic) with a full SpMM at
 * the start and every p_refresh iterations.
 */
GFW_API gfw_status_t gfw_solve(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, void *U_out,
                       int32_t *labels_out, int32_t *s_out, gfw_stats_t *stats, double *history,
                       void *stream);

/*
 * Solves `count` independent problems with one batched launch sequence; graph i uses
 * prm[i] (prm may point to a single struct when `shared_params` is 1).  Outputs as in
 * gfw_solve (U_out / labels_out are arrays of DEVICE pointers, entries may be NULL;
 * stats may be NULL).  Every result equals what gfw_solve returns for that graph alone.
 */
GFW_API gfw_status_t gfw_solve_batched(gfw_context_t ctx, int32_t count, const gfw_graph_t *graphs,
                               const gfw_params_t *prm, int32_t shared_params, void *const *U_out,
                               int32_t *const *labels_out, gfw_stats_t *stats, void *stream);

/* E(U) from its definition (eq. gl_vv2) for a DEVICE U in the graph's dtype; synchronises. */
GFW_API gfw_status_t gfw_objective(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, const void *U,
                           double *E_host, void *stream);

/*
 * E(U) as gfw_objective computes it (the same kernels, the same result bit for bit), for
 * callers that cannot allocate memory: code under HIP graph capture, serving loops and
 * harnesses that forbid allocation.  Allocates nothing and does not synchronise: the result
 * goes to the DEVICE double *E_dev, ordered on `stream`.  Its block partials live in a fixed
 * scratch array of 3 x 65536 doubles (1.5 MiB) that the library holds on each device it
 * runs on until the process ends; graphs needing more partial blocks than that (n above
 * 16,777,216 for K <= 16, above 262,144 for K > 16) get GFW_E_UNSUPPORTED before any launch.
 * Every call on a device shares that device's array: calls that overlap on one device (on
 * different streams, or from different threads) race and must be serialised by the caller.
 */
GFW_API gfw_status_t gfw_objective_noalloc(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, const void *U,
                                   double *E_dev, void *stream);

/* P = L_s U (the graph-Laplacian times n x K product of eq. gradgl_vv2g); DEVICE U, P. */
GFW_API gfw_status_t gfw_spmm(gfw_context_t ctx, gfw_graph_t g, const void *U, void *P, void *stream);

/* ---- tracing ------------------------------------------------------------------------ */
/* Kernel classes of the hot path, for gfw_trace_get. */
typedef enum {
    GFW_KERNEL_ROW = 0,    /* pending update + gradient + GLMO + per-row partials           */
    GFW_KERNEL_LABEL = 1,  /* L_s S with one-hot S (label pass)                            */
    GFW_KERNEL_FINISH = 2, /* reductions, step size, stop test                             */
    GFW_KERNEL_SPMM = 3,   /* L_s U                                                          */
    GFW_KERNEL_COUNT = 4
} gfw_kernel_t;
/* enable: 0 = off; 1 = every hot-path launch made through ctx is bracketed by HIP events on
 * the launch stream; 2 = only the label passes (GFW_KERNEL_LABEL) are; 3 = only the row
 * kernels (GFW_KERNEL_ROW) of the iterations are.  While tracing,
 * gfw_solve launches each iteration's kernels one by one instead of replaying captured
 * iterations.  Durations are accumulated when the owning call completes (tracing makes
 * gfw_solve synchronise its stream).  gfw_trace_get returns the summed milliseconds and the
 * launch count of a kernel class since the last reset.  GFW_E_INVALID_ARG for another value
 * of enable. */
GFW_API gfw_status_t gfw_trace_enable(gfw_context_t ctx, int enable);
GFW_API gfw_status_t gfw_trace_reset(gfw_context_t ctx);
GFW_API gfw_status_t gfw_trace_get(gfw_context_t ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* Measurement aid, not part of the method: the achievable HBM rate on the context's
 * device, the ceiling the roofline figures are compared with beside the 8 TB/s spec peak.
 * Allocates two buffers of `bytes` (rounded down to 16), times `reps` launches of a streaming
 * 16-byte non-temporal copy kernel with HIP events on the null stream (synchronising the
 * device), frees the buffers and returns (bytes read + bytes written) per second in GB/s. */
GFW_API gfw_status_t gfw_copy_bandwidth(gfw_context_t ctx, size_t bytes, int32_t reps, double *gbs);

/* ---- serving ------------------------------------------------------------------------ */
/*
 * A request server: submitted problems (HOST arrays, copied at submit) are admitted while
 * their device footprint fits `hbm_budget_bytes` and fewer than `max_slots` run, stay
 * resident on the GPU and are advanced together by batched launches; new requests join
 * between macro-steps (continuous batching).  Each result equals the gfw_solve result of
 * the same problem alone.  gfw_server_submit checks sizes, row pointers, labels and
 * parameters (errors are returned at once); the CSR entries are checked on the device when
 * the request is admitted, and a malformed graph makes that request alone fail with
 * GFW_E_GRAPH at gfw_server_poll.  A worker thread runs the iterations while an admission
 * thread builds the graphs of admitted requests on a second stream.
 */
GFW_API gfw_status_t gfw_server_create(gfw_context_t ctx, size_t hbm_budget_bytes, int32_t max_slots,
                               gfw_server_t *out);
GFW_API gfw_status_t gfw_server_submit(gfw_server_t s, const gfw_problem_t *p, const gfw_params_t *prm,
                               uint64_t *ticket);
/* Copies the result into HOST buffers (U_out n x K of the problem's dtype, labels_out
 * int32[n]; either may be NULL).  blocking = 0 returns GFW_E_NOT_READY if unfinished. */
GFW_API gfw_status_t gfw_server_poll(gfw_server_t s, uint64_t ticket, int blocking, void *U_out,
                             int32_t *labels_out, gfw_stats_t *stats);
GFW_API gfw_status_t gfw_server_destroy(gfw_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* GFW_H */
