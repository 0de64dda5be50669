// Internal declarations shared by the host-side translation units of libgfw.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gfw.h"
#include "gfw_kernels.h"

namespace gfw {

void set_error(const char *fmt, ...);
gfw_status_t fail(gfw_status_t s, const char *fmt, ...);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

inline int grid_for(int64_t work, int threads, int cap = 65535)
{
    int64_t b = cdiv(work > 1 ? work : 1, threads);
    return (int)(b < cap ? b : cap);
}

inline size_t dsize(gfw_dtype_t d) { return d == GFW_F32 ? 4 : 8; }

// Dynamic LDS of the row kernel per class of its bucket: a 256-row tile of U and Q in the
// graph's dtype and of P in FP64.
template <typename T>
constexpr size_t row_lds_per_class() { return (size_t)kRowBlock * (2 * sizeof(T) + sizeof(double)); }

#define GFW_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::gfw::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                     \
            return GFW_E_HIP;                                                               \
        }                                                                                   \
    } while (0)

// Per-solve device workspace, owned by a graph (one solve at a time per graph).
struct Workspace {
    void *U = nullptr, *Q = nullptr; // n x K of the graph dtype
    double *P = nullptr;             // n x K, L_s U carried in FP64
    uint8_t *s0 = nullptr, *s1 = nullptr;          // vertex indices (ping-pong)
    uint8_t *s4 = nullptr;                         // the current vertices packed two per byte (K <= 16)
    uint16_t *nv = nullptr;                        // per CSR entry, the vertex of its column (K > 16)
    double *row_part = nullptr, *lab_part = nullptr, *scratch = nullptr;
    int64_t lab_cap = 0; // entries of lab_part: one per 256-row block or per sorted tile
    double *row_fold = nullptr; // [kRowParts][n_fold]: row partials folded per label-pass block
    int64_t fold_cap = 0;       // blocks row_fold holds
    Ctl *ctl = nullptr;
    double *hist = nullptr;
    int64_t hist_cap = 0;
    // incremental solves (allocated at the first one): moving-row flags, block counts and
    // offsets, the moving rows and their count
    uint8_t *act_moving = nullptr;
    int32_t *act_cnt = nullptr, *act_rows = nullptr, *act_m = nullptr;
    // captured chunk of iterations (depends only on the buffers above)
    hipGraphExec_t iter_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    int32_t *h_flag = nullptr; // pinned host copies of the active flag
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

// Launch shape derived from the graph (fixed per graph, so reductions are deterministic
// for that graph whatever else runs).
struct Shape {
    int kmax = 4;       // register bucket for K: 4, 8, 16, or 64..1024 for the large-K kernels
    int nb_row = 1;     // 256-row blocks (row kernel, label passes, SpMM, set-up)
    int nb_big = 0;     // blocks of the large-K row kernel and SpMM (0 when K <= 16)
};

} // namespace gfw

struct gfw_context_s {
    int device = 0;
    int num_cu = 0;
    std::string arch;
    // device address of the file-scope scratch array of gfw_objective_noalloc on this
    // context's device (taken once, at context creation, with the device current)
    double *noalloc_scratch = nullptr;
    // tracing: events bracketing hot-path launches, resolved when the owning call ends
    bool trace = false;       // hot-path launches bracketed by events (no captured iterations)
    uint32_t trace_mask = 0;  // kernel classes timed while tracing (bit k: class k)
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    double trace_ms[GFW_KERNEL_COUNT] = {};
    int64_t trace_n[GFW_KERNEL_COUNT] = {};
};

namespace gfw {
// Records a start event for a traced launch (no-op when tracing is off); returns the
// event to hand to trace_end.
hipEvent_t trace_begin(gfw_context_s *c, int kernel, hipStream_t st);
void trace_end(gfw_context_s *c, int kernel, hipEvent_t a, hipStream_t st);
// Waits for `st` and folds the pending records into the totals.
gfw_status_t trace_flush(gfw_context_s *c, hipStream_t st);
} // namespace gfw

namespace gfw {
struct GaussGraph; // the operator of a fully connected Gaussian graph (gfw_gauss.hip)
} // namespace gfw

struct gfw_graph_s {
    gfw_context_s *ctx = nullptr;
    int64_t n = 0, nnz = 0;
    int32_t K = 0;
    gfw_dtype_t dtype = GFW_F32;
    gfw_graph_kind_t kind = GFW_GRAPH_W;
    int32_t *row_ptr = nullptr; // int32[n+1]
    int32_t *col = nullptr;     // int32[nnz]
    void *vals = nullptr;       // scaled operator values, dtype[nnz]
    int32_t *lab = nullptr;     // int32[n], class of labelled nodes, -1 elsewhere
    int64_t n_labelled = 0;
    double rho_max = 0.0;       // max Gershgorin radius of the operator
    // column-sorted copy of the CSR for the label pass (see k_label_sorted)
    int label_path = 0;         // 0: plain (k_label), 1: column-sorted (k_label_sorted)
    int32_t n_tiles = 0;
    int32_t tile_rows_max = 0;     // rows of the largest sorted tile
    int32_t *tile_rows = nullptr;  // int32[n_tiles + 1]
    int32_t *tile_chunk = nullptr; // int32[n_tiles + 1], first anchor of each tile
    int32_t *ganch = nullptr;      // int32[chunks], anchor column of each 64-entry chunk, -1: wide
    uint32_t *gword = nullptr;     // uint32[nnz], sorted within each tile: (col - anchor) << 17 | offset
    int64_t wide_chunks = 0;       // chunks whose columns span more than kSortedMaxSpan
    int32_t sorted_lds = 0;        // dynamic LDS of the sorted pass: bytes of the largest tile
    double locality = 0.0;        // mean distinct 128-node label lines per 64 consecutive entries
    float label_us[2] = {0, 0};   // measured launch times of the plain and sorted passes (0: not measured)
    int diag_one = 1;           // 1: operator is I + A (kind W); 0: operator is A (kind L)
    gfw::GaussGraph *gauss = nullptr; // fully connected Gaussian graph (no CSR), else null
    gfw::Shape shape;
    gfw::Workspace ws;
    size_t graph_bytes = 0, solve_bytes = 0;
};

namespace gfw {
gfw_status_t check_problem(const gfw_problem_t *p);       // every check, on the host
gfw_status_t check_problem_light(const gfw_problem_t *p); // sizes, row pointers, labels only
gfw_status_t check_params(const gfw_params_t *p, int32_t K);
// graph_create checks the CSR entries (column range and order, values, symmetry) on the
// device after the upload.  validated = true skips the O(n) host checks of check_problem_light,
// which the caller has already made (the server does so at submit).
gfw_status_t graph_create(gfw_context_s *ctx, const gfw_problem_t *p, gfw_graph_s **out, hipStream_t st,
                          bool validated = false);
void free_graph(gfw_graph_s *g);
gfw_status_t ensure_workspace(gfw_graph_s *g, int32_t max_iter);
// Column-sorted tiles (whole 256-row blocks): the entry target per tile for a graph of nnz
// entries whose fullest 256-row block has maxblock entries on a device of cus compute units
// (rounds: the launch's rounds of tiles), an upper bound of the resulting tile count for n
// rows, and the fullest block of a CSR with host row pointers.
constexpr int64_t kSortedRowCap = 16 * kSortedThreads; // rows per tile (a thread sums at most 16)
int64_t sorted_tile_target(int64_t nnz, int64_t maxblock, int64_t cus, int64_t *rounds = nullptr);
int64_t sorted_tile_bound(int64_t n, int64_t nnz, int64_t maxblock, int64_t cus);
template <typename I>
int64_t max_block_entries(int64_t n, const I *rp);
// Device bytes of one solve on the graph as it stands (its label pass included).
void refresh_solve_bytes(gfw_graph_s *g);
SolveParams solve_params(const gfw_graph_s *g, const gfw_params_t *prm);

// view of a graph and its solve workspace for the per-iteration kernels
// Label-pass blocks that fold the row kernel's partials for the finish: the sorted tiles, or
// the 256-row blocks of the large-K label pass; 0 on the plain pass.
inline int64_t fold_blocks(const gfw_graph_s *g)
{
    if (g->K > 16) return g->shape.nb_row;
    return g->label_path == 1 ? g->n_tiles : 0;
}

// Fully connected Gaussian graphs (gfw_gauss.hip): creation, release, and the three places
// where the iteration uses the operator: P = L_s U (stored as PT), the label pass Q = L_s S
// with its finish, and the block partials of E(U) (returns their count per quantity).
gfw_status_t gauss_graph_create(gfw_context_s *ctx, const gfw_gaussian_problem_t *p, gfw_graph_s **out,
                                hipStream_t st);
void gauss_free(GaussGraph *gg);
int gauss_method(const GaussGraph *gg); // GFW_GAUSS_EXACT or GFW_GAUSS_GRID
template <typename T, typename PT>
void gauss_spmm(const gfw_graph_s *g, const T *U, PT *P, hipStream_t st);
template <typename T>
void gauss_label(const gfw_graph_s *g, hipStream_t st);
template <typename T>
int gauss_energy(const gfw_graph_s *g, const T *U, double omega0, double *part, hipStream_t st);

// The outputs of a solve whose iterations have ended (U, labels, vertices, stats, history),
// E(U) into device memory (block partials in part), and the incremental solve
// (gfw_active.hip).
gfw_status_t solve_outputs(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out, int32_t *s_out,
                           gfw_stats_t *stats, double *history, hipStream_t st);
gfw_status_t objective_on_device(const gfw_graph_s *g, const gfw_params_t *prm, const void *U, double *part,
                                 double *E_dev, hipStream_t st);
gfw_status_t solve_incremental(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                               int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st);
SolveParams solve_params(const gfw_graph_s *g, const gfw_params_t *prm);

template <typename T>
GraphView<T> make_view(const gfw_graph_s *g)
{
    GraphView<T> v;
    const Workspace &w = g->ws;
    v.n = g->n;
    v.K = g->K;
    v.diag_one = g->diag_one;
    v.rp = g->row_ptr;
    v.ci = g->col;
    v.a = (const T *)g->vals;
    v.lab = g->lab;
    v.U = (T *)w.U;
    v.P = w.P;
    v.Q = (T *)w.Q;
    v.s0 = w.s0;
    v.s1 = w.s1;
    v.s4 = w.s4;
    v.nv = w.nv;
    v.ctl = w.ctl;
    v.row_part = w.row_part;
    v.lab_part = w.lab_part;
    v.n_fold = (int32_t)fold_blocks(g);
    v.row_fold = v.n_fold > 0 ? w.row_fold : nullptr;
    v.nb_row = g->shape.nb_row;
    v.nb_big = g->shape.nb_big;
    v.n_tiles = g->label_path == 1 ? g->n_tiles : 0;
    v.ticket = w.ctl ? &w.ctl->ticket : nullptr;
    v.n_lab_blocks = (g->K <= 16 && g->label_path == 1) ? g->n_tiles : g->shape.nb_row;
    v.tile_rows = g->tile_rows;
    v.tile_chunk = g->tile_chunk;
    v.ganch = g->ganch;
    v.gword = g->gword;
    return v;
}
} // namespace gfw
