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
    void *U = nullptr, *P = nullptr, *Q = nullptr; // n x K of the graph dtype
    uint8_t *s0 = nullptr, *s1 = nullptr;          // vertex indices (ping-pong)
    double *row_part = nullptr, *lab_part = nullptr, *scratch = nullptr;
    Ctl *ctl = nullptr;
    double *hist = nullptr;
    int64_t hist_cap = 0;
    // captured chunk of iterations (depends only on the buffers above)
    hipGraphExec_t iter_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    int32_t *h_flag = nullptr; // pinned host copies of the active flag
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

// Launch shape derived from the graph (fixed per graph, so reductions are deterministic
// for that graph whatever else runs).
struct Shape {
    int kmax = 4;       // register bucket for K
    int lpr = 8;        // lanes per row of the CSR kernels
    int nb_row = 1;     // blocks of the row kernel
    int nb_csr = 1;     // blocks of the CSR kernels
};

} // namespace gfw

struct gfw_context_s {
    int device = 0;
    int num_cu = 0;
    std::string arch;
    // tracing: events bracketing hot-path launches, resolved when the owning call ends
    bool trace = false;
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
hipEvent_t trace_begin(gfw_context_s *c, hipStream_t st);
void trace_end(gfw_context_s *c, int kernel, hipEvent_t a, hipStream_t st);
// Waits for `st` and folds the pending records into the totals.
gfw_status_t trace_flush(gfw_context_s *c, hipStream_t st);
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
    int32_t *tile_rows = nullptr; // int32[n_tiles + 1]
    int32_t *gcol = nullptr;      // int32[nnz], columns sorted within each tile
    uint16_t *gpos = nullptr;     // uint16[nnz], CSR offset inside the tile
    double locality = 0.0;        // mean distinct 128-node label lines per 64 consecutive entries
    int diag_one = 1;           // 1: operator is I + A (kind W); 0: operator is A (kind L)
    gfw::Shape shape;
    gfw::Workspace ws;
    size_t graph_bytes = 0, solve_bytes = 0;
};
