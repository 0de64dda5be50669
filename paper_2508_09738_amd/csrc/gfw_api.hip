// Host side of libgfw: argument checks, graph set-up, the solve loop, objective and
// SpMM entry points.  See include/gfw.h for the contract of every exported function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <thread>
#include <vector>

#include "gfw_internal.h"
#include "gfw_kernels_bigk.h"

namespace gfw {

// Block partials of gfw_objective_noalloc, [3][kNoAllocMaxBlocks] (1.5 MiB), held by every
// device the library runs on until the process ends.  Host code never passes this name to a
// kernel: it uses the device address taken with hipGetSymbolAddress at context creation.
constexpr int kNoAllocMaxBlocks = 65536;
static __device__ __align__(256) double scratch[3 * kNoAllocMaxBlocks];

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

gfw_status_t fail(gfw_status_t s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

// --------------------------------------------------------------------------------------
// tracing
// --------------------------------------------------------------------------------------

static hipEvent_t pool_event(gfw_context_s *c)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

hipEvent_t trace_begin(gfw_context_s *c, int kernel, hipStream_t st)
{
    if (!c || !c->trace || !((c->trace_mask >> kernel) & 1u)) return nullptr;
    hipEvent_t a = pool_event(c);
    if (a) (void)hipEventRecord(a, st);
    return a;
}

void trace_end(gfw_context_s *c, int kernel, hipEvent_t a, hipStream_t st)
{
    if (!c || !c->trace || !a) return;
    hipEvent_t b = pool_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c->pending.push_back({kernel, a, b});
}

gfw_status_t trace_flush(gfw_context_s *c, hipStream_t st)
{
    if (!c || c->pending.empty()) {
        if (c) c->ev_used = 0;
        return GFW_OK;
    }
    GFW_HIP_TRY(hipStreamSynchronize(st));
    for (const auto &r : c->pending) {
        float ms = 0.f;
        GFW_HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        c->trace_ms[r.kernel] += ms;
        c->trace_n[r.kernel] += 1;
    }
    c->pending.clear();
    c->ev_used = 0;
    return GFW_OK;
}

// --------------------------------------------------------------------------------------
// host validation (shared by gfw_check_problem and gfw_graph_create for host input)
// --------------------------------------------------------------------------------------

static gfw_status_t check_scalars(const gfw_problem_t *p)
{
    if (!p) return fail(GFW_E_INVALID_ARG, "problem is NULL");
    if (p->n < 1) return fail(GFW_E_INVALID_ARG, "n must be >= 1 (got %lld)", (long long)p->n);
    if (p->n >= (int64_t)INT32_MAX) return fail(GFW_E_UNSUPPORTED, "n must be < 2^31 - 1");
    if (p->K < 2) return fail(GFW_E_INVALID_ARG, "K must be >= 2 (got %d)", p->K);
    if (p->K > GFW_MAX_K) return fail(GFW_E_UNSUPPORTED, "K must be <= %d (got %d)", GFW_MAX_K, p->K);
    if (p->nnz < 0) return fail(GFW_E_INVALID_ARG, "nnz must be >= 0");
    if (p->nnz >= ((int64_t)1 << 31)) return fail(GFW_E_GRAPH, "nnz must be < 2^31");
    if (p->kind != GFW_GRAPH_W && p->kind != GFW_GRAPH_L) return fail(GFW_E_INVALID_ARG, "bad graph kind");
    if (p->dtype != GFW_F32 && p->dtype != GFW_F64) return fail(GFW_E_INVALID_ARG, "bad dtype");
    if (p->location != GFW_HOST && p->location != GFW_DEVICE) return fail(GFW_E_INVALID_ARG, "bad location");
    if (!p->row_ptr) return fail(GFW_E_INVALID_ARG, "row_ptr is NULL");
    if (p->nnz > 0 && !p->col_idx) return fail(GFW_E_INVALID_ARG, "col_idx is NULL");
    if (!p->vals && p->kind == GFW_GRAPH_L) return fail(GFW_E_INVALID_ARG, "vals may be NULL only for kind W");
    if (p->n_labelled < 0 || p->n_labelled > p->n) return fail(GFW_E_LABELS, "n_labelled out of range");
    if (p->n_labelled > 0 && (!p->labelled_idx || !p->labels))
        return fail(GFW_E_INVALID_ARG, "labelled_idx / labels is NULL");
    return GFW_OK;
}

template <typename T>
static gfw_status_t validate_host_graph(const gfw_problem_t *p)
{
    const int64_t n = p->n, nnz = p->nnz;
    const int64_t *rp = p->row_ptr;
    const int32_t *ci = p->col_idx;
    const T *w = (const T *)p->vals;
    if (rp[0] != 0) return fail(GFW_E_GRAPH, "row_ptr[0] must be 0");
    if (rp[n] != nnz) return fail(GFW_E_GRAPH, "row_ptr[n] (%lld) != nnz (%lld)", (long long)rp[n], (long long)nnz);
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(GFW_E_GRAPH, "row_ptr decreases at row %lld", (long long)i);
    for (int64_t i = 0; i < n; ++i) {
        int32_t prev = -1;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t j = ci[q];
            if (j < 0 || j >= n) return fail(GFW_E_GRAPH, "column %d out of range in row %lld", j, (long long)i);
            if (j <= prev) return fail(GFW_E_GRAPH, "columns of row %lld unsorted or repeated", (long long)i);
            prev = j;
            if (w) {
                const double v = (double)w[q];
                if (!std::isfinite(v)) return fail(GFW_E_GRAPH, "non-finite value in row %lld", (long long)i);
                if (p->kind == GFW_GRAPH_W && v < 0.0)
                    return fail(GFW_E_GRAPH, "negative weight in row %lld", (long long)i);
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t j = ci[q];
            const int32_t *b = ci + rp[j], *e = ci + rp[j + 1];
            const int32_t *f = std::lower_bound(b, e, (int32_t)i);
            if (f == e || *f != i)
                return fail(GFW_E_GRAPH, "pattern not symmetric: (%lld,%d) has no mirror", (long long)i, j);
            if (w && w[f - ci] != w[q])
                return fail(GFW_E_GRAPH, "values not symmetric at (%lld,%d)", (long long)i, j);
        }
    }
    return GFW_OK;
}

static gfw_status_t validate_host_labels(const gfw_problem_t *p)
{
    std::vector<char> seen((size_t)p->n, 0);
    for (int64_t t = 0; t < p->n_labelled; ++t) {
        const int32_t i = p->labelled_idx[t], c = p->labels[t];
        if (i < 0 || i >= p->n) return fail(GFW_E_LABELS, "labelled index %d out of range", i);
        if (seen[(size_t)i]) return fail(GFW_E_LABELS, "labelled index %d repeated", i);
        seen[(size_t)i] = 1;
        if (c < 0 || c >= p->K) return fail(GFW_E_LABELS, "label %d of node %d not in [0,K)", c, i);
    }
    return GFW_OK;
}

// The O(n) part of the host checks: sizes, row pointers, labelled set.  The O(nnz) part
// (column range and order, values, symmetry) runs on the device when a graph is created.
gfw_status_t check_problem_light(const gfw_problem_t *p)
{
    gfw_status_t s = check_scalars(p);
    if (s != GFW_OK || p->location != GFW_HOST) return s;
    const int64_t n = p->n, nnz = p->nnz;
    const int64_t *rp = p->row_ptr;
    if (rp[0] != 0) return fail(GFW_E_GRAPH, "row_ptr[0] must be 0");
    if (rp[n] != nnz) return fail(GFW_E_GRAPH, "row_ptr[n] (%lld) != nnz (%lld)", (long long)rp[n], (long long)nnz);
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(GFW_E_GRAPH, "row_ptr decreases at row %lld", (long long)i);
    return validate_host_labels(p);
}

gfw_status_t check_problem(const gfw_problem_t *p)
{
    gfw_status_t s = check_scalars(p);
    if (s != GFW_OK || p->location != GFW_HOST) return s;
    s = p->dtype == GFW_F32 ? validate_host_graph<float>(p) : validate_host_graph<double>(p);
    if (s != GFW_OK) return s;
    return validate_host_labels(p);
}

gfw_status_t check_params(const gfw_params_t *p, int32_t K)
{
    if (!p) return fail(GFW_E_INVALID_ARG, "params is NULL");
    if (!(p->eps > 0.0)) return fail(GFW_E_INVALID_ARG, "eps must be > 0 (got %g)", p->eps);
    if (!(p->omega0 >= 0.0) || std::isinf(p->omega0)) return fail(GFW_E_INVALID_ARG, "omega0 must be finite and >= 0");
    if (p->max_iter < 0) return fail(GFW_E_INVALID_ARG, "max_iter must be >= 0");
    if (std::isnan(p->tol)) return fail(GFW_E_INVALID_ARG, "tol is NaN");
    if (p->ls != GFW_LS_ARMIJO && p->ls != GFW_LS_EXACT && p->ls != GFW_LS_SHORT)
        return fail(GFW_E_INVALID_ARG, "bad line search");
    if (p->ls == GFW_LS_ARMIJO) {
        if (!(p->delta > 0.0 && p->delta < 1.0)) return fail(GFW_E_INVALID_ARG, "delta must be in (0,1)");
        if (!(p->gamma > 0.0 && p->gamma < 0.5)) return fail(GFW_E_INVALID_ARG, "gamma must be in (0,1/2)");
    }
    if (p->lmo != GFW_LMO_GREEDY && p->lmo != GFW_LMO_FULL) return fail(GFW_E_INVALID_ARG, "bad lmo");
    if (p->one_shot != 0 && p->one_shot != 1) return fail(GFW_E_INVALID_ARG, "one_shot must be 0 or 1");
    if (std::isnan(p->lipschitz)) return fail(GFW_E_INVALID_ARG, "lipschitz is NaN");
    if (p->p_refresh < 0) return fail(GFW_E_INVALID_ARG, "p_refresh must be >= 0");
    if (p->incremental != 0 && p->incremental != 1) return fail(GFW_E_INVALID_ARG, "incremental must be 0 or 1");
    if (p->incremental) {
        if (!p->U0) return fail(GFW_E_INVALID_ARG, "an incremental solve starts from U0");
        if (p->lmo != GFW_LMO_GREEDY) return fail(GFW_E_INVALID_ARG, "an incremental solve needs the GLMO");
        if (p->p_refresh != 0) return fail(GFW_E_INVALID_ARG, "an incremental solve takes p_refresh = 0");
        if (K > 16) return fail(GFW_E_UNSUPPORTED, "incremental solves take K <= 16");
    }
    if (K < 2) return fail(GFW_E_INVALID_ARG, "K must be >= 2");
    return GFW_OK;
}

// --------------------------------------------------------------------------------------
// graph set-up
// --------------------------------------------------------------------------------------

static Shape shape_for(int64_t n, int32_t K)
{
    Shape s;
    // K <= 16: register buckets of the row-per-thread kernels; above: 64 * (classes per lane)
    s.kmax = K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : 64 * (int)cdiv(K, 64);
    s.nb_row = (int)cdiv(n, kRowBlock);
    s.nb_big = K > 16 ? (int)cdiv(n, kBigRowsPerBlock) : 0;
    return s;
}


void free_graph(gfw_graph_s *g)
{
    if (!g) return;
    gauss_free(g->gauss);
    dfree(g->row_ptr);
    dfree(g->col);
    dfree(g->vals);
    dfree(g->lab);
    dfree(g->tile_rows);
    dfree(g->tile_chunk);
    dfree(g->ganch);
    dfree(g->gword);
    Workspace &w = g->ws;
    dfree(w.U);
    dfree(w.P);
    dfree(w.Q);
    dfree(w.s0);
    dfree(w.s1);
    dfree(w.s4);
    dfree(w.nv);
    dfree(w.row_part);
    dfree(w.lab_part);
    dfree(w.row_fold);
    dfree(w.scratch);
    dfree(w.ctl);
    dfree(w.hist);
    dfree(w.act_moving);
    dfree(w.act_cnt);
    dfree(w.act_rows);
    dfree(w.act_m);
    if (w.iter_exec) (void)hipGraphExecDestroy(w.iter_exec);
    if (w.cap_stream) (void)hipStreamDestroy(w.cap_stream);
    if (w.h_flag) (void)hipHostFree(w.h_flag);
    for (int i = 0; i < 2; ++i)
        if (w.poll_ev[i]) (void)hipEventDestroy(w.poll_ev[i]);
    delete g;
}

template <typename T>
static gfw_status_t form_operator(gfw_graph_s *g, const T *wdev, hipStream_t st)
{
    double *dinv = nullptr, *rho = nullptr, *rmax = nullptr;
    GFW_HIP_TRY(hipMalloc(&dinv, sizeof(double) * g->n));
    GFW_HIP_TRY(hipMalloc(&rho, sizeof(double) * g->n));
    GFW_HIP_TRY(hipMalloc(&rmax, sizeof(double)));
    T *a = (T *)g->vals;
    if (g->kind == GFW_GRAPH_W) {
        k_degrees<T><<<grid_for(g->n, 256), 256, 0, st>>>(g->n, g->row_ptr, wdev, dinv);
        k_scale_values<T><<<grid_for(g->n, 256), 256, 0, st>>>(g->n, g->row_ptr, g->col, wdev, dinv, a, rho);
        g->diag_one = 1;
    } else {
        GFW_HIP_TRY(hipMemcpyAsync(a, wdev, sizeof(T) * g->nnz, hipMemcpyDeviceToDevice, st));
        k_rho_plain<T><<<grid_for(g->n, 256), 256, 0, st>>>(g->n, g->row_ptr, a, rho);
        g->diag_one = 0;
    }
    const unsigned long long zero = 0; // the bit pattern of +0.0
    GFW_HIP_TRY(hipMemcpyAsync(rmax, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
    k_max_nonneg<<<(unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(g->n, 1024), 1), 1024), 256, 0, st>>>(
        rho, g->n, (unsigned long long *)rmax);
    GFW_HIP_TRY(hipGetLastError());
    GFW_HIP_TRY(hipMemcpyAsync(&g->rho_max, rmax, sizeof(double), hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    dfree(dinv);
    dfree(rho);
    dfree(rmax);
    return GFW_OK;
}

// Mean number of distinct 128-node label lines touched by 64 consecutive CSR entries
// (sampled): about 64 when the neighbours of consecutive rows are scattered over the graph,
// a few when they are local (grids, ordered meshes).
static double label_locality(int64_t nnz, const int32_t *col)
{
    if (nnz < 64) return 0.0;
    const int samples = 256;
    double tot = 0.0;
    for (int t = 0; t < samples; ++t) {
        const int64_t e = (nnz - 64) * (int64_t)t / samples;
        int32_t lines[64];
        for (int q = 0; q < 64; ++q) lines[q] = col[e + q] >> 7;
        std::sort(lines, lines + 64);
        tot += (double)(std::unique(lines, lines + 64) - lines);
    }
    return tot / samples;
}

// Entries per tile of the column-sorted label pass.  A CU runs one tile at a time, and the
// tiles of a launch cost about the same, so the launch takes as many rounds as the tile count
// divided by the CU count, rounded up: the target is the largest tile size (densest gathers)
// whose tiles fill a whole number of rounds.  Tiles are whole 256-row blocks (the blocks of
// the row kernel, which the persistent iteration kernel runs inside a tile), and the greedy
// tiling closes a tile only when the next block would pass the target, so every closed tile
// holds more than target - maxblock entries (maxblock: the most entries of any 256-row block)
// and there are at most cus * R tiles.
int64_t sorted_tile_target(int64_t nnz, int64_t maxblock, int64_t cus, int64_t *rounds)
{
    if (rounds) *rounds = 0;
    if (maxblock >= kSortedMaxEntries) return kSortedMaxEntries;
    const int64_t room = kSortedMaxEntries - maxblock;
    int64_t R = std::max<int64_t>(1, cdiv(nnz, cus * room));
    for (;; ++R) {
        const int64_t t = cdiv(nnz, std::max<int64_t>(cus * R - 1, 1)) + maxblock;
        if (t <= kSortedMaxEntries) {
            if (rounds) *rounds = R;
            return std::max<int64_t>(t, 1);
        }
    }
}

// Tiles closed by the entry target number fewer than cus * R (each holds more than
// nnz / (cus * R - 1) entries); the row cap closes at most n / rcap more; one is last.
int64_t sorted_tile_bound(int64_t n, int64_t nnz, int64_t maxblock, int64_t cus)
{
    int64_t R = 0;
    (void)sorted_tile_target(nnz, maxblock, cus, &R);
    if (R == 0) return cdiv(n, kRowBlock) + 1; // a block fills a whole tile: at most one tile per block
    return cus * R + cdiv(n, kSortedRowCap) + 1;
}

// The most entries of any 256-row block of a CSR with host row pointers rp.
template <typename I>
int64_t max_block_entries(int64_t n, const I *rp)
{
    int64_t m = 0;
    for (int64_t b = 0; b < n; b += kRowBlock) m = std::max<int64_t>(m, (int64_t)(rp[std::min(n, b + kRowBlock)] - rp[b]));
    return m;
}
template int64_t max_block_entries<int32_t>(int64_t, const int32_t *);
template int64_t max_block_entries<int64_t>(int64_t, const int64_t *);

// The buffers of ensure_workspace except the per-iteration history (5 doubles per iteration).
void refresh_solve_bytes(gfw_graph_s *g)
{
    const size_t vs = dsize(g->dtype), n = (size_t)g->n, K = (size_t)g->K, nnz = (size_t)g->nnz;
    const size_t nb = (size_t)g->shape.nb_row;
    const size_t row_parts = kRowParts * std::max<size_t>(nb, (size_t)g->shape.nb_big);
    const size_t lab = std::max<size_t>(nb, (size_t)g->n_tiles) // label partials, folded row partials
                       + kRowParts * std::max<size_t>((size_t)g->n_tiles, K > 16 ? nb : 0);
    const size_t scratch = 3 * std::max<size_t>({nb, (size_t)g->shape.nb_big, 64});
    g->solve_bytes = (2 * vs + 8) * n * K               // U, Q; P in FP64
                     + (K > 16 ? 4 * n + 2 * nnz : 2 * n) // vertex pair (and nv for K > 16)
                     + (n + 1) / 2                        // packed vertices
                     + sizeof(double) * (row_parts + lab + scratch) + sizeof(Ctl);
}

// Row tiles for the column-sorted label pass (whole 256-row blocks, at most kSortedRowCap
// rows) and the per-tile column order of the entries.
static gfw_status_t build_sorted_tiles(gfw_graph_s *g, const int32_t *rp, const int32_t *col, hipStream_t st)
{
    const int64_t n = g->n;
    const int64_t maxblock = max_block_entries<int32_t>(n, rp);
    if (maxblock > kSortedMaxEntries)
        return fail(GFW_E_UNSUPPORTED, "a 256-row block has more than %d entries", kSortedMaxEntries);
    const int cus = std::max(1, g->ctx->num_cu);
    const int64_t target = sorted_tile_target(g->nnz, maxblock, cus);
    std::vector<int32_t> tr;
    int64_t emax = 0, rmax = 0;
    // greedy tiling: a tile closes when the next block would pass the entry target or the
    // row cap
    auto tiling = [&](int64_t rcap) {
        tr.assign(1, 0);
        int64_t cr = 0, ce = 0;
        emax = 0;
        rmax = 0;
        for (int64_t b = 0; b < n; b += kRowBlock) {
            const int64_t rows = std::min<int64_t>(kRowBlock, n - b);
            const int64_t d = rp[b + rows] - rp[b];
            if (cr + rows > rcap || ce + d > target) {
                tr.push_back((int32_t)b);
                cr = 0;
                ce = 0;
            }
            cr += rows;
            ce += d;
            emax = std::max(emax, ce);
            rmax = std::max(rmax, cr);
        }
        tr.push_back((int32_t)n);
    };
    tiling(kSortedRowCap);
    const int32_t nt = (int32_t)tr.size() - 1;
    const int64_t nnz = g->nnz;
    // chunks of kSortedChunk sorted entries, aligned to the start of each tile
    std::vector<int32_t> tc((size_t)nt + 1);
    tc[0] = 0;
    for (int32_t t = 0; t < nt; ++t) tc[t + 1] = tc[t] + (int32_t)cdiv(rp[tr[t + 1]] - rp[tr[t]], kSortedChunk);
    const int32_t nch = tc[nt];
    std::vector<uint32_t> sw((size_t)std::max<int64_t>(nnz, 1));
    std::vector<int32_t> an((size_t)std::max<int32_t>(nch, 1));
    std::vector<int64_t> wide(16, 0);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < nth; ++w) {
        pool.emplace_back([&, w]() {
            std::vector<uint64_t> key;
            for (int32_t t = (int32_t)w; t < nt; t += (int32_t)nth) {
                const int64_t e0 = rp[tr[t]], e1 = rp[tr[t + 1]];
                key.resize((size_t)(e1 - e0));
                for (int64_t e = e0; e < e1; ++e)
                    key[(size_t)(e - e0)] = ((uint64_t)(uint32_t)col[e] << kSortedOffsetBits) | (uint64_t)(e - e0);
                std::sort(key.begin(), key.end());
                for (int64_t c0 = 0; c0 < e1 - e0; c0 += kSortedChunk) {
                    const int64_t c1 = std::min<int64_t>(e1 - e0, c0 + kSortedChunk);
                    const int32_t lo = (int32_t)(key[(size_t)c0] >> kSortedOffsetBits);
                    const int32_t hi = (int32_t)(key[(size_t)(c1 - 1)] >> kSortedOffsetBits);
                    const bool fits = hi - lo <= kSortedMaxSpan;
                    an[(size_t)(tc[t] + c0 / kSortedChunk)] = fits ? lo : -1;
                    wide[w] += fits ? 0 : 1;
                    for (int64_t q = c0; q < c1; ++q) {
                        const uint32_t off = (uint32_t)(key[(size_t)q] & kSortedOffsetMask);
                        const uint32_t dc = fits ? (uint32_t)((int32_t)(key[(size_t)q] >> kSortedOffsetBits) - lo) : 0u;
                        sw[(size_t)(e0 + q)] = (dc << kSortedOffsetBits) | off;
                    }
                }
            }
        });
    }
    for (auto &th : pool) th.join();
    dfree(g->tile_rows);
    dfree(g->tile_chunk);
    dfree(g->ganch);
    dfree(g->gword);
    g->tile_rows = nullptr;
    g->tile_chunk = nullptr;
    g->ganch = nullptr;
    g->gword = nullptr;
    if (hipMalloc(&g->tile_rows, sizeof(int32_t) * (nt + 1)) != hipSuccess ||
        hipMalloc(&g->tile_chunk, sizeof(int32_t) * (nt + 1)) != hipSuccess ||
        hipMalloc(&g->ganch, sizeof(int32_t) * std::max<int32_t>(nch, 1)) != hipSuccess ||
        hipMalloc(&g->gword, sizeof(uint32_t) * std::max<int64_t>(nnz, 1)) != hipSuccess)
        return fail(GFW_E_NOMEM, "device allocation for the sorted label pass failed");
    GFW_HIP_TRY(hipMemcpyAsync(g->tile_rows, tr.data(), sizeof(int32_t) * (nt + 1), hipMemcpyHostToDevice, st));
    GFW_HIP_TRY(hipMemcpyAsync(g->tile_chunk, tc.data(), sizeof(int32_t) * (nt + 1), hipMemcpyHostToDevice, st));
    if (nnz) {
        GFW_HIP_TRY(hipMemcpyAsync(g->ganch, an.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipMemcpyAsync(g->gword, sw.data(), sizeof(uint32_t) * nnz, hipMemcpyHostToDevice, st));
    }
    GFW_HIP_TRY(hipStreamSynchronize(st));
    g->n_tiles = nt;
    g->tile_rows_max = (int32_t)rmax;
    refresh_solve_bytes(g);
    g->sorted_lds = (int32_t)std::max<int64_t>(16, (emax + 15) / 16 * 16);
    g->wide_chunks = 0;
    for (int64_t x : wide) g->wide_chunks += x;
    g->graph_bytes += sizeof(int32_t) * (2 * (size_t)(nt + 1) + (size_t)std::max<int32_t>(nch, 1)) + 4 * (size_t)nnz;
    return GFW_OK;
}

// Chooses and prepares the label path: the column-sorted pass for large graphs whose
// neighbour labels are scattered, the plain pass otherwise.  mode: 0 auto, 1 plain, 2 sorted.
// host_col: the column indices in host memory when the caller has them (else they are
// copied back from the device when needed).
static gfw_status_t choose_label_path(gfw_graph_s *g, int mode, hipStream_t st, const int32_t *host_col = nullptr);
static gfw_status_t measure_label_paths(gfw_graph_s *g, hipStream_t st);

static gfw_status_t choose_label_path(gfw_graph_s *g, int mode, hipStream_t st, const int32_t *host_col)
{
    if (mode == 3) return measure_label_paths(g, st);
    if (mode == 1) {
        g->label_path = 0;
        return GFW_OK;
    }
    if (g->K > 16) { // the large-K kernels have one label pass (the sorted one packs K <= 16)
        if (mode == 2) return fail(GFW_E_UNSUPPORTED, "the column-sorted label pass needs K <= 16");
        g->label_path = 0;
        return GFW_OK;
    }
    const bool big = g->nnz >= ((int64_t)4 << 20);
    if (mode == 0 && !big) { // small graphs keep the plain pass whatever their locality
        g->label_path = 0;
        return GFW_OK;
    }
    std::vector<int32_t> col;
    if (!host_col) {
        col.resize((size_t)std::max<int64_t>(g->nnz, 1));
        if (g->nnz) GFW_HIP_TRY(hipMemcpyAsync(col.data(), g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        host_col = col.data();
    }
    g->locality = label_locality(g->nnz, host_col);
    const bool want = mode == 2 || g->locality > 16.0;
    if (!want) {
        g->label_path = 0;
        return GFW_OK;
    }
    if (!g->gword) {
        std::vector<int32_t> rp((size_t)g->n + 1);
        GFW_HIP_TRY(hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        gfw_status_t s = build_sorted_tiles(g, rp.data(), host_col, st);
        if (s != GFW_OK) {
            if (mode == 2) return s;
            g->label_path = 0; // a row too long for the sorted tiles: keep the plain pass
            return GFW_OK;
        }
    }
    g->label_path = 1;
    if (g->ws.iter_exec) { // the captured iteration graph holds the previous label kernel
        (void)hipGraphExecDestroy(g->ws.iter_exec);
        g->ws.iter_exec = nullptr;
    }
    return GFW_OK;
}

gfw_status_t graph_create(gfw_context_s *ctx, const gfw_problem_t *p, gfw_graph_s **out, hipStream_t st,
                          bool validated)
{
    gfw_status_t s = validated ? GFW_OK : check_problem_light(p);
    if (s != GFW_OK) return s;
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    gfw_graph_s *g = new (std::nothrow) gfw_graph_s();
    if (!g) return fail(GFW_E_NOMEM, "host allocation failed");
    g->ctx = ctx;
    g->n = p->n;
    g->nnz = p->nnz;
    g->K = p->K;
    g->dtype = p->dtype;
    g->kind = p->kind;
    g->n_labelled = p->n_labelled;
    const size_t vs = dsize(p->dtype);
    const int64_t n = p->n, nnz = p->nnz;
    struct Guard {
        gfw_graph_s *g;
        ~Guard() { if (g) free_graph(g); }
    } guard{g};
    auto dalloc = [&](void **ptr, size_t bytes) -> gfw_status_t {
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return fail(GFW_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        return GFW_OK;
    };
    if ((s = dalloc((void **)&g->row_ptr, 4 * (n + 1))) != GFW_OK) return s;
    if ((s = dalloc((void **)&g->col, 4 * nnz)) != GFW_OK) return s;
    if ((s = dalloc(&g->vals, vs * nnz)) != GFW_OK) return s;
    if ((s = dalloc((void **)&g->lab, 4 * n)) != GFW_OK) return s;

    // raw weights staged on the device (the scaled operator overwrites g->vals later)
    void *wraw = nullptr;
    unsigned int *flags = nullptr;
    if ((s = dalloc((void **)&flags, sizeof(unsigned int))) != GFW_OK) return s;
    unsigned int zero = 0;
    GFW_HIP_TRY(hipMemcpyAsync(flags, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
    k_fill_i32<<<grid_for(n, 256), 256, 0, st>>>(n, g->lab, -1);

    if (p->location == GFW_HOST) {
        // the row pointers (checked on the host) go up as int64 for the entry checks on the
        // device, then are narrowed; columns and values are checked where they land
        int64_t *rp64 = nullptr;
        if ((s = dalloc((void **)&rp64, 8 * (n + 1))) != GFW_OK) { dfree(flags); return s; }
        GFW_HIP_TRY(hipMemcpyAsync(rp64, p->row_ptr, 8 * (n + 1), hipMemcpyHostToDevice, st));
        if (nnz) GFW_HIP_TRY(hipMemcpyAsync(g->col, p->col_idx, 4 * nnz, hipMemcpyHostToDevice, st));
        if (p->vals) {
            if ((s = dalloc(&wraw, vs * nnz)) != GFW_OK) { dfree(flags); dfree(rp64); return s; }
            if (nnz) GFW_HIP_TRY(hipMemcpyAsync(wraw, p->vals, vs * nnz, hipMemcpyHostToDevice, st));
        }
        if (p->dtype == GFW_F32)
            k_validate_graph<float><<<grid_for(n, 256), 256, 0, st>>>(n, nnz, rp64, g->col, (const float *)wraw,
                                                                     p->kind == GFW_GRAPH_L, flags);
        else
            k_validate_graph<double><<<grid_for(n, 256), 256, 0, st>>>(n, nnz, rp64, g->col, (const double *)wraw,
                                                                      p->kind == GFW_GRAPH_L, flags);
        k_rowptr_narrow<<<grid_for(n + 1, 256), 256, 0, st>>>(n, rp64, g->row_ptr);
        GFW_HIP_TRY(hipStreamSynchronize(st));
        dfree(rp64);
        if (p->n_labelled) {
            int32_t *ti = nullptr, *tl = nullptr;
            if ((s = dalloc((void **)&ti, 4 * p->n_labelled)) != GFW_OK) { dfree(flags); dfree(wraw); return s; }
            if ((s = dalloc((void **)&tl, 4 * p->n_labelled)) != GFW_OK) { dfree(flags); dfree(wraw); dfree(ti); return s; }
            GFW_HIP_TRY(hipMemcpyAsync(ti, p->labelled_idx, 4 * p->n_labelled, hipMemcpyHostToDevice, st));
            GFW_HIP_TRY(hipMemcpyAsync(tl, p->labels, 4 * p->n_labelled, hipMemcpyHostToDevice, st));
            k_scatter_labels<<<grid_for(p->n_labelled, 256), 256, 0, st>>>(n, p->n_labelled, p->K, ti, tl, g->lab, flags);
            GFW_HIP_TRY(hipStreamSynchronize(st));
            dfree(ti);
            dfree(tl);
        }
    } else {
        // device input: bounds of row_ptr first, then a validation kernel
        int64_t ends[2] = {0, 0};
        GFW_HIP_TRY(hipMemcpyAsync(&ends[0], p->row_ptr, 8, hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipMemcpyAsync(&ends[1], p->row_ptr + n, 8, hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        if (ends[0] != 0 || ends[1] != nnz) {
            dfree(flags);
            return fail(GFW_E_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        }
        if (p->dtype == GFW_F32)
            k_validate_graph<float><<<grid_for(n, 256), 256, 0, st>>>(n, nnz, p->row_ptr, p->col_idx,
                                                                     (const float *)p->vals, p->kind == GFW_GRAPH_L, flags);
        else
            k_validate_graph<double><<<grid_for(n, 256), 256, 0, st>>>(n, nnz, p->row_ptr, p->col_idx,
                                                                      (const double *)p->vals, p->kind == GFW_GRAPH_L, flags);
        if (p->n_labelled)
            k_scatter_labels<<<grid_for(p->n_labelled, 256), 256, 0, st>>>(n, p->n_labelled, p->K, p->labelled_idx,
                                                                             p->labels, g->lab, flags);
        unsigned int hf = 0;
        GFW_HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        if (hf & 1u) { dfree(flags); return fail(GFW_E_GRAPH, "CSR malformed (row_ptr, column range or order)"); }
        if (hf & 4u) { dfree(flags); return fail(GFW_E_GRAPH, "negative or non-finite weight"); }
        if (hf & 2u) { dfree(flags); return fail(GFW_E_GRAPH, "graph is not symmetric"); }
        if (hf & 8u) { dfree(flags); return fail(GFW_E_LABELS, "labelled set invalid (range, repeat or class)"); }
        k_rowptr_narrow<<<grid_for(n + 1, 256), 256, 0, st>>>(n, p->row_ptr, g->row_ptr);
        if (nnz) GFW_HIP_TRY(hipMemcpyAsync(g->col, p->col_idx, 4 * nnz, hipMemcpyDeviceToDevice, st));
        if (p->vals) {
            if ((s = dalloc(&wraw, vs * nnz)) != GFW_OK) { dfree(flags); return s; }
            if (nnz) GFW_HIP_TRY(hipMemcpyAsync(wraw, p->vals, vs * nnz, hipMemcpyDeviceToDevice, st));
        }
    }
    GFW_HIP_TRY(hipGetLastError());
    if (p->location == GFW_HOST) {
        unsigned int hf = 0;
        GFW_HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        const char *what = (hf & 1u) ? "CSR malformed (column range or order)"
                           : (hf & 4u) ? "negative or non-finite weight"
                           : (hf & 2u) ? "graph is not symmetric" : nullptr;
        if (what) { dfree(flags); dfree(wraw); return fail(GFW_E_GRAPH, "%s", what); }
        if (hf) { dfree(flags); dfree(wraw); return fail(GFW_E_LABELS, "labelled set invalid"); }
    }
    dfree(flags);
    s = p->dtype == GFW_F32 ? form_operator<float>(g, (const float *)wraw, st)
                            : form_operator<double>(g, (const double *)wraw, st);
    dfree(wraw);
    if (s != GFW_OK) return s;
    g->shape = shape_for(n, p->K);
    if ((s = choose_label_path(g, 0, st, p->location == GFW_HOST ? p->col_idx : nullptr)) != GFW_OK) return s;
    g->graph_bytes += 4 * (n + 1) + (4 + vs) * nnz + 4 * n;
    refresh_solve_bytes(g);
    guard.g = nullptr;
    *out = g;
    return GFW_OK;
}

gfw_status_t ensure_workspace(gfw_graph_s *g, int32_t max_iter)
{
    Workspace &w = g->ws;
    const size_t vs = dsize(g->dtype);
    const size_t nK = (size_t)g->n * g->K;
    auto dalloc = [&](void **ptr, size_t bytes) -> gfw_status_t {
        if (*ptr) return GFW_OK;
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return fail(GFW_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        return GFW_OK;
    };
    gfw_status_t s;
    if ((s = dalloc(&w.U, vs * nK)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.P, sizeof(double) * nK)) != GFW_OK) return s;
    if ((s = dalloc(&w.Q, vs * nK)) != GFW_OK) return s;
    const size_t sb = g->K > 16 ? 2 : 1; // vertex bytes: 16-bit for the large-K kernels
    if ((s = dalloc((void **)&w.s0, sb * g->n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.s1, sb * g->n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.s4, (size_t)(g->n + 1) / 2)) != GFW_OK) return s;
    if (g->K > 16 && (s = dalloc((void **)&w.nv, sizeof(uint16_t) * (size_t)g->nnz)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.row_part, sizeof(double) * kRowParts * std::max(g->shape.nb_row, g->shape.nb_big)))
        != GFW_OK) return s;
    // one label-pass partial per 256-row block (plain pass) or per tile (sorted pass, whose
    // tiles may be built after the first solve: then the buffer grows, and the captured
    // iterations, which hold the old buffer, are dropped)
    const int64_t need_lab = std::max<int64_t>(g->shape.nb_row, g->n_tiles);
    if (w.lab_part && w.lab_cap < need_lab) {
        if (w.iter_exec) {
            (void)hipGraphExecDestroy(w.iter_exec);
            w.iter_exec = nullptr;
        }
        dfree(w.lab_part);
        w.lab_part = nullptr;
    }
    if (!w.lab_part) {
        if ((s = dalloc((void **)&w.lab_part, sizeof(double) * need_lab)) != GFW_OK) return s;
        w.lab_cap = need_lab;
    }
    const int64_t need_fold = std::max<int64_t>(g->n_tiles, g->K > 16 ? g->shape.nb_row : 0);
    if (need_fold > 0 && w.fold_cap < need_fold) { // row partials folded by the label pass
        if (w.iter_exec) {
            (void)hipGraphExecDestroy(w.iter_exec);
            w.iter_exec = nullptr;
        }
        dfree(w.row_fold);
        w.row_fold = nullptr;
        if ((s = dalloc((void **)&w.row_fold, sizeof(double) * kRowParts * (size_t)need_fold)) != GFW_OK) return s;
        w.fold_cap = need_fold;
    }
    if ((s = dalloc((void **)&w.scratch, sizeof(double) * 3 * std::max({g->shape.nb_row, g->shape.nb_big, 64}))) !=
        GFW_OK)
        return s;
    if ((s = dalloc((void **)&w.ctl, sizeof(Ctl))) != GFW_OK) return s;
    const int64_t need = 5 * ((int64_t)max_iter + 1);
    if (w.hist_cap < need) {
        dfree(w.hist);
        w.hist = nullptr;
        if ((s = dalloc((void **)&w.hist, sizeof(double) * need)) != GFW_OK) return s;
        w.hist_cap = need;
    }
    return GFW_OK;
}

// --------------------------------------------------------------------------------------
// kernel dispatch
// --------------------------------------------------------------------------------------


// every register bucket with kernels: the row-per-thread buckets and 64 * (1..16)
#define GFW_FOR_EACH_KMAX(X) \
    X(4) X(8) X(16) X(64) X(128) X(192) X(256) X(320) X(384) X(448) X(512) X(576) X(640) X(704) X(768) X(832) \
    X(896) X(960) X(1024)

// The single-graph column-sorted pass and row kernel are instantiated for every class count
// K <= 16: each entry's histogram update, and each row's class loops, cost K steps instead of
// the bucket's.  Classes past K take no part in any result, so every instantiation gives the
// same results (the batched launches use the buckets).
#define GFW_FOR_EACH_SORTED_K(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename T, int KMAX>
static void set_lds_limits()
{
    if constexpr (KMAX <= 16) { // the large-K kernels use static LDS only
        // the largest dynamic LDS any launch of these kernels asks for
#define GFW_SET_SORTED(KX)                                                                                       \
    (void)hipFuncSetAttribute((const void *)k_label_sorted<T, uint8_t, KX>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              kSortedMaxEntries);                                                                \
    (void)hipFuncSetAttribute((const void *)k_row<T, uint8_t, KX>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                              (int)row_lds_per_class<T>() * KX);
        GFW_FOR_EACH_SORTED_K(GFW_SET_SORTED)
#undef GFW_SET_SORTED
        (void)hipFuncSetAttribute((const void *)k_row<T, uint8_t, KMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)row_lds_per_class<T>() * KMAX);
    }
}

template <typename T>
static void launch_label_sorted(const gfw_graph_s *g, hipStream_t st)
{
    switch (g->K) {
#define GFW_SORTED_CASE(KX)                                                                                      \
    case KX:                                                                                                     \
        k_label_sorted<T, uint8_t, KX><<<g->n_tiles, kSortedThreads, g->sorted_lds, st>>>(make_view<T>(g));      \
        break;
        GFW_FOR_EACH_SORTED_K(GFW_SORTED_CASE)
#undef GFW_SORTED_CASE
    default: break; // K > 16 has no sorted pass
    }
}

static size_t row_lds_bytes(const gfw_graph_s *g)
{
    return (g->dtype == GFW_F32 ? row_lds_per_class<float>() : row_lds_per_class<double>()) * (size_t)g->K;
}

template <typename T>
static void launch_row_exact(const gfw_graph_s *g, int apply_only, hipStream_t st)
{
    switch (g->K) {
#define GFW_ROW_CASE(KX)                                                                                         \
    case KX:                                                                                                     \
        k_row<T, uint8_t, KX><<<g->shape.nb_row, kRowBlock, row_lds_bytes(g), st>>>(make_view<T>(g), apply_only); \
        break;
        GFW_FOR_EACH_SORTED_K(GFW_ROW_CASE)
#undef GFW_ROW_CASE
    default: break; // K > 16 runs the large-K row kernel
    }
}


template <typename T, int KMAX, typename PT>
static void launch_spmm(const gfw_graph_s *g, const T *U, PT *P, hipStream_t st)
{
    if constexpr (KMAX > 16)
        k_spmm_big<T, KMAX / 64, PT><<<g->shape.nb_big, kBigThreads, 0, st>>>(make_view<T>(g), U, P);
    else
        k_spmm<T, KMAX, PT><<<g->shape.nb_row, kSpmmThreads, 0, st>>>(make_view<T>(g), U, P);
}

template <typename T, int KMAX>
static void launch_label(const gfw_graph_s *g, hipStream_t st)
{
    if constexpr (KMAX > 16) {
        k_label_big<T><<<g->shape.nb_row, kRowBlock, 0, st>>>(make_view<T>(g));
    } else if (g->gauss) {
        gauss_label<T>(g, st);
    } else if (g->label_path == 1) {
        launch_label_sorted<T>(g, st);
    } else {
        const size_t lds = sizeof(T) * kRowBlock * g->K;
        k_label<T, uint8_t, KMAX><<<g->shape.nb_row, kRowBlock, lds, st>>>(make_view<T>(g));
    }
}

// Mean duration of `reps` launches of the graph's current label pass, timed with events.
// The pass reads whatever vertices the workspace holds (any values give the same work).
template <typename T, int KMAX>
static float time_label_pass(gfw_graph_s *g, hipStream_t st, int reps)
{
    if constexpr (KMAX > 16) {
        return 0.0f;
    } else {
        static const bool lds_set = (set_lds_limits<T, KMAX>(), true);
        (void)lds_set;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return -1.0f;
        }
        launch_label<T, KMAX>(g, st); // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r) launch_label<T, KMAX>(g, st);
        (void)hipEventRecord(e1, st);
        float ms = -1.0f;
        if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ms < 0.0f ? -1.0f : 1e3f * ms / (float)reps;
    }
}

template <typename T>
static float time_label_any(gfw_graph_s *g, hipStream_t st, int reps)
{
    switch (g->shape.kmax) {
    case 4: return time_label_pass<T, 4>(g, st, reps);
    case 8: return time_label_pass<T, 8>(g, st, reps);
    case 16: return time_label_pass<T, 16>(g, st, reps);
    default: return 0.0f;
    }
}

// Measured choice of the label pass: both passes run on the graph itself (the column-sorted
// copy is built if needed) and the faster one is kept.  Both give the same Q bit for bit.
static gfw_status_t measure_label_paths(gfw_graph_s *g, hipStream_t st)
{
    if (g->K > 16) { // one label pass for many classes
        g->label_path = 0;
        return GFW_OK;
    }
    gfw_status_t s = choose_label_path(g, 2, st); // builds the sorted tiles once
    if (s != GFW_OK) {
        g->label_path = 0; // a row too long for the sorted tiles: the plain pass it is
        return GFW_OK;
    }
    if ((s = ensure_workspace(g, 0)) != GFW_OK) return s;
    Workspace &w = g->ws;
    Ctl c;
    std::memset(&c, 0, sizeof(c));
    c.active = 1;
    c.last_eval = -1;
    // a ticket count the timed passes never complete: no launch makes the finish of an
    // iteration, so every launch does the same work
    c.ticket = 0x80000000u;
    GFW_HIP_TRY(hipMemcpyAsync(w.ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
    GFW_HIP_TRY(hipMemsetAsync(w.s0, 0, g->n, st));
    GFW_HIP_TRY(hipMemsetAsync(w.s4, 0, (size_t)(g->n + 1) / 2, st));
    constexpr int reps = 5;
    float us[2];
    for (int path = 0; path < 2; ++path) {
        g->label_path = path;
        us[path] = g->dtype == GFW_F32 ? time_label_any<float>(g, st, reps) : time_label_any<double>(g, st, reps);
        GFW_HIP_TRY(hipGetLastError());
        if (us[path] < 0.0f) return fail(GFW_E_HIP, "timing the label passes failed");
    }
    g->label_us[0] = us[0];
    g->label_us[1] = us[1];
    g->label_path = us[1] < us[0] ? 1 : 0;
    return GFW_OK;
}

// P = L_s U with FP64 sums, stored as PT (the graph's dtype, or FP64 for the carried P)
template <typename T, typename PT>
static void spmm_any(const gfw_graph_s *g, const T *U, PT *P, hipStream_t st)
{
    if (g->gauss) return gauss_spmm<T, PT>(g, U, P, st);
    switch (g->shape.kmax) {
#define GFW_SPMM_CASE(KM) \
    case KM: launch_spmm<T, KM, PT>(g, U, P, st); break;
        GFW_FOR_EACH_KMAX(GFW_SPMM_CASE)
#undef GFW_SPMM_CASE
    default: break;
    }
}

SolveParams solve_params(const gfw_graph_s *g, const gfw_params_t *prm)
{
    SolveParams sp;
    sp.inv_eps = std::isinf(prm->eps) ? 0.0 : 1.0 / prm->eps;
    sp.omega0 = prm->omega0;
    sp.tol = prm->tol;
    sp.delta = prm->delta;
    sp.gamma = prm->gamma;
    sp.lipschitz = prm->lipschitz > 0.0 ? prm->lipschitz : g->rho_max + 2.0 * sp.inv_eps + prm->omega0;
    sp.ls = (int32_t)prm->ls;
    sp.lmo = (int32_t)prm->lmo;
    return sp;
}

template <typename T, int KMAX>
static void launch_row(gfw_graph_s *g, int apply_only, hipStream_t st)
{
    if constexpr (KMAX > 16)
        k_row_big<T, KMAX / 64><<<g->shape.nb_big, kBigThreads, 0, st>>>(make_view<T>(g), apply_only);
    else
        launch_row_exact<T>(g, apply_only, st);
}

// One GFW iteration (row kernel, label pass, finish), optionally bracketed by trace events.
// The iteration index lives in the device control block.
template <typename T, int KMAX>
static void launch_iteration(gfw_graph_s *g, hipStream_t st, bool traced)
{
    gfw_context_s *cx = traced ? g->ctx : nullptr;
    hipEvent_t ev = trace_begin(cx, GFW_KERNEL_ROW, st);
    launch_row<T, KMAX>(g, 0, st);
    trace_end(cx, GFW_KERNEL_ROW, ev, st);
    ev = trace_begin(cx, GFW_KERNEL_LABEL, st);
    launch_label<T, KMAX>(g, st);
    trace_end(cx, GFW_KERNEL_LABEL, ev, st);
    // the finish of the iteration is made by the label pass's last workgroup (finish_if_last)
}

constexpr int kGraphChunk = 16; // iterations per captured graph

// Captures kGraphChunk iterations once per graph object; the kernels take all per-solve
// values from the device control block, so the same executable graph serves every solve.
template <typename T, int KMAX>
static gfw_status_t ensure_iteration_graph(gfw_graph_s *g)
{
    Workspace &w = g->ws;
    if (w.iter_exec) return GFW_OK;
    if (!w.cap_stream) GFW_HIP_TRY(hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    GFW_HIP_TRY(hipStreamBeginCapture(w.cap_stream, hipStreamCaptureModeThreadLocal));
    for (int c = 0; c < kGraphChunk; ++c) launch_iteration<T, KMAX>(g, w.cap_stream, false);
    GFW_HIP_TRY(hipStreamEndCapture(w.cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&w.iter_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        w.iter_exec = nullptr;
        return fail(GFW_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    return GFW_OK;
}

template <typename T, int KMAX>
static gfw_status_t solve_impl(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                               int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st)
{
    gfw_status_t s = ensure_workspace(g, prm->max_iter);
    if (s != GFW_OK) return s;
    static const bool lds_set = (set_lds_limits<T, KMAX>(), true); // once per instantiation, thread-safe
    (void)lds_set;
    Workspace &w = g->ws;
    T *U = (T *)w.U;
    double *P = w.P;
    gfw_context_s *cx = g->ctx;
    Ctl c0;
    std::memset(&c0, 0, sizeof(c0));
    c0.active = prm->max_iter > 0 ? 1 : 0;
    c0.max_iter = prm->max_iter;
    c0.one_shot = prm->one_shot;
    c0.last_eval = -1;
    c0.alpha = 0.0;
    c0.alpha_last = std::numeric_limits<double>::quiet_NaN();
    c0.gap = std::numeric_limits<double>::quiet_NaN();
    c0.sp = solve_params(g, prm);
    c0.hist = w.hist;
    c0.hist_stride = prm->max_iter + 1;
    GFW_HIP_TRY(hipMemcpyAsync(w.ctl, &c0, sizeof(c0), hipMemcpyHostToDevice, st));
    k_init_u<T><<<g->shape.nb_row, kRowBlock, 0, st>>>(make_view<T>(g), (const T *)prm->U0);
    hipEvent_t ev = trace_begin(cx, GFW_KERNEL_SPMM, st);
    spmm_any<T>(g, U, P, st);
    trace_end(cx, GFW_KERNEL_SPMM, ev, st);
    const bool use_graph = !cx->trace && prm->p_refresh == 0 && prm->max_iter >= kGraphChunk;
    if (use_graph) {
        if ((s = ensure_iteration_graph<T, KMAX>(g)) != GFW_OK) return s;
        if (!w.h_flag) GFW_HIP_TRY(hipHostMalloc((void **)&w.h_flag, 2 * sizeof(int32_t), hipHostMallocDefault));
        for (int i = 0; i < 2; ++i)
            if (!w.poll_ev[i]) GFW_HIP_TRY(hipEventCreateWithFlags(&w.poll_ev[i], hipEventDisableTiming));
        // replays; extra iterations past the stop are no-ops.  The stop flag is read back one
        // replay behind, so the queue always holds a replay while the host waits.
        const int reps = (int)cdiv(prm->max_iter, kGraphChunk);
        for (int r = 0; r < reps; ++r) {
            GFW_HIP_TRY(hipGraphLaunch(w.iter_exec, st));
            if (prm->tol < 0.0 && !prm->one_shot) continue; // no early stop to watch for
            GFW_HIP_TRY(hipMemcpyAsync(&w.h_flag[r & 1], &w.ctl->active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            GFW_HIP_TRY(hipEventRecord(w.poll_ev[r & 1], st));
            if (r >= 1) {
                GFW_HIP_TRY(hipEventSynchronize(w.poll_ev[(r - 1) & 1]));
                if (w.h_flag[(r - 1) & 1] == 0) break;
            }
        }
    } else {
        for (int32_t k = 0; k < prm->max_iter; ++k) {
            if (prm->p_refresh > 0 && k > 0 && k % prm->p_refresh == 0) {
                launch_row<T, KMAX>(g, 1, st);
                k_clear_pending<<<1, 64, 0, st>>>(w.ctl);
                spmm_any<T>(g, U, P, st);
            }
            launch_iteration<T, KMAX>(g, st, cx->trace);
        }
    }
    // commit the last pending update
    launch_row<T, KMAX>(g, 1, st);
    GFW_HIP_TRY(hipGetLastError());
    if ((s = trace_flush(cx, st)) != GFW_OK) return s;
    return solve_outputs(g, prm, U_out, labels_out, s_out, stats, history, st);
}

template <typename T, typename ST>
static gfw_status_t solve_outputs_t(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                                    int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st)
{
    Workspace &w = g->ws;
    const T *U = (const T *)w.U;
    const int64_t nK = g->n * g->K;
    if (U_out) GFW_HIP_TRY(hipMemcpyAsync(U_out, U, sizeof(T) * nK, hipMemcpyDeviceToDevice, st));
    if (labels_out || s_out)
        k_outputs<T, ST><<<grid_for(g->n, 256), 256, 0, st>>>(g->n, g->K, U, (const ST *)w.s0, (const ST *)w.s1,
                                                             w.ctl, labels_out, s_out);
    GFW_HIP_TRY(hipGetLastError());
    if (stats || history) {
        Ctl ch;
        GFW_HIP_TRY(hipMemcpyAsync(&ch, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        std::vector<double> hh;
        if (history) {
            hh.resize(5 * ((size_t)prm->max_iter + 1));
            GFW_HIP_TRY(hipMemcpyAsync(hh.data(), w.hist, sizeof(double) * hh.size(), hipMemcpyDeviceToHost, st));
        }
        GFW_HIP_TRY(hipStreamSynchronize(st));
        if (history) {
            const int64_t hs = (int64_t)prm->max_iter + 1;
            const int32_t nev = ch.last_eval + 1; // evaluated iterates
            for (int64_t t = 0; t < 5 * hs; ++t) {
                const int64_t k = t % hs;
                history[t] = k < nev ? hh[(size_t)t] : std::numeric_limits<double>::quiet_NaN();
            }
        }
        if (stats) {
            stats->iters = ch.iters;
            stats->stop_reason = ch.stop_reason;
            stats->gap = ch.gap;
            stats->alpha_last = ch.alpha_last;
            stats->objective = std::numeric_limits<double>::quiet_NaN();
        }
    }
    return GFW_OK;
}

gfw_status_t solve_outputs(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out, int32_t *s_out,
                           gfw_stats_t *stats, double *history, hipStream_t st)
{
    if (g->dtype == GFW_F32)
        return g->K > 16 ? solve_outputs_t<float, uint16_t>(g, prm, U_out, labels_out, s_out, stats, history, st)
                         : solve_outputs_t<float, uint8_t>(g, prm, U_out, labels_out, s_out, stats, history, st);
    return g->K > 16 ? solve_outputs_t<double, uint16_t>(g, prm, U_out, labels_out, s_out, stats, history, st)
                     : solve_outputs_t<double, uint8_t>(g, prm, U_out, labels_out, s_out, stats, history, st);
}

template <typename T>
static gfw_status_t solve_dispatch(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                                   int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st)
{
    switch (g->shape.kmax) {
#define GFW_SOLVE_CASE(KM) \
    case KM: return solve_impl<T, KM>(g, prm, U_out, labels_out, s_out, stats, history, st);
        GFW_FOR_EACH_KMAX(GFW_SOLVE_CASE)
#undef GFW_SOLVE_CASE
    default: return fail(GFW_E_UNSUPPORTED, "no kernels for K = %d", g->K);
    }
}

// Block partials of E(U) (no P buffer: each row of L U is used where it is formed); returns
// the number of partials per quantity written to part ([3][count]).
template <typename T>
static int energy_partials(const gfw_graph_s *g, const T *U, double omega0, double *part, hipStream_t st)
{
    if (g->gauss) return gauss_energy<T>(g, U, omega0, part, st);
    const GraphView<T> v = make_view<T>(g);
    switch (g->shape.kmax) {
    case 4: k_energy<T, 4><<<g->shape.nb_row, kSpmmThreads, 0, st>>>(v, U, omega0, part); return g->shape.nb_row;
    case 8: k_energy<T, 8><<<g->shape.nb_row, kSpmmThreads, 0, st>>>(v, U, omega0, part); return g->shape.nb_row;
    case 16: k_energy<T, 16><<<g->shape.nb_row, kSpmmThreads, 0, st>>>(v, U, omega0, part); return g->shape.nb_row;
#define GFW_ENERGY_BIG(KM)                                                                                       \
    case KM: k_energy_big<T, KM / 64><<<g->shape.nb_big, kBigThreads, 0, st>>>(v, U, omega0, part);              \
        return g->shape.nb_big;
        GFW_ENERGY_BIG(64) GFW_ENERGY_BIG(128) GFW_ENERGY_BIG(192) GFW_ENERGY_BIG(256) GFW_ENERGY_BIG(320)
        GFW_ENERGY_BIG(384) GFW_ENERGY_BIG(448) GFW_ENERGY_BIG(512) GFW_ENERGY_BIG(576) GFW_ENERGY_BIG(640)
        GFW_ENERGY_BIG(704) GFW_ENERGY_BIG(768) GFW_ENERGY_BIG(832) GFW_ENERGY_BIG(896) GFW_ENERGY_BIG(960)
        GFW_ENERGY_BIG(1024)
#undef GFW_ENERGY_BIG
    default: return 0;
    }
}

// Stream-ordered E(U) into device memory *E_dev: block partials in part ([3][blocks]), then a
// fixed-order sum.
template <typename T>
static gfw_status_t objective_to_device(const gfw_graph_s *g, const gfw_params_t *prm, const T *U, double *part,
                                        double *E_dev, hipStream_t st)
{
    const int nb = energy_partials<T>(g, U, prm->omega0, part, st);
    if (nb <= 0) return fail(GFW_E_UNSUPPORTED, "no kernels for K = %d", g->K);
    const double inv_eps = std::isinf(prm->eps) ? 0.0 : 1.0 / prm->eps;
    k_energy_sum<<<1, kFinishThreads, 0, st>>>(part, nb, inv_eps, E_dev);
    GFW_HIP_TRY(hipGetLastError());
    return GFW_OK;
}

gfw_status_t objective_on_device(const gfw_graph_s *g, const gfw_params_t *prm, const void *U, double *part,
                                 double *E_dev, hipStream_t st)
{
    return g->dtype == GFW_F32 ? objective_to_device<float>(g, prm, (const float *)U, part, E_dev, st)
                               : objective_to_device<double>(g, prm, (const double *)U, part, E_dev, st);
}

template <typename T>
static gfw_status_t objective_impl(gfw_graph_s *g, const gfw_params_t *prm, const T *U, double *E, hipStream_t st)
{
    gfw_status_t s = ensure_workspace(g, 0);
    if (s != GFW_OK) return s;
    if ((s = objective_to_device<T>(g, prm, U, g->ws.scratch, g->ws.row_part, st)) != GFW_OK) return s;
    GFW_HIP_TRY(hipMemcpyAsync(E, g->ws.row_part, sizeof(double), hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    return GFW_OK;
}

} // namespace gfw

using namespace gfw;

// ======================================================================================
// exported C ABI
// ======================================================================================

extern "C" {

const char *gfw_status_string(gfw_status_t s)
{
    switch (s) {
    case GFW_OK: return "ok";
    case GFW_E_INVALID_ARG: return "invalid argument";
    case GFW_E_GRAPH: return "malformed graph";
    case GFW_E_LABELS: return "invalid labelled set";
    case GFW_E_NOMEM: return "out of device memory";
    case GFW_E_HIP: return "HIP runtime error";
    case GFW_E_UNSUPPORTED: return "unsupported";
    case GFW_E_BUDGET: return "over the HBM budget";
    case GFW_E_NOT_READY: return "not ready";
    case GFW_E_NUMERIC: return "numeric failure (NaN)";
    }
    return "unknown status";
}

const char *gfw_last_error(void) { return gfw::g_last_error; }

void gfw_params_default(gfw_params_t *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eps = 50.0;
    p->omega0 = 1000.0;
    p->max_iter = 30;
    p->tol = 1e-6;
    p->ls = GFW_LS_ARMIJO;
    p->delta = 0.5;
    p->gamma = 1e-6;
    p->lmo = GFW_LMO_GREEDY;
    p->one_shot = 0;
    p->lipschitz = 0.0;
    p->U0 = nullptr;
    p->p_refresh = 0;
    p->incremental = 0;
}

gfw_status_t gfw_check_problem(const gfw_problem_t *p) { return check_problem(p); }

gfw_status_t gfw_check_params(const gfw_params_t *p, int32_t K) { return check_params(p, K); }

gfw_status_t gfw_context_create(gfw_context_t *ctx, int device)
{
    if (!ctx) return fail(GFW_E_INVALID_ARG, "ctx is NULL");
    *ctx = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(GFW_E_HIP, "no HIP device available");
    if (device < 0 || device >= count) return fail(GFW_E_INVALID_ARG, "device %d out of range", device);
    hipDeviceProp_t prop;
    GFW_HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GFW_E_UNSUPPORTED, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
    gfw_context_s *c = new (std::nothrow) gfw_context_s();
    if (!c) return fail(GFW_E_NOMEM, "host allocation failed");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    // the scratch array of gfw_objective_noalloc on this device, taken with the device current
    hipError_t e2 = hipSetDevice(device);
    if (e2 == hipSuccess) e2 = hipGetSymbolAddress((void **)&c->noalloc_scratch, HIP_SYMBOL(gfw::scratch));
    if (e2 != hipSuccess || !c->noalloc_scratch) {
        delete c;
        return fail(GFW_E_HIP, "hipGetSymbolAddress of the objective scratch failed on device %d: %s", device,
                    hipGetErrorString(e2));
    }
    *ctx = c;
    return GFW_OK;
}

gfw_status_t gfw_context_destroy(gfw_context_t ctx)
{
    if (ctx)
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return GFW_OK;
}

gfw_status_t gfw_graph_create(gfw_context_t ctx, const gfw_problem_t *p, gfw_graph_t *out, void *stream)
{
    if (!ctx || !out) return fail(GFW_E_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    return graph_create(ctx, p, out, (hipStream_t)stream);
}

gfw_status_t gfw_graph_destroy(gfw_graph_t g)
{
    if (g) (void)hipDeviceSynchronize();
    free_graph(g);
    return GFW_OK;
}

gfw_status_t gfw_graph_footprint(gfw_graph_t g, size_t *graph_bytes, size_t *solve_bytes)
{
    if (!g) return fail(GFW_E_INVALID_ARG, "graph is NULL");
    if (graph_bytes) *graph_bytes = g->graph_bytes;
    if (solve_bytes) *solve_bytes = g->solve_bytes;
    return GFW_OK;
}

gfw_status_t gfw_graph_tune(gfw_graph_t g, gfw_tune_t key, int64_t value)
{
    if (!g) return fail(GFW_E_INVALID_ARG, "graph is NULL");
    if (key != GFW_TUNE_LABEL_PATH) return fail(GFW_E_INVALID_ARG, "unknown tuning key %d", (int)key);
    if (value < 0 || value > 3) return fail(GFW_E_INVALID_ARG, "label path must be 0, 1, 2 or 3");
    if (g->gauss) return fail(GFW_E_UNSUPPORTED, "a Gaussian graph has one label pass");
    GFW_HIP_TRY(hipSetDevice(g->ctx->device));
    const int before = g->label_path;
    gfw_status_t s = choose_label_path(g, (int)value, nullptr);
    if (s == GFW_OK && before != g->label_path && g->ws.iter_exec) {
        (void)hipGraphExecDestroy(g->ws.iter_exec);
        g->ws.iter_exec = nullptr;
    }
    return s;
}

gfw_status_t gfw_graph_query(gfw_graph_t g, gfw_tune_t key, int64_t *value)
{
    if (!g || !value) return fail(GFW_E_INVALID_ARG, "NULL argument");
    switch (key) {
    case GFW_TUNE_LABEL_PATH: *value = g->label_path == 1 ? 2 : 1; return GFW_OK;
    case GFW_TUNE_LABEL_PLAIN_NS: *value = (int64_t)(1e3 * g->label_us[0]); return GFW_OK;
    case GFW_TUNE_LABEL_SORTED_NS: *value = (int64_t)(1e3 * g->label_us[1]); return GFW_OK;
    case GFW_TUNE_SORTED_WIDE_CHUNKS: *value = g->wide_chunks; return GFW_OK;
    case GFW_TUNE_GAUSS_METHOD: *value = g->gauss ? gauss_method(g->gauss) : 0; return GFW_OK;
    default: return fail(GFW_E_INVALID_ARG, "unknown tuning key %d", (int)key);
    }
}

gfw_status_t gfw_solve(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                       int32_t *s_out, gfw_stats_t *stats, double *history, void *stream)
{
    if (!ctx || !g) return fail(GFW_E_INVALID_ARG, "ctx or graph is NULL");
    gfw_status_t s = check_params(prm, g->K);
    if (s != GFW_OK) return s;
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (prm->incremental) {
        if (g->gauss) return fail(GFW_E_UNSUPPORTED, "incremental solves take CSR graphs");
        s = solve_incremental(g, prm, U_out, labels_out, s_out, stats, history, st);
    } else {
        s = g->dtype == GFW_F32 ? solve_dispatch<float>(g, prm, U_out, labels_out, s_out, stats, history, st)
                                : solve_dispatch<double>(g, prm, U_out, labels_out, s_out, stats, history, st);
    }
    if (s != GFW_OK) return s;
    if (stats) {
        double E = 0.0;
        s = g->dtype == GFW_F32 ? objective_impl<float>(g, prm, (const float *)g->ws.U, &E, st)
                                : objective_impl<double>(g, prm, (const double *)g->ws.U, &E, st);
        if (s != GFW_OK) return s;
        stats->objective = E;
        if (stats->stop_reason == GFW_STOP_NUMERIC) return fail(GFW_E_NUMERIC, "NaN met during the iteration");
    }
    return GFW_OK;
}

gfw_status_t gfw_objective(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, const void *U, double *E_host,
                           void *stream)
{
    if (!ctx || !g || !U || !E_host) return fail(GFW_E_INVALID_ARG, "NULL argument");
    gfw_status_t s = check_params(prm, g->K);
    if (s != GFW_OK) return s;
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    return g->dtype == GFW_F32 ? objective_impl<float>(g, prm, (const float *)U, E_host, (hipStream_t)stream)
                               : objective_impl<double>(g, prm, (const double *)U, E_host, (hipStream_t)stream);
}

gfw_status_t gfw_objective_noalloc(gfw_context_t ctx, gfw_graph_t g, const gfw_params_t *prm, const void *U,
                                   double *E_dev, void *stream)
{
    if (!ctx || !g || !U || !E_dev) return fail(GFW_E_INVALID_ARG, "NULL argument");
    gfw_status_t s = check_params(prm, g->K);
    if (s != GFW_OK) return s;
    const int blocks = g->K > 16 ? g->shape.nb_big : g->shape.nb_row;
    if (blocks > kNoAllocMaxBlocks)
        return fail(GFW_E_UNSUPPORTED,
                    "gfw_objective_noalloc: n = %lld needs %d partial blocks, above its fixed scratch of %d "
                    "(n <= %lld for K <= 16, n <= %lld for K > 16)",
                    (long long)g->n, blocks, kNoAllocMaxBlocks, (long long)kNoAllocMaxBlocks * kRowBlock,
                    (long long)kNoAllocMaxBlocks * kBigRowsPerBlock);
    if (!ctx->noalloc_scratch) return fail(GFW_E_HIP, "no objective scratch on device %d", ctx->device);
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    return g->dtype == GFW_F32
               ? objective_to_device<float>(g, prm, (const float *)U, ctx->noalloc_scratch, E_dev, st)
               : objective_to_device<double>(g, prm, (const double *)U, ctx->noalloc_scratch, E_dev, st);
}

gfw_status_t gfw_copy_bandwidth(gfw_context_t ctx, size_t bytes, int32_t reps, double *gbs)
{
    if (!ctx || !gbs || reps < 1 || bytes < 16) return fail(GFW_E_INVALID_ARG, "bad argument");
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n16 = (int64_t)(bytes / 16);
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, 16 * (size_t)n16) != hipSuccess) return fail(GFW_E_NOMEM, "copy buffer");
    if (hipMalloc(&b, 16 * (size_t)n16) != hipSuccess) {
        dfree(a);
        return fail(GFW_E_NOMEM, "copy buffer");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    gfw_status_t s = GFW_OK;
    float ms = 0.f;
    const int grid = std::max(1, ctx->num_cu) * 8;
    if (hipMemset(a, 0, 16 * (size_t)n16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        s = fail(GFW_E_HIP, "copy set-up failed");
    } else {
        k_stream_copy<<<grid, 256>>>((const v4u *)a, (v4u *)b, n16); // warm-up
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) k_stream_copy<<<grid, 256>>>((const v4u *)a, (v4u *)b, n16);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f)
            s = fail(GFW_E_HIP, "copy timing failed");
        else
            *gbs = 2.0 * 16.0 * (double)n16 * reps / (1e-3 * ms) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(a);
    dfree(b);
    return s;
}

gfw_status_t gfw_trace_enable(gfw_context_t ctx, int enable)
{
    if (!ctx) return fail(GFW_E_INVALID_ARG, "ctx is NULL");
    if (enable < 0 || enable > 3) return fail(GFW_E_INVALID_ARG, "trace mode must be 0, 1, 2 or 3 (got %d)", enable);
    ctx->trace = enable != 0;
    ctx->trace_mask = enable == 1   ? (1u << GFW_KERNEL_COUNT) - 1u
                      : enable == 2 ? 1u << GFW_KERNEL_LABEL
                      : enable == 3 ? 1u << GFW_KERNEL_ROW
                                    : 0u;
    return GFW_OK;
}

gfw_status_t gfw_trace_reset(gfw_context_t ctx)
{
    if (!ctx) return fail(GFW_E_INVALID_ARG, "ctx is NULL");
    for (int k = 0; k < GFW_KERNEL_COUNT; ++k) {
        ctx->trace_ms[k] = 0.0;
        ctx->trace_n[k] = 0;
    }
    return GFW_OK;
}

gfw_status_t gfw_trace_get(gfw_context_t ctx, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!ctx) return fail(GFW_E_INVALID_ARG, "ctx is NULL");
    if (kernel < 0 || kernel >= GFW_KERNEL_COUNT) return fail(GFW_E_INVALID_ARG, "bad kernel id %d", kernel);
    if (total_ms) *total_ms = ctx->trace_ms[kernel];
    if (launches) *launches = ctx->trace_n[kernel];
    return GFW_OK;
}

gfw_status_t gfw_spmm(gfw_context_t ctx, gfw_graph_t g, const void *U, void *P, void *stream)
{
    if (!ctx || !g || !U || !P) return fail(GFW_E_INVALID_ARG, "NULL argument");
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    if (g->dtype == GFW_F32) spmm_any<float>(g, (const float *)U, (float *)P, (hipStream_t)stream);
    else spmm_any<double>(g, (const double *)U, (double *)P, (hipStream_t)stream);
    GFW_HIP_TRY(hipGetLastError());
    return GFW_OK;
}

} // extern "C"
