// Batched solves and the request server of libgfw: many graphs advance in the same
// launches.  Every kernel here runs the same device functions as the single-graph path on
// the same tiles of each graph, so a graph's results do not depend on its companions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include <new>
#include <string>

#include "gfw_internal.h"
#include "gfw_kernels_bigk.h"

namespace gfw {

template <typename T, int KMAX>
static void set_batch_lds_limits()
{
    (void)hipFuncSetAttribute((const void *)k_label_sorted_batch<T, uint8_t, KMAX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kSortedMaxEntries);
    (void)hipFuncSetAttribute((const void *)k_row_batch<T, uint8_t, KMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)row_lds_per_class<T>() * KMAX);
}

// --------------------------------------------------------------------------------------
// batched solves
// --------------------------------------------------------------------------------------

static int bucket_of(int kmax) { return kmax == 4 ? 0 : kmax == 8 ? 1 : 2; }
// K > 16: classes per lane rounded up to 1, 2, 4, 8 or 16
constexpr int kBigBuckets = 5;
static int big_bucket_of(int kmax)
{
    const int mc = kmax / 64;
    return mc <= 1 ? 0 : mc <= 2 ? 1 : mc <= 4 ? 2 : mc <= 8 ? 3 : 4;
}

// A grow-only device array (kept across macro-steps of the server).
template <typename E>
struct DevArr {
    E *p = nullptr;
    size_t cap = 0;
    ~DevArr() { dfree(p); }
    gfw_status_t reserve(size_t n)
    {
        if (n <= cap) return GFW_OK;
        dfree(p);
        p = nullptr;
        cap = 0;
        const size_t c = n + n / 2 + 16;
        if (hipMalloc((void **)&p, sizeof(E) * c) != hipSuccess) return fail(GFW_E_NOMEM, "batch table allocation");
        cap = c;
        return GFW_OK;
    }
};

// Device tables of one batch: the graph views and, per K bucket, the (graph, tile) lists of
// the row-wise kernels and of the two label passes.  Reusable: prepare() refills them.
template <typename T>
struct BatchTables {
    std::vector<GraphView<T>> views;
    std::vector<TileRef> rows[3], plain[3], sorted[3], all_rows;
    int32_t sorted_lds[3] = {}; // dynamic LDS of a bucket's sorted launch: its largest tile
    int32_t lt[3] = {kLabelTile, kLabelTile, kLabelTile}; // sub-tile of a bucket's plain label launch
    std::vector<TileRef> big_rows[kBigBuckets], big_lab; // K > 16: row tiles per MC bucket, 256-row label tiles
    // host staging of the per-graph control blocks, U_0 pointers and label destinations; kept
    // here so that they outlive the asynchronous copies that read them
    std::vector<Ctl> ctl0;
    std::vector<const T *> u0;
    std::vector<int32_t *> lab_out;
    DevArr<GraphView<T>> dv;
    DevArr<TileRef> drows[3], dplain[3], dsorted[3], dall, dbig[kBigBuckets], dbiglab;
    DevArr<int32_t> dflag;
    DevArr<const T *> dU0;
    DevArr<int32_t *> dlab;
    DevArr<Ctl> dctl0, dctl_out;
    DevArr<double> dE;
    int32_t *h_flag = nullptr;
    // device pointers of the current contents
    GraphView<T> *d_views = nullptr;
    TileRef *d_rows[3] = {}, *d_plain[3] = {}, *d_sorted[3] = {}, *d_all = nullptr;
    TileRef *d_big[kBigBuckets] = {}, *d_biglab = nullptr;
    int32_t *d_flag = nullptr;
    const T **d_U0 = nullptr;
    int32_t **d_lab_out = nullptr;
    Ctl *d_ctl0 = nullptr, *d_ctl_out = nullptr;
    double *d_E = nullptr;
    void reset()
    {
        views.clear();
        for (int b = 0; b < 3; ++b) {
            rows[b].clear();
            plain[b].clear();
            sorted[b].clear();
            sorted_lds[b] = 0;
            lt[b] = kLabelTile;
        }
        all_rows.clear();
        for (int b = 0; b < kBigBuckets; ++b) big_rows[b].clear();
        big_lab.clear();
        d_U0 = nullptr;
        d_lab_out = nullptr;
    }
    ~BatchTables()
    {
        if (h_flag) (void)hipHostFree(h_flag);
    }
};

template <typename E>
static gfw_status_t upload(std::vector<E> &v, DevArr<E> &arr, E **d, hipStream_t st)
{
    if (v.empty()) {
        *d = nullptr;
        return GFW_OK;
    }
    gfw_status_t s = arr.reserve(v.size());
    if (s != GFW_OK) return s;
    *d = arr.p;
    GFW_HIP_TRY(hipMemcpyAsync(*d, v.data(), sizeof(E) * v.size(), hipMemcpyHostToDevice, st));
    return GFW_OK;
}

template <typename T>
static void batch_big_launch(BatchTables<T> &bt, int kind, int flag, hipStream_t st)
{
    // kind 0: row kernel (flag = apply_only); kind 1: SpMM P_0 = L_s U_0; kind 2: objective partials
#define GFW_BIG_BUCKET(B, MC)                                                                                    \
    if (!bt.big_rows[B].empty()) {                                                                             \
        if (kind == 0)                                                                                         \
            k_row_big_batch<T, MC><<<bt.big_rows[B].size(), kBigThreads, 0, st>>>(bt.d_views, bt.d_big[B], flag); \
        else if (kind == 1)                                                                                    \
            k_spmm_big_batch<T, MC><<<bt.big_rows[B].size(), kBigThreads, 0, st>>>(bt.d_views, bt.d_big[B]);   \
        else                                                                                                   \
            k_energy_big_batch<T, MC><<<bt.big_rows[B].size(), kBigThreads, 0, st>>>(bt.d_views, bt.d_big[B]); \
    }
    GFW_BIG_BUCKET(0, 1)
    GFW_BIG_BUCKET(1, 2)
    GFW_BIG_BUCKET(2, 4)
    GFW_BIG_BUCKET(3, 8)
    GFW_BIG_BUCKET(4, 16)
#undef GFW_BIG_BUCKET
}

template <typename T>
static void batch_row_launch(BatchTables<T> &bt, int apply_only, hipStream_t st)
{
    batch_big_launch<T>(bt, 0, apply_only, st);
    if (!bt.rows[0].empty())
        k_row_batch<T, uint8_t, 4><<<bt.rows[0].size(), kRowBlock, row_lds_per_class<T>() * 4, st>>>(
            bt.d_views, bt.d_rows[0], apply_only);
    if (!bt.rows[1].empty())
        k_row_batch<T, uint8_t, 8><<<bt.rows[1].size(), kRowBlock, row_lds_per_class<T>() * 8, st>>>(
            bt.d_views, bt.d_rows[1], apply_only);
    if (!bt.rows[2].empty())
        k_row_batch<T, uint8_t, 16><<<bt.rows[2].size(), kRowBlock, row_lds_per_class<T>() * 16, st>>>(
            bt.d_views, bt.d_rows[2], apply_only);
}

template <typename T, int KB>
static void batch_label_plain(BatchTables<T> &bt, int b, int lt, hipStream_t st)
{
    const unsigned nb = (unsigned)bt.plain[b].size();
    const size_t lds = sizeof(T) * kRowBlock * KB;
    if (lt == 1024) k_label_batch<T, uint8_t, KB, 1024><<<nb, kRowBlock, lds, st>>>(bt.d_views, bt.d_plain[b]);
    else if (lt == 4096) k_label_batch<T, uint8_t, KB, 4096><<<nb, kRowBlock, lds, st>>>(bt.d_views, bt.d_plain[b]);
    else k_label_batch<T, uint8_t, KB, 2048><<<nb, kRowBlock, lds, st>>>(bt.d_views, bt.d_plain[b]);
}

template <typename T, int KB>
static void batch_label_bucket(BatchTables<T> &bt, int b, hipStream_t st)
{
    if (!bt.plain[b].empty()) batch_label_plain<T, KB>(bt, b, bt.lt[b], st);
    if (!bt.sorted[b].empty())
        k_label_sorted_batch<T, uint8_t, KB><<<bt.sorted[b].size(), kSortedThreads, bt.sorted_lds[b], st>>>(
            bt.d_views, bt.d_sorted[b]);
}

template <typename T>
static void batch_iteration(BatchTables<T> &bt, hipStream_t st)
{
    batch_row_launch<T>(bt, 0, st);
    batch_label_bucket<T, 4>(bt, 0, st);
    batch_label_bucket<T, 8>(bt, 1, st);
    batch_label_bucket<T, 16>(bt, 2, st);
    if (!bt.big_lab.empty()) k_label_big_batch<T><<<bt.big_lab.size(), kRowBlock, 0, st>>>(bt.d_views, bt.d_biglab);
    // each graph's finish is made by the last workgroup of its label pass (finish_if_last)
}

// Builds the device tables of a batch (graphs gs with settings prms; every graph's
// workspace must exist) and uploads the initial control blocks.
template <typename T>
static gfw_status_t batch_prepare(BatchTables<T> &bt, int32_t count, gfw_graph_s *const *gs,
                                  const gfw_params_t *const *prms, int32_t *const *labels_out, hipStream_t st,
                                  bool init_state, int32_t *max_iter_out, bool *watch_stop_out)
{
    static const bool lds_set = (set_batch_lds_limits<T, 4>(), set_batch_lds_limits<T, 8>(),
                                 set_batch_lds_limits<T, 16>(), true); // once, thread-safe
    (void)lds_set;
    bt.reset();
    std::vector<Ctl> &ctl0 = bt.ctl0;
    std::vector<const T *> &u0 = bt.u0;
    std::vector<int32_t *> &lab_out = bt.lab_out;
    ctl0.assign((size_t)count, Ctl{});
    u0.assign((size_t)count, nullptr);
    lab_out.assign((size_t)count, nullptr);
    int32_t max_iter = 0;
    bool any_u0 = false, watch_stop = false;
    for (int32_t i = 0; i < count; ++i) {
        gfw_graph_s *g = gs[i];
        const gfw_params_t *prm = prms[i];
        bt.views.push_back(make_view<T>(g));
        if (g->K > 16) {
            const int b = big_bucket_of(g->shape.kmax);
            for (int32_t t = 0; t < g->shape.nb_big; ++t) bt.big_rows[b].push_back({i, t});
            for (int32_t t = 0; t < g->shape.nb_row; ++t) {
                bt.big_lab.push_back({i, t});
                bt.all_rows.push_back({i, t});
            }
        } else {
            const int b = bucket_of(g->shape.kmax);
            for (int32_t t = 0; t < g->shape.nb_row; ++t) {
                bt.rows[b].push_back({i, t});
                bt.all_rows.push_back({i, t});
                if (g->label_path != 1) bt.plain[b].push_back({i, t});
            }
            if (g->label_path == 1) {
                for (int32_t t = 0; t < g->n_tiles; ++t) bt.sorted[b].push_back({i, t});
                bt.sorted_lds[b] = std::max(bt.sorted_lds[b], g->sorted_lds);
            }
        }
        if (init_state) {
            Ctl &c = ctl0[(size_t)i];
            std::memset(&c, 0, sizeof(c));
            c.active = prm->max_iter > 0 ? 1 : 0;
            c.max_iter = prm->max_iter;
            c.one_shot = prm->one_shot;
            c.last_eval = -1;
            c.alpha_last = std::numeric_limits<double>::quiet_NaN();
            c.gap = std::numeric_limits<double>::quiet_NaN();
            c.sp = solve_params(g, prm);
            c.hist = g->ws.hist;
            c.hist_stride = prm->max_iter + 1;
            u0[(size_t)i] = (const T *)prm->U0;
            any_u0 = any_u0 || prm->U0;
            max_iter = std::max(max_iter, prm->max_iter);
            watch_stop = watch_stop || prm->tol >= 0.0 || prm->one_shot;
        }
        lab_out[(size_t)i] = labels_out ? labels_out[i] : nullptr;
    }
    gfw_status_t s;
    if ((s = upload(bt.views, bt.dv, &bt.d_views, st)) != GFW_OK) return s;
    for (int b = 0; b < 3; ++b) {
        if ((s = upload(bt.rows[b], bt.drows[b], &bt.d_rows[b], st)) != GFW_OK) return s;
        if ((s = upload(bt.plain[b], bt.dplain[b], &bt.d_plain[b], st)) != GFW_OK) return s;
        if ((s = upload(bt.sorted[b], bt.dsorted[b], &bt.d_sorted[b], st)) != GFW_OK) return s;
    }
    if ((s = upload(bt.all_rows, bt.dall, &bt.d_all, st)) != GFW_OK) return s;
    for (int b = 0; b < kBigBuckets; ++b)
        if ((s = upload(bt.big_rows[b], bt.dbig[b], &bt.d_big[b], st)) != GFW_OK) return s;
    if ((s = upload(bt.big_lab, bt.dbiglab, &bt.d_biglab, st)) != GFW_OK) return s;
    if (labels_out && (s = upload(lab_out, bt.dlab, &bt.d_lab_out, st)) != GFW_OK) return s;
    if ((s = bt.dflag.reserve(1)) != GFW_OK) return s;
    bt.d_flag = bt.dflag.p;
    if (!bt.h_flag) GFW_HIP_TRY(hipHostMalloc((void **)&bt.h_flag, 2 * sizeof(int32_t), hipHostMallocDefault));
    if (init_state) {
        if ((s = upload(ctl0, bt.dctl0, &bt.d_ctl0, st)) != GFW_OK) return s;
        if (any_u0 && (s = upload(u0, bt.dU0, &bt.d_U0, st)) != GFW_OK) return s;
        // U_0 and P_0 = L_s U_0 for every graph
        k_set_ctl_batch<T><<<grid_for(count, 256), 256, 0, st>>>(bt.d_views, bt.d_ctl0, count);
        k_init_u_batch<T><<<bt.all_rows.size(), kRowBlock, 0, st>>>(bt.d_views, bt.d_all, bt.d_U0);
        if (!bt.rows[0].empty()) k_spmm_batch<T, 4><<<bt.rows[0].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[0]);
        if (!bt.rows[1].empty()) k_spmm_batch<T, 8><<<bt.rows[1].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[1]);
        if (!bt.rows[2].empty())
            k_spmm_batch<T, 16><<<bt.rows[2].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[2]);
        batch_big_launch<T>(bt, 1, 0, st);
        GFW_HIP_TRY(hipGetLastError());
    }
    if (max_iter_out) *max_iter_out = max_iter;
    if (watch_stop_out) *watch_stop_out = watch_stop;
    return GFW_OK;
}

// Runs up to `iters` iterations of every graph of the batch; with `watch`, returns early
// (one chunk behind) once no graph has work left.  *any_left reports whether some graph
// may still have work.
template <typename T>
static gfw_status_t batch_run(BatchTables<T> &bt, int32_t iters, bool watch, hipStream_t st, bool *any_left,
                              bool capture = false)
{
    constexpr int chunk = 8;
    const int count = (int)bt.views.size();
    const int reps = (int)cdiv(iters, chunk);
    struct Res { // released on every return path
        hipGraphExec_t exec = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        hipStream_t st = nullptr;
        ~Res()
        {
            if (exec) {
                (void)hipStreamSynchronize(st);
                (void)hipGraphExecDestroy(exec);
            }
            for (int i = 0; i < 2; ++i)
                if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    } res;
    res.st = st;
    // capture: the chunk of iterations is recorded once as a HIP graph (the batch tables do
    // not change during the call) and replayed; iterations past a graph's stop are no-ops
    hipGraphExec_t &exec = res.exec;
    if (capture && reps >= 2) {
        hipStream_t cs = nullptr;
        GFW_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int c = 0; c < chunk; ++c) batch_iteration<T>(bt, cs);
            e = hipStreamEndCapture(cs, &graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return fail(GFW_E_HIP, "capturing the batched iteration failed: %s", hipGetErrorString(e));
    }
    hipEvent_t *ev = res.ev;
    for (int i = 0; i < 2; ++i) GFW_HIP_TRY(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    bool left = true;
    for (int r = 0; r < reps; ++r) {
        const int n_it = std::min(chunk, iters - r * chunk);
        if (exec && n_it == chunk) {
            GFW_HIP_TRY(hipGraphLaunch(exec, st));
        } else {
            for (int c = 0; c < n_it; ++c) batch_iteration<T>(bt, st);
        }
        if (!watch) continue;
        k_any_active<T><<<1, 256, 0, st>>>(bt.d_views, count, bt.d_flag);
        GFW_HIP_TRY(hipMemcpyAsync(&bt.h_flag[r & 1], bt.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipEventRecord(ev[r & 1], st));
        if (r >= 1) {
            GFW_HIP_TRY(hipEventSynchronize(ev[(r - 1) & 1]));
            if (bt.h_flag[(r - 1) & 1] == 0) {
                left = false;
                break;
            }
        }
    }
    GFW_HIP_TRY(hipGetLastError());
    if (any_left) *any_left = left;
    return GFW_OK; // res waits for the replays before releasing the executable graph
}

// Commits every pending update (apply-only row pass) and clears the pending flags, so that
// U and P of every graph are current and a later iteration starts from a clean state.
template <typename T>
static void batch_commit(BatchTables<T> &bt, hipStream_t st)
{
    batch_row_launch<T>(bt, 1, st);
    k_clear_pending_batch<T><<<grid_for((int64_t)bt.views.size(), 256), 256, 0, st>>>(bt.d_views,
                                                                                       (int)bt.views.size());
}

// Labels (if asked), objective and control blocks of every graph; synchronises `st`.
template <typename T>
static gfw_status_t batch_collect(BatchTables<T> &bt, bool labels, std::vector<double> &E, std::vector<Ctl> &cs,
                                  hipStream_t st)
{
    const int count = (int)bt.views.size();
    if (labels) k_labels_batch<T><<<bt.all_rows.size(), kRowBlock, 0, st>>>(bt.d_views, bt.d_all, bt.d_lab_out);
    if (!bt.rows[0].empty()) k_energy_batch<T, 4><<<bt.rows[0].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[0]);
    if (!bt.rows[1].empty()) k_energy_batch<T, 8><<<bt.rows[1].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[1]);
    if (!bt.rows[2].empty())
        k_energy_batch<T, 16><<<bt.rows[2].size(), kSpmmThreads, 0, st>>>(bt.d_views, bt.d_rows[2]);
    batch_big_launch<T>(bt, 2, 0, st);
    gfw_status_t s;
    if ((s = bt.dE.reserve(count)) != GFW_OK || (s = bt.dctl_out.reserve(count)) != GFW_OK) return s;
    bt.d_E = bt.dE.p;
    bt.d_ctl_out = bt.dctl_out.p;
    k_collect_batch<T><<<count, kFinishThreads, 0, st>>>(bt.d_views, bt.d_E, bt.d_ctl_out);
    E.resize((size_t)count);
    cs.resize((size_t)count);
    GFW_HIP_TRY(hipMemcpyAsync(E.data(), bt.d_E, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipMemcpyAsync(cs.data(), bt.d_ctl_out, sizeof(Ctl) * count, hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    GFW_HIP_TRY(hipGetLastError());
    return GFW_OK;
}

// ---- the batch's label-pass autotuner ----------------------------------------------------
// The plain label pass of each K bucket stages its CSR entries in sub-tiles of 1,024, 2,048 or
// 4,096 entries: more entries give more gathers in flight per thread, fewer give more
// workgroups per CU (half the LDS per block).  The sub-tile changes no sum, so the choice is
// made by measurement: before a batch's first iteration, each size is launched on the batch's
// own tiles (with every graph's ticket preset so that no timed launch makes a finish), the
// fastest kept, and the choice cached per (dtype, bucket, log2 of the bucket's tile count).
// The server uses the cached choices (a server batch is mid-solve, so it is never timed).
struct TuneKey {
    int dsz, bucket, size_class;
    bool operator<(const TuneKey &o) const
    {
        return dsz != o.dsz ? dsz < o.dsz : bucket != o.bucket ? bucket < o.bucket : size_class < o.size_class;
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune_lt;

static TuneKey tune_key(int dsz, int b, size_t tiles)
{
    int c = 0;
    while (((size_t)1 << (c + 1)) <= tiles) ++c;
    return TuneKey{dsz, b, c};
}

template <typename T>
static void batch_use_tuned(BatchTables<T> &bt)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int b = 0; b < 3; ++b) {
        if (bt.plain[b].empty()) continue;
        auto it = g_tune_lt.find(tune_key((int)sizeof(T), b, bt.plain[b].size()));
        if (it != g_tune_lt.end()) bt.lt[b] = it->second;
    }
}

template <typename T, int KB>
static gfw_status_t tune_bucket(BatchTables<T> &bt, int b, hipStream_t st, int *best)
{
    static const int sizes[3] = {1024, 2048, 4096};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GFW_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GFW_E_HIP, "hipEventCreate failed");
    }
    float bestms = -1.0f;
    *best = kLabelTile;
    gfw_status_t s = GFW_OK;
    for (int v = 0; v < 3 && s == GFW_OK; ++v) {
        batch_label_plain<T, KB>(bt, b, sizes[v], st); // warm-up
        hipError_t e = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) batch_label_plain<T, KB>(bt, b, sizes[v], st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) s = fail(GFW_E_HIP, "timing the batched label pass failed: %s", hipGetErrorString(e));
        else if (bestms < 0.0f || ms < bestms) {
            bestms = ms;
            *best = sizes[v];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

// Times the plain label pass sizes of every bucket not in the cache (the batch's control
// blocks are initialised and no iteration has run), then applies the cached choices.
template <typename T>
static gfw_status_t batch_tune(BatchTables<T> &bt, hipStream_t st)
{
    bool need = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int b = 0; b < 3; ++b)
            if (!bt.plain[b].empty() && !g_tune_lt.count(tune_key((int)sizeof(T), b, bt.plain[b].size()))) need = true;
    }
    if (need) {
        const int count = (int)bt.views.size();
        k_set_tickets_batch<T><<<grid_for(count, 256), 256, 0, st>>>(bt.d_views, count, 0x80000000u);
        gfw_status_t s = GFW_OK;
        for (int b = 0; b < 3 && s == GFW_OK; ++b) {
            if (bt.plain[b].empty()) continue;
            const TuneKey key = tune_key((int)sizeof(T), b, bt.plain[b].size());
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                if (g_tune_lt.count(key)) continue;
            }
            int best = kLabelTile;
            s = b == 0 ? tune_bucket<T, 4>(bt, b, st, &best) : b == 1 ? tune_bucket<T, 8>(bt, b, st, &best)
                                                                   : tune_bucket<T, 16>(bt, b, st, &best);
            if (s == GFW_OK) {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune_lt[key] = best;
            }
        }
        k_set_tickets_batch<T><<<grid_for(count, 256), 256, 0, st>>>(bt.d_views, count, 0u);
        GFW_HIP_TRY(hipGetLastError());
        if (s != GFW_OK) return s;
    }
    batch_use_tuned<T>(bt);
    return GFW_OK;
}

template <typename T>
static gfw_status_t solve_batched_impl(gfw_context_s *cx, int32_t count, gfw_graph_s *const *gs,
                                       const gfw_params_t *const *prms, void *const *U_out,
                                       int32_t *const *labels_out, gfw_stats_t *stats, hipStream_t st)
{
    (void)cx;
    for (int32_t i = 0; i < count; ++i) {
        gfw_status_t s = ensure_workspace(gs[i], prms[i]->max_iter);
        if (s != GFW_OK) return s;
    }
    BatchTables<T> bt;
    int32_t max_iter = 0;
    bool watch = false;
    gfw_status_t s = batch_prepare<T>(bt, count, gs, prms, labels_out, st, true, &max_iter, &watch);
    if (s != GFW_OK) return s;
    if ((s = batch_tune<T>(bt, st)) != GFW_OK) return s;
    // every graph advances in the same launches until its own stop
    if ((s = batch_run<T>(bt, max_iter, watch, st, nullptr, true)) != GFW_OK) return s;
    batch_row_launch<T>(bt, 1, st); // commit the last pending updates
    if (U_out)
        for (int32_t i = 0; i < count; ++i)
            if (U_out[i])
                GFW_HIP_TRY(hipMemcpyAsync(U_out[i], gs[i]->ws.U, dsize(gs[i]->dtype) * gs[i]->n * gs[i]->K,
                                           hipMemcpyDeviceToDevice, st));
    if (stats) {
        std::vector<double> E;
        std::vector<Ctl> cs;
        if ((s = batch_collect<T>(bt, labels_out != nullptr, E, cs, st)) != GFW_OK) return s;
        bool nan = false;
        for (int32_t i = 0; i < count; ++i) {
            stats[i].iters = cs[(size_t)i].iters;
            stats[i].stop_reason = cs[(size_t)i].stop_reason;
            stats[i].gap = cs[(size_t)i].gap;
            stats[i].alpha_last = cs[(size_t)i].alpha_last;
            stats[i].objective = E[(size_t)i];
            nan = nan || cs[(size_t)i].stop_reason == GFW_STOP_NUMERIC;
        }
        if (nan) return fail(GFW_E_NUMERIC, "NaN met in at least one graph of the batch");
    } else {
        if (labels_out)
            k_labels_batch<T><<<bt.all_rows.size(), kRowBlock, 0, st>>>(bt.d_views, bt.d_all, bt.d_lab_out);
        GFW_HIP_TRY(hipStreamSynchronize(st)); // the batch tables are freed on return
    }
    GFW_HIP_TRY(hipGetLastError());
    return GFW_OK;
}

// --------------------------------------------------------------------------------------
// request server (continuous batching)
// --------------------------------------------------------------------------------------

// Device bytes a problem will hold while resident (graph + one solve), an upper bound of
// gfw_graph_footprint for the same problem.
static size_t request_footprint(const gfw_problem_t *p, int32_t max_iter, bool warm, int cus)
{
    const size_t v = dsize(p->dtype);
    const size_t n = (size_t)p->n, nnz = (size_t)p->nnz, K = (size_t)p->K;
    const size_t nb = (size_t)cdiv(p->n, kRowBlock);
    size_t graph = 4 * (n + 1) + (4 + v) * nnz + 4 * n;
    size_t tiles = 0; // label-pass partials beyond one per 256-row block (sorted tiles)
    if (p->nnz >= ((int64_t)4 << 20) && K <= 16) {
        const int64_t maxblock = max_block_entries<int64_t>(p->n, p->row_ptr);
        tiles = (size_t)sorted_tile_bound(p->n, p->nnz, maxblock, std::max(1, cus));
        // column-sorted copy (4 bytes per entry), its anchors (one per 64 entries plus one
        // partial run per tile) and two tile tables
        graph += 4 * nnz + 4 * (nnz / 64 + tiles) + 8 * (tiles + 1);
    }
    const size_t nb_parts = K > 16 ? std::max(nb, (size_t)cdiv(p->n, kBigRowsPerBlock)) : nb;
    const size_t solve = (2 * v + 8) * n * K + (K > 16 ? 4 * n + 2 * nnz : 2 * n) + n / 2 + 16 +
                         8 * ((size_t)(kRowParts + 4) * nb_parts + std::max(tiles, nb) +
                              kRowParts * std::max(tiles, K > 16 ? nb : (size_t)0) + 64) +
                         sizeof(Ctl) +
                         8 * 5 * ((size_t)max_iter + 1) + 4096;
    return graph + solve + (warm ? v * n * K : 0); // a warm start holds its U_0 until retirement
}

struct ServerRequest {
    uint64_t ticket = 0;
    gfw_problem_t prob{};
    std::vector<int64_t> rp;
    std::vector<int32_t> ci, li, lb;
    std::vector<unsigned char> vals;
    std::vector<unsigned char> u0h; // warm start: U_0 copied at submit
    void *u0d = nullptr;            // its device copy while resident
    gfw_params_t prm{};
    size_t footprint = 0;
    int state = 0;         // 0 queued or resident, 2 done (read and written under the server mutex)
    bool finished = false; // set by the worker thread only; published as state 2 under the mutex
    gfw_status_t status = GFW_OK;
    std::string error;
    gfw_graph_s *g = nullptr;
    std::vector<unsigned char> U;
    std::vector<int32_t> labels;
    gfw_stats_t stats{};
};

} // namespace gfw

struct gfw_server_s {
    gfw_context_s *ctx = nullptr;
    size_t budget = 0, used = 0;
    int32_t max_slots = 0;
    hipStream_t st = nullptr;       // iterations (worker thread)
    hipStream_t st_admit = nullptr; // graph set-up of admitted requests (admission thread)
    std::thread worker, admitter;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_admit;
    bool stop = false;
    uint64_t next_ticket = 1;
    int32_t in_setup = 0;                  // admitted, graph being built
    std::deque<gfw::ServerRequest *> queue; // submitted, not admitted
    std::deque<gfw::ServerRequest *> ready; // graph built, waiting for the next macro-step
    std::vector<gfw::ServerRequest *> resident;
    std::map<uint64_t, gfw::ServerRequest *> all;
    // device tables reused by every macro-step (grow-only): admission, iteration, retirement
    gfw::BatchTables<float> bt32[3];
    gfw::BatchTables<double> bt64[3];
    gfw::DevArr<int32_t> lab_pool; // labels of the requests retired in one macro-step
};

namespace gfw {

static constexpr int kMacroIters = 32; // iterations between admissions / retirements

static BatchTables<float> *server_tables(gfw_server_s *sv, float *) { return sv->bt32; }
static BatchTables<double> *server_tables(gfw_server_s *sv, double *) { return sv->bt64; }

template <typename T>
static gfw_status_t server_step(gfw_server_s *sv, std::vector<ServerRequest *> &fresh,
                                std::vector<ServerRequest *> &run)
{
    hipStream_t st = sv->st;
    gfw_status_t s;
    BatchTables<T> *tabs = server_tables(sv, (T *)nullptr);
    if (!fresh.empty()) { // U_0, P_0 and control blocks of the newly admitted requests
        std::vector<gfw_graph_s *> gs;
        std::vector<const gfw_params_t *> ps;
        for (auto *r : fresh) {
            gs.push_back(r->g);
            ps.push_back(&r->prm);
        }
        if ((s = batch_prepare<T>(tabs[0], (int32_t)gs.size(), gs.data(), ps.data(), nullptr, st, true, nullptr,
                                  nullptr)) != GFW_OK)
            return s;
    }
    if (run.empty()) return GFW_OK;
    std::vector<gfw_graph_s *> gs;
    std::vector<const gfw_params_t *> ps;
    std::vector<int32_t *> lab_out;
    for (auto *r : run) {
        gs.push_back(r->g);
        ps.push_back(&r->prm);
    }
    BatchTables<T> &bt = tabs[1];
    if ((s = batch_prepare<T>(bt, (int32_t)gs.size(), gs.data(), ps.data(), nullptr, st, false, nullptr, nullptr)) !=
        GFW_OK)
        return s;
    batch_use_tuned<T>(bt);
    if ((s = batch_run<T>(bt, kMacroIters, false, st, nullptr)) != GFW_OK) return s;
    batch_commit<T>(bt, st);
    // which requests are finished
    const int count = (int)gs.size();
    if ((s = bt.dctl_out.reserve(count)) != GFW_OK) return s;
    Ctl *d_c = bt.dctl_out.p;
    k_ctl_gather_batch<T><<<grid_for(count, 256), 256, 0, st>>>(bt.d_views, d_c, count);
    std::vector<Ctl> cs((size_t)count);
    GFW_HIP_TRY(hipMemcpyAsync(cs.data(), d_c, sizeof(Ctl) * count, hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    std::vector<ServerRequest *> done;
    for (int i = 0; i < count; ++i)
        if (!cs[(size_t)i].active && !cs[(size_t)i].pending) done.push_back(run[(size_t)i]);
    if (done.empty()) return GFW_OK;
    // results of the finished requests: U, labels, objective, stats
    std::vector<gfw_graph_s *> dg;
    std::vector<const gfw_params_t *> dp;
    std::vector<int32_t *> dl;
    size_t lab_total = 0;
    for (auto *r : done) lab_total += (size_t)r->g->n;
    if ((s = sv->lab_pool.reserve(lab_total)) != GFW_OK) return s;
    lab_total = 0;
    for (auto *r : done) {
        dg.push_back(r->g);
        dp.push_back(&r->prm);
        dl.push_back(sv->lab_pool.p + lab_total);
        lab_total += (size_t)r->g->n;
    }
    BatchTables<T> &bd = tabs[2];
    if ((s = batch_prepare<T>(bd, (int32_t)dg.size(), dg.data(), dp.data(), dl.data(), st, false, nullptr, nullptr)) !=
        GFW_OK)
        return s;
    std::vector<double> E;
    std::vector<Ctl> dc;
    if ((s = batch_collect<T>(bd, true, E, dc, st)) != GFW_OK) return s;
    for (size_t i = 0; i < done.size(); ++i) {
        ServerRequest *r = done[i];
        gfw_graph_s *g = r->g;
        r->U.resize(dsize(g->dtype) * (size_t)g->n * g->K);
        r->labels.resize((size_t)g->n);
        GFW_HIP_TRY(hipMemcpyAsync(r->U.data(), g->ws.U, r->U.size(), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipMemcpyAsync(r->labels.data(), dl[i], 4 * (size_t)g->n, hipMemcpyDeviceToHost, st));
        r->stats.iters = dc[i].iters;
        r->stats.stop_reason = dc[i].stop_reason;
        r->stats.gap = dc[i].gap;
        r->stats.alpha_last = dc[i].alpha_last;
        r->stats.objective = E[i];
        r->status = dc[i].stop_reason == GFW_STOP_NUMERIC ? GFW_E_NUMERIC : GFW_OK;
        if (r->status != GFW_OK) r->error = "NaN met during the iteration";
    }
    GFW_HIP_TRY(hipStreamSynchronize(st));
    for (auto *r : done) r->finished = true;
    return GFW_OK;
}

// Admission thread: takes queued requests in order while the budget and the slots allow,
// builds their graphs on its own stream (copies to the device, operator, workspace, warm
// start), and hands them to the worker.  Graph set-up thus overlaps the worker's iterations.
static void admit_loop(gfw_server_s *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
        ServerRequest *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_admit.wait(lk, [&] {
                return sv->stop ||
                       (!sv->queue.empty() &&
                        (int32_t)(sv->resident.size() + sv->ready.size()) + sv->in_setup < sv->max_slots &&
                        sv->used + sv->queue.front()->footprint <= sv->budget);
            });
            if (sv->stop) return;
            r = sv->queue.front();
            sv->queue.pop_front();
            sv->used += r->footprint;
            ++sv->in_setup;
        }
        gfw_graph_s *g = nullptr;
        gfw_status_t s = graph_create(sv->ctx, &r->prob, &g, sv->st_admit, true); // O(n) checks made at submit
        if (s == GFW_OK) s = ensure_workspace(g, r->prm.max_iter);
        if (s == GFW_OK && !r->u0h.empty()) { // warm start: U_0 goes to the device with the graph
            if (hipMalloc(&r->u0d, r->u0h.size()) != hipSuccess ||
                hipMemcpyAsync(r->u0d, r->u0h.data(), r->u0h.size(), hipMemcpyHostToDevice, sv->st_admit) !=
                    hipSuccess) {
                s = fail(GFW_E_NOMEM, "warm-start U_0 allocation");
                dfree(r->u0d);
                r->u0d = nullptr;
            } else {
                r->prm.U0 = r->u0d;
            }
        }
        if (s == GFW_OK && hipStreamSynchronize(sv->st_admit) != hipSuccess) s = fail(GFW_E_HIP, "graph set-up failed");
        std::lock_guard<std::mutex> lk(sv->mu);
        --sv->in_setup;
        if (s != GFW_OK) {
            r->status = s;
            r->error = gfw_last_error();
            if (g) free_graph(g);
            sv->used -= r->footprint;
            r->state = 2;
            sv->cv_done.notify_all();
            sv->cv_admit.notify_all();
            continue;
        }
        r->g = g;
        r->rp.clear();
        r->ci.clear();
        r->vals.clear(); // the device copy is the reference from here on
        sv->ready.push_back(r);
        sv->cv_work.notify_all();
    }
}

// Worker thread: every macro-step takes in the requests whose graphs are ready, advances all
// resident requests by kMacroIters batched iterations, and retires the finished ones.
static void server_loop(gfw_server_s *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
        std::vector<ServerRequest *> fresh;
        std::vector<ServerRequest *> run32, run64, fr32, fr64;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->ready.empty() || !sv->resident.empty(); });
            if (sv->stop) return;
            while (!sv->ready.empty()) {
                fresh.push_back(sv->ready.front());
                sv->ready.pop_front();
            }
            for (ServerRequest *r : fresh) sv->resident.push_back(r);
            for (ServerRequest *r : sv->resident) (r->g->dtype == GFW_F32 ? run32 : run64).push_back(r);
        }
        for (ServerRequest *r : fresh) (r->g->dtype == GFW_F32 ? fr32 : fr64).push_back(r);
        gfw_status_t s = GFW_OK;
        if (!run32.empty() || !fr32.empty()) s = server_step<float>(sv, fr32, run32);
        if (s == GFW_OK && (!run64.empty() || !fr64.empty())) s = server_step<double>(sv, fr64, run64);
        std::vector<ServerRequest *> retired;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (s != GFW_OK) { // a device failure ends every resident request
                for (ServerRequest *r : sv->resident) {
                    r->status = s;
                    r->error = gfw_last_error();
                    r->finished = true;
                }
            }
            std::vector<ServerRequest *> keep;
            for (ServerRequest *r : sv->resident) (r->finished ? retired : keep).push_back(r);
            sv->resident.swap(keep);
        }
        // device memory of the retired requests is released outside the lock
        for (ServerRequest *r : retired) {
            free_graph(r->g);
            r->g = nullptr;
            dfree(r->u0d);
            r->u0d = nullptr;
            r->u0h.clear();
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        for (ServerRequest *r : retired) {
            sv->used -= r->footprint;
            r->state = 2;
        }
        sv->cv_done.notify_all();
        sv->cv_admit.notify_all();
    }
}

} // namespace gfw


using namespace gfw;

extern "C" {

gfw_status_t gfw_solve_batched(gfw_context_t ctx, int32_t count, const gfw_graph_t *graphs, const gfw_params_t *prm,
                               int32_t shared_params, void *const *U_out, int32_t *const *labels_out,
                               gfw_stats_t *stats, void *stream)
{
    if (!ctx || !graphs || !prm) return fail(GFW_E_INVALID_ARG, "NULL argument");
    if (count < 0) return fail(GFW_E_INVALID_ARG, "count must be >= 0");
    if (count == 0) return GFW_OK;
    std::vector<gfw_graph_s *> gs((size_t)count);
    std::vector<const gfw_params_t *> ps((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        gs[(size_t)i] = graphs[i];
        if (!graphs[i]) return fail(GFW_E_INVALID_ARG, "graph %d is NULL", i);
        if (graphs[i]->ctx != ctx) return fail(GFW_E_INVALID_ARG, "graph %d belongs to another context", i);
        if (graphs[i]->dtype != graphs[0]->dtype) return fail(GFW_E_UNSUPPORTED, "a batch must share one dtype");
        if (graphs[i]->gauss) return fail(GFW_E_UNSUPPORTED, "graph %d is a Gaussian graph: solve it alone", i);
        ps[(size_t)i] = shared_params ? prm : prm + i;
        gfw_status_t s = check_params(ps[(size_t)i], graphs[i]->K);
        if (s != GFW_OK) return s;
        if (ps[(size_t)i]->p_refresh != 0) return fail(GFW_E_UNSUPPORTED, "p_refresh is not supported in batches");
        if (ps[(size_t)i]->incremental) return fail(GFW_E_UNSUPPORTED, "incremental solves are not batched");
    }
    std::vector<gfw_graph_s *> sorted_gs = gs;
    std::sort(sorted_gs.begin(), sorted_gs.end());
    if (std::adjacent_find(sorted_gs.begin(), sorted_gs.end()) != sorted_gs.end())
        return fail(GFW_E_INVALID_ARG, "a graph appears twice in the batch");
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    return graphs[0]->dtype == GFW_F32
               ? solve_batched_impl<float>(ctx, count, gs.data(), ps.data(), U_out, labels_out, stats, st)
               : solve_batched_impl<double>(ctx, count, gs.data(), ps.data(), U_out, labels_out, stats, st);
}


gfw_status_t gfw_server_create(gfw_context_t ctx, size_t hbm_budget_bytes, int32_t max_slots, gfw_server_t *out)
{
    if (!ctx || !out) return fail(GFW_E_INVALID_ARG, "ctx or out is NULL");
    if (max_slots < 1) return fail(GFW_E_INVALID_ARG, "max_slots must be >= 1");
    if (hbm_budget_bytes == 0) return fail(GFW_E_INVALID_ARG, "the HBM budget must be > 0");
    *out = nullptr;
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    gfw_server_s *sv = new (std::nothrow) gfw_server_s();
    if (!sv) return fail(GFW_E_NOMEM, "host allocation failed");
    sv->ctx = ctx;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    if (hipStreamCreateWithFlags(&sv->st, hipStreamNonBlocking) != hipSuccess) {
        delete sv;
        return fail(GFW_E_HIP, "stream creation failed");
    }
    if (hipStreamCreateWithFlags(&sv->st_admit, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(sv->st);
        delete sv;
        return fail(GFW_E_HIP, "stream creation failed");
    }
    sv->worker = std::thread(server_loop, sv);
    sv->admitter = std::thread(admit_loop, sv);
    *out = sv;
    return GFW_OK;
}

gfw_status_t gfw_server_submit(gfw_server_t sv, const gfw_problem_t *p, const gfw_params_t *prm, uint64_t *ticket)
{
    if (!sv || !p || !prm || !ticket) return fail(GFW_E_INVALID_ARG, "NULL argument");
    if (p->location != GFW_HOST) return fail(GFW_E_INVALID_ARG, "server requests must be host-resident");
    gfw_status_t s = check_problem_light(p); // the CSR entries are checked on the device at admission
    if (s != GFW_OK) return s;
    if ((s = check_params(prm, p->K)) != GFW_OK) return s;
    if (prm->p_refresh) return fail(GFW_E_UNSUPPORTED, "p_refresh is not supported by the server");
    if (prm->incremental) return fail(GFW_E_UNSUPPORTED, "incremental solves are not served");
    const size_t fp = request_footprint(p, prm->max_iter, prm->U0 != nullptr, sv->ctx->num_cu);
    if (fp > sv->budget) return fail(GFW_E_BUDGET, "request needs %zu bytes, budget is %zu", fp, sv->budget);
    auto *r = new (std::nothrow) ServerRequest();
    if (!r) return fail(GFW_E_NOMEM, "host allocation failed");
    const size_t v = dsize(p->dtype);
    r->rp.assign(p->row_ptr, p->row_ptr + p->n + 1);
    r->ci.assign(p->col_idx, p->col_idx + p->nnz);
    if (p->vals) r->vals.assign((const unsigned char *)p->vals, (const unsigned char *)p->vals + v * p->nnz);
    r->li.assign(p->labelled_idx, p->labelled_idx + p->n_labelled);
    r->lb.assign(p->labels, p->labels + p->n_labelled);
    r->prob = *p;
    r->prob.row_ptr = r->rp.data();
    r->prob.col_idx = r->ci.data();
    r->prob.vals = p->vals ? r->vals.data() : nullptr;
    r->prob.labelled_idx = r->li.data();
    r->prob.labels = r->lb.data();
    r->prm = *prm;
    if (prm->U0) { // a HOST array for server requests; copied like the graph
        const size_t ub = v * (size_t)p->n * (size_t)p->K;
        r->u0h.assign((const unsigned char *)prm->U0, (const unsigned char *)prm->U0 + ub);
        r->prm.U0 = nullptr; // set to the device copy at admission
    }
    r->footprint = fp;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->ticket = sv->next_ticket++;
        sv->all[r->ticket] = r;
        sv->queue.push_back(r);
    }
    sv->cv_admit.notify_all();
    *ticket = r->ticket;
    return GFW_OK;
}

gfw_status_t gfw_server_poll(gfw_server_t sv, uint64_t ticket, int blocking, void *U_out, int32_t *labels_out,
                             gfw_stats_t *stats)
{
    if (!sv) return fail(GFW_E_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return fail(GFW_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    ServerRequest *r = it->second;
    if (r->state != 2) {
        if (!blocking) return GFW_E_NOT_READY;
        sv->cv_done.wait(lk, [&] { return r->state == 2; });
    }
    sv->all.erase(it);
    lk.unlock();
    gfw_status_t s = r->status;
    if (s == GFW_OK) {
        if (U_out) std::memcpy(U_out, r->U.data(), r->U.size());
        if (labels_out) std::memcpy(labels_out, r->labels.data(), 4 * r->labels.size());
        if (stats) *stats = r->stats;
    } else {
        fail(s, "%s", r->error.c_str());
    }
    delete r;
    return s;
}

gfw_status_t gfw_server_destroy(gfw_server_t sv)
{
    if (!sv) return GFW_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_admit.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->admitter.joinable()) sv->admitter.join();
    (void)hipStreamSynchronize(sv->st);
    (void)hipStreamSynchronize(sv->st_admit);
    for (auto &kv : sv->all) {
        if (kv.second->g) free_graph(kv.second->g);
        dfree(kv.second->u0d);
        delete kv.second;
    }
    (void)hipStreamDestroy(sv->st);
    (void)hipStreamDestroy(sv->st_admit);
    delete sv;
    return GFW_OK;
}

} // extern "C"
