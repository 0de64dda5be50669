// Incremental solves: inference for new nodes from a warm start (Section 4, closing remarks).
//
// Under the GLMO a binary row of U keeps its vertex (s_i = u_i), so its rows of U, of S and of
// the direction D = S - U stay fixed for the whole solve.  Only the m rows of U_0 that are not
// binary (the new nodes, typically) can move, and every quantity of an iteration restricts to
// them:
//   * the pending update and the gradient, GLMO and partials of a moving row need its rows of
//     U, P = L_s U and Q = L_s S only (row_one, the full iteration's row step);
//   * Q_i = (L_s S)_i for a moving row reads the vertices of all its neighbours, moving or
//     not: the vertices of binary rows are written once, at the start;
//   * g_k = sum_i <grad_i, u_i - s_i>, ||D||^2 and the count of non-binary rows vanish on
//     binary rows;
//   * the curvature q_k = <D, L D> - (2/eps)||D||^2 + sum_i omega_i ||d_i||^2 is summed in its
//     direct form sum_i d_i . (Q_i - P_i) + ... over the moving rows (d_i = 0 elsewhere);
//   * E is quadratic, so E(U_k + a D_k) = E(U_k) - a g_k + a^2 q_k / 2 exactly: E(U_0) is
//     evaluated once on the whole graph and carried from there (only when a history is asked
//     for: the step sizes need g and q alone).
// One iteration thus costs O(m K + the CSR entries of the moving rows).  P and Q are held for
// the moving rows only (m x K, P in FP64, in the first rows of the solve's P and Q); U, s0, s1
// are the solve's full arrays.

#include "gfw_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace gfw {

// Workgroups of the moving-row kernels for m moving rows (one, with no row, when m = 0: its
// finish then sees g = 0, as the full iteration does on a solve where every row is binary).
__host__ __device__ inline int act_blocks(int64_t m) { return m > 0 ? (int)((m + kRowBlock - 1) / kRowBlock) : 1; }

// Marks the moving rows of U (not binary) and gives the binary rows their vertex (the position
// of their 1) in both vertex arrays; cnt[b] = moving rows in 256-row block b.
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_act_mark(int64_t n, int32_t K, const T *__restrict__ U,
                                                               uint8_t *__restrict__ s0, uint8_t *__restrict__ s1,
                                                               uint8_t *__restrict__ moving, int32_t *__restrict__ cnt)
{
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    int mv = 0;
    if (i < n) {
        bool binary = true;
        int32_t v = 0;
        for (int32_t c = K - 1; c >= 0; --c) {
            const T u = U[i * K + c];
            if (!(u == (T)0 || u == (T)1)) binary = false;
            if (u == (T)1) v = c;
        }
        if (binary) {
            s0[i] = (uint8_t)v;
            s1[i] = (uint8_t)v;
        }
        mv = binary ? 0 : 1;
        moving[i] = (uint8_t)mv;
    }
    const int total = __syncthreads_count(mv);
    if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// Exclusive prefix sum of cnt[0..nb) into off[], and the total into *m (one workgroup of 1024
// threads: contiguous chunks per thread, the chunk sums scanned across the workgroup in ten
// doubling steps through LDS).
static __global__ void __launch_bounds__(1024) k_act_scan(int32_t nb, const int32_t *__restrict__ cnt,
                                                          int32_t *__restrict__ off, int32_t *__restrict__ m)
{
    __shared__ int32_t part[2][1024];
    const int t = threadIdx.x;
    const int32_t per = (nb + 1023) / 1024;
    const int32_t b0 = t * per, b1 = min(nb, b0 + per);
    int32_t sum = 0;
    for (int32_t b = b0; b < b1; ++b) sum += cnt[b];
    // inclusive scan of the chunk sums (ping-pong buffers)
    int cur = 0;
    part[cur][t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int32_t v = part[cur][t] + (t >= d ? part[cur][t - d] : 0);
        part[cur ^ 1][t] = v;
        cur ^= 1;
        __syncthreads();
    }
    if (t == 1023) *m = part[cur][1023];
    int32_t run = part[cur][t] - sum;
    for (int32_t b = b0; b < b1; ++b) {
        off[b] = run;
        run += cnt[b];
    }
}

// act[off[b] + rank] = i for the moving rows i of block b, in increasing order.
static __global__ void __launch_bounds__(kRowBlock) k_act_scatter(int64_t n, const uint8_t *__restrict__ moving,
                                                                  const int32_t *__restrict__ off,
                                                                  int32_t *__restrict__ act)
{
    __shared__ int32_t wave_cnt[kRowBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    const bool mv = i < n && moving[i];
    const uint64_t mask = __ballot(mv);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_cnt[wave] = __popcll(mask);
    __syncthreads();
    int32_t base = off[blockIdx.x];
    for (int w = 0; w < wave; ++w) base += wave_cnt[w];
    if (mv) act[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)i;
}

// P_a[r] = row act[r] of L_s U (FP64), kSpmmLanes lanes per row, the full SpMM's row sums;
// kActSpmmRows rows per workgroup, so that a few thousand rows still spread over the CUs.
constexpr int kActSpmmRows = 64;

template <typename T, int KB>
static __global__ void __launch_bounds__(kActSpmmRows * kSpmmLanes) k_act_spmm(GraphView<T> gv,
                                                                               const int32_t *__restrict__ act,
                                                                               int32_t m, double *__restrict__ Pa)
{
    constexpr int MC = KB / kSpmmLanes;
    const int64_t r = (int64_t)blockIdx.x * kActSpmmRows + threadIdx.x / kSpmmLanes;
    const int64_t i = r < m ? act[r] : -1;
    double acc[MC];
    spmm_row<T, KB>(gv, gv.U, i, acc);
    if (r < m) {
        const int l = threadIdx.x % kSpmmLanes;
#pragma unroll
        for (int c2 = 0; c2 < MC; ++c2) {
            const int c = l + kSpmmLanes * c2;
            if (c < gv.K) Pa[r * gv.K + c] = acc[c2];
        }
    }
}

// The row step of the moving rows (thread r: row act[r]): pending update, gradient, GLMO and
// partials by row_one on the rows in memory (U in place, P_a and Q_a compact); the partials of
// g, ||D||^2 and the non-binary count per block at row_part[j * nb + block].
template <typename T, int KB>
static __global__ void __launch_bounds__(kRowBlock) k_act_row(GraphView<T> gv, const int32_t *__restrict__ act,
                                                              int32_t m, double *__restrict__ Pa,
                                                              const T *__restrict__ Qa, int apply_only)
{
    const Ctl *__restrict__ ctl = gv.ctl;
    RowStep st;
    st.active = apply_only ? 0 : ctl->active;
    st.pending = ctl->pending;
    if (!st.active && !st.pending) return;
    st.alpha = ctl->alpha;
    st.sp = ctl->sp;
    const uint8_t *__restrict__ s_prev = (ctl->last_eval & 1) ? gv.s1 : gv.s0;
    uint8_t *__restrict__ s_cur = (ctl->k & 1) ? gv.s1 : gv.s0;
    const int32_t K = gv.K;
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double acc[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) acc[j] = 0.0;
    if (r < m) {
        const int64_t i = act[r];
        T q[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) q[c] = (st.pending && c < K) ? Qa[r * K + c] : (T)0;
        const int32_t sp_i = st.pending ? (int32_t)s_prev[i] : 0;
        int32_t s_row = 0;
        row_one<T, uint8_t, KB>(gv, st, i, gv.U + i * K, Pa + r * K, q, sp_i, s_cur, acc, s_row);
    }
    if (!st.active) return;
    block_sum_store_strided<kRowParts>(acc, gv.row_part + blockIdx.x, act_blocks(m));
}

// The label step of the moving rows (thread r: row i = act[r]): Q_a[r] = (L_s S_k)_i from the
// vertices of i's neighbours (CSR order and grouping, then the identity's term, as the full
// label passes),
// rounded to the graph's dtype; the curvature term d_i . (Q_i - P_i) - (2/eps)||d_i||^2 +
// omega_i ||d_i||^2 per block; the finish of the iteration by the last block.
template <typename T, int KB>
static __global__ void __launch_bounds__(kRowBlock) k_act_label(GraphView<T> gv, const int32_t *__restrict__ act,
                                                                int32_t m, const double *__restrict__ Pa,
                                                                T *__restrict__ Qa)
{
    Ctl *ctl = gv.ctl;
    if (!ctl->active) return label_inactive(gv, blockIdx.x);
    const uint8_t *__restrict__ s = (ctl->k & 1) ? gv.s1 : gv.s0;
    const int32_t K = gv.K;
    const SolveParams sp = ctl->sp;
    const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    double qd = 0.0;
    if (r < m) {
        const int64_t i = act[r];
        double acc[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[c] = 0.0;
        const int32_t e0 = gv.rp[i], e1 = gv.rp[i + 1];
        int32_t e = e0;
        if constexpr (sizeof(T) == 4) {
            // groups of 8 entries summed per class in FP32, as the full label passes do
            for (; e + 8 <= e1; e += 8) {
                float part[KB];
#pragma unroll
                for (int c = 0; c < KB; ++c) part[c] = 0.0f;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int32_t sj = (int32_t)s[gv.ci[e + u]];
                    const float v = (float)gv.a[e + u];
#pragma unroll
                    for (int c = 0; c < KB; ++c) part[c] += (c == sj) ? v : 0.0f;
                }
#pragma unroll
                for (int c = 0; c < KB; ++c) acc[c] += (double)part[c];
            }
        }
        for (; e < e1; ++e) {
            const int32_t sj = (int32_t)s[gv.ci[e]];
            const double v = (double)gv.a[e];
#pragma unroll
            for (int c = 0; c < KB; ++c) acc[c] += (c == sj) ? v : 0.0;
        }
        const int32_t si = (int32_t)s[i];
        const double om_i = gv.lab[i] >= 0 ? sp.omega0 : 0.0;
        double dq = 0.0, dd = 0.0;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < K) {
                const T qv = (T)(acc[c] + ((gv.diag_one && c == si) ? 1.0 : 0.0));
                Qa[r * K + c] = qv;
                const double d = (c == si ? 1.0 : 0.0) - (double)gv.U[i * K + c];
                dq += d * ((double)qv - Pa[r * K + c]);
                dd += d * d;
            }
        }
        qd = dq - 2.0 * sp.inv_eps * dd + om_i * dd;
    }
    const int nb = act_blocks(m);
    double v[1] = {qd};
    block_sum_store_strided<1, true>(v, gv.lab_part + blockIdx.x, nb);
    // finish: the last block to arrive
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned int ticket = atomicAdd(gv.ticket, 1u);
        last = ticket + 1u == (unsigned int)nb;
    }
    __syncthreads();
    if (!last) return;
    double t[kRowParts + 1];
    finish_sums(gv.row_part, nb, gv.lab_part, nb, t);
    if (threadIdx.x != 0) return;
    // E(U_k) carried; q in the direct form (so the assembled form's label term is zero)
    t[PART_E] = ctl->E_run;
    t[PART_CURV] = t[kRowParts];
    t[kRowParts] = 0.0;
    const Decision d = finish_decide(t, ctl->sp, ctl->one_shot);
    finish_commit(ctl, ctl->k, d, t[PART_NB]);
    if (d.step) ctl->E_run = d.E - d.alpha * d.g + 0.5 * d.alpha * d.alpha * d.q;
    *gv.ticket = 0u;
}

template <typename T, int KB>
static gfw_status_t incremental_impl(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                                     int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st)
{
    gfw_status_t s = ensure_workspace(g, prm->max_iter);
    if (s != GFW_OK) return s;
    Workspace &w = g->ws;
    gfw_context_s *cx = g->ctx;
    const int64_t n = g->n;
    const int32_t K = g->K;
    const int nb_all = g->shape.nb_row;
    // buffers of the set-up, kept in the workspace for later solves: flags, block counts and
    // offsets, the row list; P_a and Q_a take the first m rows of the solve's P and Q
    auto dalloc = [&](void **ptr, size_t bytes) -> gfw_status_t {
        if (*ptr) return GFW_OK;
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return fail(GFW_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        return GFW_OK;
    };
    if ((s = dalloc((void **)&w.act_moving, (size_t)n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.act_cnt, 8 * (size_t)nb_all)) != GFW_OK) return s; // counts, then offsets
    if ((s = dalloc((void **)&w.act_rows, 4 * (size_t)n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&w.act_m, sizeof(int32_t))) != GFW_OK) return s;
    uint8_t *moving = w.act_moving;
    int32_t *cnt = w.act_cnt, *off = w.act_cnt + nb_all, *act = w.act_rows, *mdev = w.act_m;
    double *Pa = w.P;
    T *Qa = (T *)w.Q;

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
    const GraphView<T> v = make_view<T>(g);
    T *U = (T *)w.U;
    k_init_u<T><<<nb_all, kRowBlock, 0, st>>>(v, (const T *)prm->U0);
    // E(U_0) on the whole graph, into the control block, when the history reports E(U_k) (the
    // step sizes use g and q only); else E_run stays 0
    if (history && (s = objective_on_device(g, prm, U, w.scratch, &w.ctl->E_run, st)) != GFW_OK) return s;
    k_act_mark<T><<<nb_all, kRowBlock, 0, st>>>(n, K, U, w.s0, w.s1, moving, cnt);
    k_act_scan<<<1, 1024, 0, st>>>(nb_all, cnt, off, mdev);
    k_act_scatter<<<nb_all, kRowBlock, 0, st>>>(n, moving, off, act);
    GFW_HIP_TRY(hipGetLastError());
    int32_t m = 0;
    GFW_HIP_TRY(hipMemcpyAsync(&m, mdev, sizeof(m), hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    const unsigned nb = (unsigned)act_blocks(m);
    hipEvent_t ev = trace_begin(cx, GFW_KERNEL_SPMM, st);
    k_act_spmm<T, KB><<<(unsigned)std::max<int64_t>(1, cdiv(m, kActSpmmRows)), kActSpmmRows * kSpmmLanes, 0, st>>>(
        v, act, m, Pa);
    trace_end(cx, GFW_KERNEL_SPMM, ev, st);
    if (!w.h_flag) GFW_HIP_TRY(hipHostMalloc((void **)&w.h_flag, 2 * sizeof(int32_t), hipHostMallocDefault));
    for (int i = 0; i < 2; ++i)
        if (!w.poll_ev[i]) GFW_HIP_TRY(hipEventCreateWithFlags(&w.poll_ev[i], hipEventDisableTiming));
    // the iterations, in chunks of 1, 1, 2, 4, 8, 16, 16, ... (new nodes settle in a few); the
    // stop flag is read back one chunk behind, so the queue holds work while the host waits
    int k0 = 0;
    for (int rep = 0; k0 < prm->max_iter; ++rep) {
        const int chunk = rep == 0 ? 1 : std::min(16, 1 << (rep - 1));
        const int k1 = std::min(prm->max_iter, k0 + chunk);
        for (int k = k0; k < k1; ++k) {
            ev = trace_begin(cx, GFW_KERNEL_ROW, st);
            k_act_row<T, KB><<<nb, kRowBlock, 0, st>>>(v, act, m, Pa, Qa, 0);
            trace_end(cx, GFW_KERNEL_ROW, ev, st);
            ev = trace_begin(cx, GFW_KERNEL_LABEL, st);
            k_act_label<T, KB><<<nb, kRowBlock, 0, st>>>(v, act, m, Pa, Qa);
            trace_end(cx, GFW_KERNEL_LABEL, ev, st);
        }
        k0 = k1;
        if (prm->tol < 0.0 && !prm->one_shot) continue;
        GFW_HIP_TRY(hipMemcpyAsync(&w.h_flag[rep & 1], &w.ctl->active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GFW_HIP_TRY(hipEventRecord(w.poll_ev[rep & 1], st));
        if (rep >= 1) {
            GFW_HIP_TRY(hipEventSynchronize(w.poll_ev[(rep - 1) & 1]));
            if (w.h_flag[(rep - 1) & 1] == 0) break;
        }
    }
    // commit the last pending update
    k_act_row<T, KB><<<nb, kRowBlock, 0, st>>>(v, act, m, Pa, Qa, 1);
    GFW_HIP_TRY(hipGetLastError());
    if ((s = trace_flush(cx, st)) != GFW_OK) return s;
    return solve_outputs(g, prm, U_out, labels_out, s_out, stats, history, st);
}

gfw_status_t solve_incremental(gfw_graph_s *g, const gfw_params_t *prm, void *U_out, int32_t *labels_out,
                               int32_t *s_out, gfw_stats_t *stats, double *history, hipStream_t st)
{
    if (g->K > 16) return fail(GFW_E_UNSUPPORTED, "incremental solves take K <= 16");
    const int kb = g->shape.kmax;
    if (g->dtype == GFW_F32) {
        if (kb == 4) return incremental_impl<float, 4>(g, prm, U_out, labels_out, s_out, stats, history, st);
        if (kb == 8) return incremental_impl<float, 8>(g, prm, U_out, labels_out, s_out, stats, history, st);
        return incremental_impl<float, 16>(g, prm, U_out, labels_out, s_out, stats, history, st);
    }
    if (kb == 4) return incremental_impl<double, 4>(g, prm, U_out, labels_out, s_out, stats, history, st);
    if (kb == 8) return incremental_impl<double, 8>(g, prm, U_out, labels_out, s_out, stats, history, st);
    return incremental_impl<double, 16>(g, prm, U_out, labels_out, s_out, stats, history, st);
}

} // namespace gfw
