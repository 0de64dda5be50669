// Device kernels of the GFW hot path for gfx950 (CDNA4, wave64).
//
// One GFW iteration k (Alg. 3 of the paper) is split into three launches:
//   row    : apply the pending update of iteration k-1
//              U_k = (1-a) U_{k-1} + a S_{k-1},  P_k = (1-a) P_{k-1} + a Q_{k-1}
//            (P = L_s U is carried by linearity instead of recomputed), then form the
//            gradient G = P + (1/eps)(1 - 2U) - D_w (Uhat - U) (eq. gradgl_vv2g), the
//            GLMO vertex s_i (Section 4) and the per-row terms of g_k, E(U_k) and the
//            curvature; block partials in FP64.
//   label  : Q_k = L_s S_k, a sparse product with a one-hot right operand, i.e. a
//            per-row histogram of neighbour labels s_j weighted by the scaled edge
//            values; plus the per-row term (L_s S_k)_{i,s_i} of <S_k, L_s S_k>.
//   finish : one workgroup reduces all partials in a fixed order, forms g_k, E(U_k),
//            q_k = <D, Hess E D> and the step size (Armijo in closed form, since E is
//            quadratic: E(U) - E(U + aD) = a g - a^2 q / 2), the stop decision, and
//            the history entry.
// Control state lives in device memory so that a chunk of iterations can be captured
// once as a HIP graph and replayed without host round trips.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfw {

constexpr int kRowBlock = 256;     // threads per block of the row-wise kernels
constexpr int kFinishThreads = 1024;
constexpr int kRowParts = 8;       // per-row partial sums written by the row kernel
// partial slots of the row kernel
enum : int {
    PART_GAP = 0,   // sum_c G_ic (u_ic - S_ic)               -> g_k
    PART_UP = 1,    // <u_i, P_i>                              -> <U, L_s U>
    PART_PS = 2,    // P_{i, s_i}                              -> <S, L_s U>
    PART_DD = 3,    // ||d_i||^2                               -> ||D||^2
    PART_WDD = 4,   // omega_i ||d_i||^2
    PART_PEN = 5,   // sum_c u_ic (1 - u_ic)                   -> penalty
    PART_FID = 6,   // omega_i ||uhat_i - u_i||^2              -> fidelity
    PART_NB = 7     // 1 if row i is not binary
};

// Device-resident control block of one solve (written by the finish kernel only).
struct Ctl {
    int32_t active;      // iteration `k` is to be evaluated
    int32_t pending;     // an update with `alpha` is due before the next evaluation
    int32_t k;           // index of the iteration being evaluated
    int32_t max_iter;
    int32_t iters;       // updates committed so far
    int32_t stop_reason; // 0 max_iter, 1 tol, 2 numeric
    int32_t one_shot;
    int32_t last_eval;   // index of the last evaluated iteration (-1: none)
    double alpha;        // step of the pending update
    double alpha_last;
    double gap;          // last g_k
    double E_last;       // last E(U_k)
};

struct SolveParams {
    double inv_eps, omega0, tol, delta, gamma, lipschitz;
    int32_t ls, lmo;
};

// ---------------------------------------------------------------------------------
// wave / block reductions in a fixed order (deterministic for a fixed launch shape)
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double *out)
{
    __shared__ double red[kRowBlock / 64][N];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) red[wid][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------------
// set-up kernels (once per graph)
// ---------------------------------------------------------------------------------

// d_i = sum_j w_ij in FP64, dinv_i = d_i^{-1/2} (0 for an isolated node)
template <typename T>
__global__ void k_degrees(int64_t n, const int32_t *__restrict__ rp, const T *__restrict__ w,
                          double *__restrict__ dinv)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d = 0.0;
        if (w) {
            for (int32_t p = rp[i]; p < rp[i + 1]; ++p) d += (double)w[p];
        } else {
            d = (double)(rp[i + 1] - rp[i]);
        }
        dinv[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
}

// a_p = -d_i^{-1/2} w_ij d_j^{-1/2} (off-diagonal part of L_s = I - D^{-1/2} W D^{-1/2});
// rho_i = Gershgorin radius |1 + a_ii| + sum_{j != i} |a_ij| of row i.
template <typename T>
__global__ void k_scale_values(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const T *__restrict__ w, const double *__restrict__ dinv, T *__restrict__ a,
                               double *__restrict__ rho)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double di = dinv[i];
        double diag = 1.0, off = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int32_t j = ci[p];
            const double wv = w ? (double)w[p] : 1.0;
            const double v = -(di * wv * dinv[j]);
            a[p] = (T)v;
            if (j == i) diag += v; else off += fabs(v);
        }
        rho[i] = fabs(diag) + off;
    }
}

// Gershgorin radius of a user-supplied operator L (kind L, diagonal stored explicitly)
template <typename T>
__global__ void k_rho_plain(int64_t n, const int32_t *__restrict__ rp, const T *__restrict__ a,
                            double *__restrict__ rho)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += fabs((double)a[p]);
        rho[i] = s;
    }
}

// Structural checks of a device-resident CSR (same rules as the host validator).
// flags bit 0: graph malformed, bit 1: asymmetric, bit 2: bad weight.
template <typename T>
__global__ void k_validate_graph(int64_t n, int64_t nnz, const int64_t *__restrict__ rp64,
                                 const int32_t *__restrict__ ci, const T *__restrict__ w, int kind_L,
                                 unsigned int *flags)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = rp64[i], e = rp64[i + 1];
        if (b < 0 || e < b || e > nnz) { atomicOr(flags, 1u); continue; }
        int32_t prev = -1;
        for (int64_t p = b; p < e; ++p) {
            const int32_t j = ci[p];
            if (j < 0 || j >= n || j <= prev) { atomicOr(flags, 1u); break; }
            prev = j;
            double v = w ? (double)w[p] : 1.0;
            if (!(v == v) || isinf(v) || (!kind_L && v < 0.0)) atomicOr(flags, 4u);
            // symmetry: entry (j, i) must exist with the same value
            int64_t lo = rp64[j], hi = rp64[j + 1] - 1;
            bool found = false;
            if (lo >= 0 && hi < nnz) {
                while (lo <= hi) {
                    int64_t mid = (lo + hi) >> 1;
                    int32_t cm = ci[mid];
                    if (cm == i) { found = (w ? (double)w[mid] : 1.0) == v; break; }
                    if (cm < i) lo = mid + 1; else hi = mid - 1;
                }
            }
            if (!found) atomicOr(flags, 2u);
        }
    }
}

__global__ void k_rowptr_narrow(int64_t n, const int64_t *__restrict__ rp64, int32_t *__restrict__ rp32)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        rp32[i] = (int32_t)rp64[i];
}

// lab[i] = class of a labelled node, -1 otherwise; flags bit 3: bad label set
__global__ void k_scatter_labels(int64_t n, int64_t nl, int32_t K, const int32_t *__restrict__ idx,
                                 const int32_t *__restrict__ labels, int32_t *__restrict__ lab, unsigned int *flags)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nl; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = idx[t], c = labels[t];
        if (i < 0 || i >= n || c < 0 || c >= K) { atomicOr(flags, 8u); continue; }
        if (atomicCAS(&lab[i], -1, c) != -1) atomicOr(flags, 8u); // repeated index
    }
}

__global__ void k_fill_i32(int64_t n, int32_t *p, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------------
// per-solve kernels
// ---------------------------------------------------------------------------------

// U_0 = Uhat: labelled rows one-hot, others 1/K (Section 5.1); or a copy of U0.
template <typename T>
__global__ void k_init_u(int64_t n, int32_t K, const int32_t *__restrict__ lab, const T *__restrict__ U0,
                         T *__restrict__ U)
{
    const int64_t nK = n * K;
    const T invK = (T)(1.0 / (double)K);
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nK; t += (int64_t)gridDim.x * blockDim.x) {
        if (U0) { U[t] = U0[t]; continue; }
        const int64_t i = t / K;
        const int32_t c = (int32_t)(t - i * K);
        const int32_t y = lab[i];
        U[t] = y >= 0 ? (c == y ? (T)1 : (T)0) : invK;
    }
}

// P = c U + A U with A the stored CSR values and c = 1 (L_s) or 0 (kind L).
// LPR lanes cooperate on a row; each lane accumulates KMAX partial sums over its share of
// the row's entries, and the lanes are combined by a butterfly.  K <= KMAX.
template <typename T, int KMAX, int LPR>
__global__ void __launch_bounds__(kRowBlock) k_spmm(int64_t n, int32_t K, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                     int diag_one, const T *__restrict__ U, T *__restrict__ P)
{
    const int lane = threadIdx.x % LPR;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kRowBlock / LPR);
    for (int64_t i = blockIdx.x * (int64_t)(kRowBlock / LPR) + threadIdx.x / LPR; i < n; i += rows_per_grid) {
        double acc[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
        const int32_t b = rp[i], e = rp[i + 1];
        for (int32_t p = b + lane; p < e; p += LPR) {
            const int64_t j = ci[p];
            const double av = (double)a[p];
            const T *uj = U + j * K;
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < K) acc[c] += av * (double)uj[c];
        }
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < KMAX; ++c) acc[c] += __shfl_xor(acc[c], off, LPR);
        if (lane == 0) {
            const T *ui = U + i * K;
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c < K) P[i * K + c] = (T)(diag_one ? (double)ui[c] + acc[c] : acc[c]);
        }
    }
}

// Row kernel: pending update, gradient, GLMO, per-row partials.  One thread per row.
template <typename T, typename ST, int KMAX>
__global__ void __launch_bounds__(kRowBlock) k_row(int64_t n, int32_t K, const int32_t *__restrict__ lab,
                                                    T *__restrict__ U, T *__restrict__ P, const T *__restrict__ Q,
                                                    const ST *__restrict__ s_prev, ST *__restrict__ s_cur,
                                                    const Ctl *__restrict__ ctl, SolveParams sp,
                                                    double *__restrict__ part, int apply_only)
{
    // apply_only: commit the pending update and evaluate nothing
    const int32_t active = apply_only ? 0 : ctl->active, pending = ctl->pending;
    if (!active && !pending) return;
    const double alpha = ctl->alpha;
    double acc[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) acc[j] = 0.0;

    for (int64_t i = blockIdx.x * (int64_t)kRowBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRowBlock) {
        double u[KMAX], p[KMAX];
        T *Ui = U + i * K;
        T *Pi = P + i * K;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            u[c] = c < K ? (double)Ui[c] : 0.0;
            p[c] = c < K ? (double)Pi[c] : 0.0;
        }
        bool binary = true;
#pragma unroll
        for (int c = 0; c < KMAX; ++c)
            if (c < K && !(u[c] == 0.0 || u[c] == 1.0)) binary = false;
        if (pending) {
            const int32_t sp_i = (int32_t)s_prev[i];
            const T *Qi = Q + i * K;
            const double om = 1.0 - alpha;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                if (c < K) {
                    p[c] = (double)(T)(om * p[c] + alpha * (double)Qi[c]);
                    Pi[c] = (T)p[c];
                }
            }
            // a row whose direction d_i = e_{s_i} - u_i is zero (a binary row kept by the
            // GLMO) is left exactly as it is; every other row moves to (1-a) u + a e_s
            double at_s = 0.0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c)
                if (c == sp_i) at_s = u[c];
            if (!(binary && at_s == 1.0)) {
#pragma unroll
                for (int c = 0; c < KMAX; ++c) {
                    if (c < K) {
                        u[c] = (double)(T)(om * u[c] + (c == sp_i ? alpha : 0.0));
                        Ui[c] = (T)u[c];
                    }
                }
                binary = true;
#pragma unroll
                for (int c = 0; c < KMAX; ++c)
                    if (c < K && !(u[c] == 0.0 || u[c] == 1.0)) binary = false;
            }
        }
        if (!active) continue;

        const int32_t y = lab[i];
        const double om_i = y >= 0 ? sp.omega0 : 0.0;
        double g[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < K) {
                const double uhat = y >= 0 ? (c == y ? 1.0 : 0.0) : 0.0;
                const double fid = om_i != 0.0 ? om_i * (uhat - u[c]) : 0.0;
                g[c] = p[c] + sp.inv_eps * (1.0 - 2.0 * u[c]) - fid;
            }
        }
        int32_t s = 0;
        if (binary && sp.lmo == 0) {
            // GLMO keeps a binary row: its vertex is the position of its 1
#pragma unroll
            for (int c = KMAX - 1; c >= 0; --c)
                if (c < K && u[c] == 1.0) s = c;
        } else {
            double best = 0.0;
            int32_t bi = -1;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                if (c < K && (sp.lmo == 1 || u[c] != 0.0)) {
                    if (bi < 0 || g[c] < best) { best = g[c]; bi = c; }
                }
            }
            s = bi < 0 ? 0 : bi;
        }
        s_cur[i] = (ST)s;
        double gap = 0.0, up = 0.0, dd = 0.0, pen = 0.0, fid = 0.0, ps = 0.0;
#pragma unroll
        for (int c = 0; c < KMAX; ++c) {
            if (c < K) {
                const double d = (c == s ? 1.0 : 0.0) - u[c];
                gap -= g[c] * d;
                up += u[c] * p[c];
                dd += d * d;
                pen += u[c] * (1.0 - u[c]);
                if (c == s) ps = p[c];
                if (om_i != 0.0) {
                    const double e = (y == c ? 1.0 : 0.0) - u[c];
                    fid += e * e;
                }
            }
        }
        acc[PART_GAP] += gap;
        acc[PART_UP] += up;
        acc[PART_PS] += ps;
        acc[PART_DD] += dd;
        acc[PART_WDD] += om_i * dd;
        acc[PART_PEN] += pen;
        acc[PART_FID] += om_i * fid;
        acc[PART_NB] += binary ? 0.0 : 1.0;
    }
    if (!active) return;
    block_sum_store<kRowParts>(acc, part + (int64_t)blockIdx.x * kRowParts);
}

// Label pass: Q = L_s S for one-hot S given by s, and the per-row terms Q_{i, s_i}.
template <typename T, typename ST, int KMAX, int LPR>
__global__ void __launch_bounds__(kRowBlock) k_label(int64_t n, int32_t K, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                      int diag_one, const ST *__restrict__ s, T *__restrict__ Q,
                                                      const Ctl *__restrict__ ctl, double *__restrict__ part)
{
    if (!ctl->active) return;
    const int lane = threadIdx.x % LPR;
    double tot = 0.0;
    const int64_t rows_per_grid = (int64_t)gridDim.x * (kRowBlock / LPR);
    for (int64_t i = blockIdx.x * (int64_t)(kRowBlock / LPR) + threadIdx.x / LPR; i < n; i += rows_per_grid) {
        double acc[KMAX];
#pragma unroll
        for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
        const int32_t b = rp[i], e = rp[i + 1];
        for (int32_t p = b + lane; p < e; p += LPR) {
            const int32_t sj = (int32_t)s[ci[p]];
            const double av = (double)a[p];
#pragma unroll
            for (int c = 0; c < KMAX; ++c) acc[c] += (c == sj) ? av : 0.0;
        }
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < KMAX; ++c) acc[c] += __shfl_xor(acc[c], off, LPR);
        if (lane == 0) {
            const int32_t si = (int32_t)s[i];
            double own = 0.0;
#pragma unroll
            for (int c = 0; c < KMAX; ++c) {
                if (c < K) {
                    const double v = acc[c] + ((diag_one && c == si) ? 1.0 : 0.0);
                    Q[i * K + c] = (T)v;
                    if (c == si) own = (double)(T)v;
                }
            }
            tot += own;
        }
    }
    double v[1] = {tot};
    block_sum_store<1>(v, part + blockIdx.x);
}

// Finish: fixed-order reduction of the partials, gap, objective, curvature, step size.
__global__ void __launch_bounds__(kFinishThreads) k_finish(const double *__restrict__ row_part, int nb_row,
                                                           const double *__restrict__ lab_part, int nb_lab,
                                                           Ctl *__restrict__ ctl, SolveParams sp,
                                                           double *__restrict__ hist, int hist_stride)
{
    if (!ctl->active) {
        if (threadIdx.x == 0) ctl->pending = 0;
        return;
    }
    __shared__ double red[kFinishThreads / 64][kRowParts + 1];
    double v[kRowParts + 1];
#pragma unroll
    for (int j = 0; j <= kRowParts; ++j) v[j] = 0.0;
    for (int b = threadIdx.x; b < nb_row; b += kFinishThreads)
#pragma unroll
        for (int j = 0; j < kRowParts; ++j) v[j] += row_part[(int64_t)b * kRowParts + j];
    for (int b = threadIdx.x; b < nb_lab; b += kFinishThreads) v[kRowParts] += lab_part[b];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j <= kRowParts; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j <= kRowParts; ++j) red[wid][j] = v[j];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[kRowParts + 1];
    for (int j = 0; j <= kRowParts; ++j) {
        double s = 0.0;
        for (int w = 0; w < kFinishThreads / 64; ++w) s += red[w][j];
        t[j] = s;
    }
    const int k = ctl->k;
    ctl->last_eval = k;
    const double g = t[PART_GAP];
    const double E = 0.5 * t[PART_UP] + sp.inv_eps * t[PART_PEN] + 0.5 * t[PART_FID];
    // <D, L D> = <S, L S> - 2 <S, L U> + <U, L U> (L symmetric)
    const double dld = t[kRowParts] - 2.0 * t[PART_PS] + t[PART_UP];
    const double q = dld - 2.0 * sp.inv_eps * t[PART_DD] + t[PART_WDD];
    ctl->gap = g;
    ctl->E_last = E;
    double alpha = __builtin_nan("");
    bool step = true;
    if (!(g == g) || !(E == E)) {
        ctl->stop_reason = 2;
        step = false;
    } else if (sp.tol >= 0.0 && g <= sp.tol) {
        ctl->stop_reason = 1;
        step = false;
    }
    if (step) {
        if (ctl->one_shot) {
            alpha = 1.0;
        } else if (sp.ls == 0) {
            alpha = 1.0;
            for (int j = 0; j <= 1074; ++j) {
                const double dec = alpha * g - 0.5 * alpha * alpha * q;
                if (dec >= sp.gamma * alpha * g) break;
                alpha *= sp.delta;
            }
        } else if (sp.ls == 1) {
            alpha = q <= 0.0 ? 1.0 : fmin(1.0, g / q);
        } else {
            alpha = fmin(1.0, g / (sp.lipschitz * t[PART_DD]));
        }
    }
    if (hist) {
        hist[0 * hist_stride + k] = E;
        hist[1 * hist_stride + k] = g;
        hist[2 * hist_stride + k] = step ? q : __builtin_nan("");
        hist[3 * hist_stride + k] = alpha;
        hist[4 * hist_stride + k] = t[PART_NB];
    }
    if (step) {
        ctl->alpha = alpha;
        ctl->alpha_last = alpha;
        ctl->pending = 1;
        ctl->iters = k + 1;
        ctl->k = k + 1;
        ctl->active = (k + 1 < ctl->max_iter && !ctl->one_shot) ? 1 : 0;
        if (!ctl->active) ctl->stop_reason = 0;
    } else {
        ctl->pending = 0;
        ctl->active = 0;
        ctl->iters = k;
    }
}

// labels_i = lowest-index argmax_c U_ic; s_out = vertex indices of the last GLMO output
// (-1 when no iteration was evaluated).
template <typename T, typename ST>
__global__ void k_outputs(int64_t n, int32_t K, const T *__restrict__ U, const ST *__restrict__ s0,
                          const ST *__restrict__ s1, const Ctl *__restrict__ ctl, int32_t *__restrict__ labels,
                          int32_t *__restrict__ s_out)
{
    const int32_t le = ctl->last_eval;
    const ST *s = le < 0 ? nullptr : ((le & 1) ? s1 : s0);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (labels) {
            const T *u = U + i * K;
            int32_t at = 0;
            T best = u[0];
            for (int32_t c = 1; c < K; ++c)
                if (u[c] > best) { best = u[c]; at = c; }
            labels[i] = at;
        }
        if (s_out) s_out[i] = s ? (int32_t)s[i] : -1;
    }
}

__global__ void k_clear_pending(Ctl *ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->pending = 0;
}

// Terms of E(U) from its definition given P = L U: <u,P>, penalty, fidelity.
template <typename T>
__global__ void __launch_bounds__(kRowBlock) k_energy_rows(int64_t n, int32_t K, const int32_t *__restrict__ lab,
                                                            const T *__restrict__ U, const T *__restrict__ P,
                                                            double omega0, double *__restrict__ part)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)kRowBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRowBlock) {
        const int32_t y = lab[i];
        for (int32_t c = 0; c < K; ++c) {
            const double u = (double)U[i * K + c];
            acc[0] += u * (double)P[i * K + c];
            acc[1] += u * (1.0 - u);
            if (y >= 0) {
                const double e = (c == y ? 1.0 : 0.0) - u;
                acc[2] += omega0 * e * e;
            }
        }
    }
    block_sum_store<3>(acc, part + (int64_t)blockIdx.x * 3);
}

__global__ void k_sum_parts(const double *__restrict__ part, int nb, int width, double *__restrict__ out)
{
    __shared__ double red[kFinishThreads / 64];
    for (int j = 0; j < width; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[(int64_t)b * width + j];
        v = wave_sum(v);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
            out[j] = s;
        }
        __syncthreads();
    }
}

__global__ void k_max_reduce(const double *__restrict__ v, int64_t n, double *__restrict__ out)
{
    __shared__ double red[kFinishThreads / 64];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
        *out = s;
    }
}

} // namespace gfw
