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
constexpr int kFinishThreads = 512;
constexpr int kRowParts = 5;       // per-row partial sums written by the row kernel
// partial slots of the row kernel (per-row quantities combined in FP64 before summing)
enum : int {
    PART_GAP = 0,   // sum_c G_ic (u_ic - S_ic)                                   -> g_k
    PART_E = 1,     // 1/2 <u_i,P_i> + (1/eps) sum_c u_ic(1-u_ic) + omega_i/2 ||uhat_i-u_i||^2 -> E(U_k)
    PART_CURV = 2,  // <u_i,P_i> - 2 P_{i,s_i} - (2/eps)||d_i||^2 + omega_i ||d_i||^2
                    //   -> q_k once <S, L_s S> (label pass) is added
    PART_DD = 3,    // ||d_i||^2                                                  -> ||D||^2
    PART_NB = 4     // 1 if row i is not binary
};

struct SolveParams {
    double inv_eps, omega0, tol, delta, gamma, lipschitz;
    int32_t ls, lmo;
};

// Device-resident control block of one solve.  Written by the host before the first
// launch and afterwards by the finish kernel only; every kernel reads its parameters from
// here, so that a captured chunk of iterations carries no per-solve argument.
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
    SolveParams sp;
    double *hist;        // 5 x hist_stride history (may be null)
    int32_t hist_stride;
    int32_t pad_;
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

// Block sum of N per-thread values, stored at out[j * stride] (fixed order).
template <int N>
__device__ __forceinline__ void block_sum_store_strided(double (&v)[N], double *out, int64_t stride)
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
        out[threadIdx.x * stride] = s;
    }
}

// Row kernel: pending update, gradient, GLMO, per-row partials.
// A block owns kRowBlock consecutive rows.  Their U, P and Q rows form contiguous runs of
// rows*K elements, moved between HBM and LDS with coalesced accesses; each thread then
// works on one row out of LDS.  Partials are stored transposed: part[j * gridDim.x + b].
// Dynamic LDS: 3 * kRowBlock * K * sizeof(T).
template <typename T, typename ST, int KB>
__global__ void __launch_bounds__(kRowBlock) k_row(int64_t n, int32_t K, const int32_t *__restrict__ lab,
                                                    T *__restrict__ U, T *__restrict__ P, const T *__restrict__ Q,
                                                    ST *__restrict__ s0, ST *__restrict__ s1,
                                                    const Ctl *__restrict__ ctl, double *__restrict__ part,
                                                    int apply_only)
{
    // apply_only: commit the pending update and evaluate nothing
    const int32_t active = apply_only ? 0 : ctl->active, pending = ctl->pending;
    if (!active && !pending) return;
    // iteration k writes its vertices to s[k & 1]; the pending update is the one of the
    // last evaluated iteration
    const ST *__restrict__ s_prev = (ctl->last_eval & 1) ? s1 : s0;
    ST *__restrict__ s_cur = (ctl->k & 1) ? s1 : s0;
    const double alpha = ctl->alpha;
    const SolveParams sp = ctl->sp;
    extern __shared__ unsigned char lds_raw[];
    T *lu = reinterpret_cast<T *>(lds_raw);
    T *lp = lu + kRowBlock * K;
    T *lq = lp + kRowBlock * K;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kRowBlock;
    const int rows = (int)min((int64_t)kRowBlock, n - r0);
    const int cnt = rows * K;
    const int64_t base = r0 * K;
    // The block's run of rows*K elements starts on a 16-byte boundary (256*K*sizeof(T) is a
    // multiple of 16); full blocks move it with 16-byte vectors, the ragged last block with
    // scalars.  All loads are issued before the LDS stores.
    constexpr int VE = 16 / sizeof(T);                  // elements per 16-byte vector
    constexpr int VPT = (KB * kRowBlock / VE + kRowBlock - 1) / kRowBlock; // vectors per thread
    const bool full = rows == kRowBlock;
    if (full) {
        const int nvec = cnt / VE;
        const uint4 *gu = reinterpret_cast<const uint4 *>(U + base);
        const uint4 *gp = reinterpret_cast<const uint4 *>(P + base);
        const uint4 *gq = reinterpret_cast<const uint4 *>(Q + base);
        uint4 vu[VPT], vp[VPT], vq[VPT];
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = min(tid + m * kRowBlock, nvec - 1);
            vu[m] = gu[v];
            vp[m] = gp[v];
            vq[m] = gq[v]; // Q is only used when an update is pending (every iteration but the first)
        }
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = tid + m * kRowBlock;
            if (v < nvec) {
                reinterpret_cast<uint4 *>(lu)[v] = vu[m];
                reinterpret_cast<uint4 *>(lp)[v] = vp[m];
                reinterpret_cast<uint4 *>(lq)[v] = vq[m];
            }
        }
    } else {
        for (int q = tid; q < cnt; q += kRowBlock) {
            lu[q] = U[base + q];
            lp[q] = P[base + q];
            if (pending) lq[q] = Q[base + q];
        }
    }
    __syncthreads();

    double acc[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) acc[j] = 0.0;
    if (tid < rows) {
        const int64_t i = r0 + tid;
        T *ur = lu + tid * K;
        T *pr = lp + tid * K;
        double u[KB], p[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            u[c] = c < K ? (double)ur[c] : 0.0;
            p[c] = c < K ? (double)pr[c] : 0.0;
        }
        bool binary = true;
#pragma unroll
        for (int c = 0; c < KB; ++c)
            if (c < K && !(u[c] == 0.0 || u[c] == 1.0)) binary = false;
        if (pending) {
            const int32_t sp_i = (int32_t)s_prev[i];
            const T *qr = lq + tid * K;
            const double om = 1.0 - alpha;
#pragma unroll
            for (int c = 0; c < KB; ++c) {
                if (c < K) {
                    p[c] = (double)(T)(om * p[c] + alpha * (double)qr[c]);
                    pr[c] = (T)p[c];
                }
            }
            // a row whose direction d_i = e_{s_i} - u_i is zero (a binary row kept by the
            // GLMO) is left exactly as it is; every other row moves to (1-a) u + a e_s
            double at_s = 0.0;
#pragma unroll
            for (int c = 0; c < KB; ++c)
                if (c == sp_i) at_s = u[c];
            if (!(binary && at_s == 1.0)) {
#pragma unroll
                for (int c = 0; c < KB; ++c) {
                    if (c < K) {
                        u[c] = (double)(T)(om * u[c] + (c == sp_i ? alpha : 0.0));
                        ur[c] = (T)u[c];
                    }
                }
                binary = true;
#pragma unroll
                for (int c = 0; c < KB; ++c)
                    if (c < K && !(u[c] == 0.0 || u[c] == 1.0)) binary = false;
            }
        }
        if (active) {
            const int32_t y = lab[i];
            const double om_i = y >= 0 ? sp.omega0 : 0.0;
            double g[KB];
#pragma unroll
            for (int c = 0; c < KB; ++c) {
                if (c < K) {
                    const double uhat = (c == y) ? 1.0 : 0.0;
                    const double fid = om_i != 0.0 ? om_i * (uhat - u[c]) : 0.0;
                    g[c] = p[c] + sp.inv_eps * (1.0 - 2.0 * u[c]) - fid;
                } else {
                    g[c] = 0.0;
                }
            }
            int32_t s = 0;
            if (binary && sp.lmo == 0) {
                // the GLMO keeps a binary row: its vertex is the position of its 1
#pragma unroll
                for (int c = KB - 1; c >= 0; --c)
                    if (c < K && u[c] == 1.0) s = c;
            } else {
                double best = 0.0;
                int32_t bi = -1;
#pragma unroll
                for (int c = 0; c < KB; ++c) {
                    if (c < K && (sp.lmo == 1 || u[c] != 0.0)) {
                        if (bi < 0 || g[c] < best) {
                            best = g[c];
                            bi = c;
                        }
                    }
                }
                s = bi < 0 ? 0 : bi;
            }
            s_cur[i] = (ST)s;
            double gap = 0.0, up = 0.0, dd = 0.0, pen = 0.0, fid = 0.0, ps = 0.0;
#pragma unroll
            for (int c = 0; c < KB; ++c) {
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
            acc[PART_GAP] = gap;
            acc[PART_E] = 0.5 * up + sp.inv_eps * pen + 0.5 * (om_i * fid);
            acc[PART_CURV] = up - 2.0 * ps - 2.0 * sp.inv_eps * dd + om_i * dd;
            acc[PART_DD] = dd;
            acc[PART_NB] = binary ? 0.0 : 1.0;
        }
    }
    __syncthreads();
    if (pending) {
        if (full) {
            const int nvec = cnt / VE;
            uint4 *gu = reinterpret_cast<uint4 *>(U + base);
            uint4 *gp = reinterpret_cast<uint4 *>(P + base);
#pragma unroll
            for (int m = 0; m < VPT; ++m) {
                const int v = tid + m * kRowBlock;
                if (v < nvec) {
                    gu[v] = reinterpret_cast<const uint4 *>(lu)[v];
                    gp[v] = reinterpret_cast<const uint4 *>(lp)[v];
                }
            }
        } else {
            for (int q = tid; q < cnt; q += kRowBlock) {
                U[base + q] = lu[q];
                P[base + q] = lp[q];
            }
        }
    }
    if (!active) return;
    block_sum_store_strided<kRowParts>(acc, part + blockIdx.x, gridDim.x);
}

constexpr int kLabelTile = 2048; // CSR entries staged in LDS per step of the label pass

// Label pass: Q = L_s S for the one-hot S given by s (a per-row histogram of neighbour
// labels weighted by the stored values), and the per-row terms Q_{i, s_i}.
// A block owns kRowBlock consecutive rows, i.e. one contiguous range of CSR entries.  The
// range is streamed through LDS in tiles: all threads load column indices and values with
// coalesced accesses and gather the one-byte labels of the columns; then each thread sums
// the entries of its own row in CSR order.  Q is staged in LDS (dynamic, kRowBlock * K *
// sizeof(T)) and written back coalesced.  One partial per block.
template <typename T, typename ST, int KB>
__global__ void __launch_bounds__(kRowBlock) k_label(int64_t n, int32_t K, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const T *__restrict__ a,
                                                      int diag_one, const ST *__restrict__ s0,
                                                      const ST *__restrict__ s1, T *__restrict__ Q,
                                                      const Ctl *__restrict__ ctl, double *__restrict__ part)
{
    if (!ctl->active) return;
    const ST *__restrict__ s = (ctl->k & 1) ? s1 : s0;
    __shared__ ST ls[kLabelTile];
    __shared__ T lv[kLabelTile];
    extern __shared__ unsigned char lds_raw[];
    T *lq = reinterpret_cast<T *>(lds_raw);
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kRowBlock;
    const int rows = (int)min((int64_t)kRowBlock, n - r0);
    const bool has_row = tid < rows;
    const int64_t i = r0 + tid;
    const int32_t b = has_row ? rp[i] : 0, e = has_row ? rp[i + 1] : 0;
    const int32_t t_begin = rp[r0], t_end = rp[r0 + rows];
    T acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = (T)0;
    constexpr int PER = kLabelTile / kRowBlock;
    for (int32_t t0 = t_begin; t0 < t_end; t0 += kLabelTile) {
        const int cnt = (int)min((int32_t)kLabelTile, t_end - t0);
        // issue every load of the tile before using any of them: indices and values (clamped
        // to the last entry of the tile, so that every address is valid), then the label
        // gathers, then the LDS stores
        int32_t jj[PER];
        T vv[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int q = min(tid + m * kRowBlock, cnt - 1);
            jj[m] = __builtin_nontemporal_load(ci + t0 + q);
            vv[m] = __builtin_nontemporal_load(a + t0 + q);
        }
        ST ss[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) ss[m] = s[jj[m]];
        __syncthreads(); // the previous tile has been consumed
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int q = tid + m * kRowBlock;
            if (q < cnt) {
                ls[q] = ss[m];
                lv[q] = vv[m];
            }
        }
        __syncthreads();
        if (has_row) {
            const int32_t pb = max(b, t0), pe = min(e, t0 + cnt);
            int32_t p = pb;
            for (; p + 4 <= pe; p += 4) {
                int32_t sj[4];
                T v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    sj[u] = (int32_t)ls[p + u - t0];
                    v[u] = lv[p + u - t0];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < KB; ++c) acc[c] += (c == sj[u]) ? v[u] : (T)0;
            }
            for (; p < pe; ++p) {
                const int32_t sj = (int32_t)ls[p - t0];
                const T v = lv[p - t0];
#pragma unroll
                for (int c = 0; c < KB; ++c) acc[c] += (c == sj) ? v : (T)0;
            }
        }
    }
    double own = 0.0;
    if (has_row) {
        const int32_t si = (int32_t)s[i];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < K) {
                const T v = acc[c] + ((diag_one && c == si) ? (T)1 : (T)0);
                lq[tid * K + c] = v;
                if (c == si) own = (double)v;
            }
        }
    }
    __syncthreads();
    const int cntq = rows * K;
    const int64_t base = r0 * K;
    for (int q = tid; q < cntq; q += kRowBlock) Q[base + q] = lq[q];
    double v[1] = {own};
    block_sum_store_strided<1>(v, part + blockIdx.x, gridDim.x);
}

// Finish: fixed-order reduction of the partials, gap, objective, curvature, step size.
// row_part is [kRowParts][nb_row], lab_part is [nb_lab].
__global__ void __launch_bounds__(kFinishThreads) k_finish(const double *__restrict__ row_part, int nb_row,
                                                           const double *__restrict__ lab_part, int nb_lab,
                                                           Ctl *__restrict__ ctl)
{
    if (!ctl->active) {
        if (threadIdx.x == 0) ctl->pending = 0;
        return;
    }
    __shared__ double red[kFinishThreads / 64][kRowParts + 1];
    double v[kRowParts + 1];
#pragma unroll
    for (int j = 0; j <= kRowParts; ++j) v[j] = 0.0;
    // four block partials per thread and quantity in flight
    constexpr int CH = 4;
    for (int b0 = 0; b0 < nb_row; b0 += CH * kFinishThreads) {
        double x[kRowParts][CH];
#pragma unroll
        for (int j = 0; j < kRowParts; ++j)
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int b = b0 + threadIdx.x + c * kFinishThreads;
                x[j][c] = b < nb_row ? row_part[(int64_t)j * nb_row + b] : 0.0;
            }
#pragma unroll
        for (int j = 0; j < kRowParts; ++j)
#pragma unroll
            for (int c = 0; c < CH; ++c) v[j] += x[j][c];
    }
    for (int b0 = 0; b0 < nb_lab; b0 += 4 * kFinishThreads) {
        double x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int b = b0 + threadIdx.x + c * kFinishThreads;
            x[c] = b < nb_lab ? lab_part[b] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) v[kRowParts] += x[c];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j <= kRowParts; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j <= kRowParts; ++j) red[wid][j] = v[j];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[kRowParts + 1];
#pragma unroll
    for (int j = 0; j <= kRowParts; ++j) {
        double s = 0.0;
        for (int w = 0; w < kFinishThreads / 64; ++w) s += red[w][j];
        t[j] = s;
    }
    const SolveParams sp = ctl->sp;
    double *hist = ctl->hist;
    const int hist_stride = ctl->hist_stride;
    const int k = ctl->k;
    ctl->last_eval = k;
    const double g = t[PART_GAP];
    const double E = t[PART_E];
    // q = <D, L D> - (2/eps)||D||^2 + sum omega_i ||d_i||^2 with
    // <D, L D> = <S, L S> - 2 <S, L U> + <U, L U> (L symmetric).  ||D||^2 is exactly 0 iff
    // D = 0, and then q is exactly 0 (the assembled form would leave a rounding residue).
    const double q = t[PART_DD] == 0.0 ? 0.0 : t[kRowParts] + t[PART_CURV];
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
