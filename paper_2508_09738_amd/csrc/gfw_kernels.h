// Device kernels of the GFW hot path for gfx950 (CDNA4, wave64).
//
// One GFW iteration k (Alg. 3 of the paper) is split into three launches:
//   row    : apply the pending update of iteration k-1
//              U_k = (1-a) U_{k-1} + a S_{k-1},  P_k = (1-a) P_{k-1} + a Q_{k-1}
//            (P = L_s U is carried by linearity instead of recomputed, in FP64 whatever
//            the graph's dtype: P is a small difference of O(1) terms, and rounding it to
//            FP32 at every update lets it drift away from L_s U over a few hundred
//            iterations until a step size changes), then form the
//            gradient G = P + (1/eps)(1 - 2U) - D_w (Uhat - U) (eq. gradgl_vv2g), the
//            GLMO vertex s_i (Section 4) and the per-row terms of g_k, E(U_k) and the
//            curvature; block partials in FP64.
//   label  : Q_k = L_s S_k, a sparse product with a one-hot right operand, i.e. a
//            per-row histogram of neighbour labels s_j weighted by the scaled edge
//            values, summed in FP64 and stored once in the graph's dtype; plus the
//            per-row term (L_s S_k)_{i,s_i} of <S_k, L_s S_k>.
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

typedef unsigned v4u __attribute__((ext_vector_type(4))); // 16-byte vector moves

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
    uint32_t ticket;     // label-pass workgroups done with the iteration (finish_if_last)
    double E_run;        // incremental solves: E(U_k) carried by E_{k+1} = E_k - a g_k + a^2 q_k / 2
};

// ---------------------------------------------------------------------------------
// wave / block reductions in a fixed order (deterministic for a fixed launch shape)
//
// Wavefront reductions run on DPP lane permutations (VALU operand modifiers, no LDS
// traffic), in six steps over the 64 lanes (four rows of 16):
//   quad_perm [1,0,3,2] and [2,3,0,1]  -> every lane holds its quad's result
//   row_half_mirror, row_mirror         -> every lane holds its row's result
//   row_bcast:15 into rows 1 and 3      -> rows 1 and 3 hold rows 0-1 and 2-3
//   row_bcast:31 into rows 2 and 3      -> lane 63 holds the whole wavefront's result
// and lane 63 is read into every lane.  The callers run with every lane of the wavefront
// active (the reductions sit before block barriers or under wavefront-uniform conditions).
// ---------------------------------------------------------------------------------
constexpr int kDppQuadSwap1 = 0xb1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4e;     // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;    // lane i of a row reads lane 15 - i
constexpr int kDppRowHalfMirror = 0x141; // lane i of a half-row reads lane 7 - i
constexpr int kDppRowBcast15 = 0x142;   // a row reads lane 15 of the row before it
constexpr int kDppRowBcast31 = 0x143;   // a row reads lane 31

// src permuted by CTRL in the rows of ROW_MASK; lanes of the other rows get `old`
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i32(int src, int old)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double src, double old)
{
    const long long s = __double_as_longlong(src), o = __double_as_longlong(old);
    const int lo = dpp_i32<CTRL, ROW_MASK>((int)(s & 0xffffffffll), (int)(o & 0xffffffffll));
    const int hi = dpp_i32<CTRL, ROW_MASK>((int)(s >> 32), (int)(o >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long s = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(s & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(s >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<kDppQuadSwap1>(v, 0.0);
    v += dpp_f64<kDppQuadSwap2>(v, 0.0);
    v += dpp_f64<kDppRowHalfMirror>(v, 0.0);
    v += dpp_f64<kDppRowMirror>(v, 0.0);
    v += dpp_f64<kDppRowBcast15, 0xa>(v, 0.0);
    v += dpp_f64<kDppRowBcast31, 0xc>(v, 0.0);
    return readlane_f64(v, 63);
}

// ---------------------------------------------------------------------------------
// set-up kernels (once per graph)
// ---------------------------------------------------------------------------------

// d_i = sum_j w_ij in FP64, dinv_i = d_i^{-1/2} (0 for an isolated node)
template <typename T>
static __global__ void k_degrees(int64_t n, const int32_t *__restrict__ rp, const T *__restrict__ w,
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
static __global__ void k_scale_values(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
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
static __global__ void k_rho_plain(int64_t n, const int32_t *__restrict__ rp, const T *__restrict__ a,
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
static __global__ void k_validate_graph(int64_t n, int64_t nnz, const int64_t *__restrict__ rp64,
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

static __global__ void k_rowptr_narrow(int64_t n, const int64_t *__restrict__ rp64, int32_t *__restrict__ rp32)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        rp32[i] = (int32_t)rp64[i];
}

// lab[i] = class of a labelled node, -1 otherwise; flags bit 3: bad label set
static __global__ void k_scatter_labels(int64_t n, int64_t nl, int32_t K, const int32_t *__restrict__ idx,
                                 const int32_t *__restrict__ labels, int32_t *__restrict__ lab, unsigned int *flags)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nl; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = idx[t], c = labels[t];
        if (i < 0 || i >= n || c < 0 || c >= K) { atomicOr(flags, 8u); continue; }
        if (atomicCAS(&lab[i], -1, c) != -1) atomicOr(flags, 8u); // repeated index
    }
}

static __global__ void k_fill_i32(int64_t n, int32_t *p, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------------
// per-solve kernels
// ---------------------------------------------------------------------------------

// A store that writes through to memory (device-scope coherent): partials that the last
// workgroup of a label pass reads while the other workgroups of the launch run.
__device__ __forceinline__ void store_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block sum of N per-thread values, stored at out[j * stride] (fixed order); COH: the store
// writes through to memory.
template <int N, bool COH = false>
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
        if (COH)
            store_coherent(out + threadIdx.x * stride, s);
        else
            out[threadIdx.x * stride] = s;
    }
}

constexpr int kLabelTile = 2048;       // CSR entries staged in LDS per step of the SpMM and batched label pass
constexpr int kLabelTileSingle = 4096; // the same for the single-graph label pass (more gathers in flight)
constexpr int kSortedThreads = 1024;   // threads per tile of the column-sorted label pass
constexpr int kSortedMaxEntries = 131072; // CSR entries per tile (17-bit offsets, at most 128 KB of labels)
constexpr int kSortedOffsetBits = 17;     // low bits of a column-sorted word: the entry's CSR offset
constexpr uint32_t kSortedOffsetMask = (1u << kSortedOffsetBits) - 1u;
constexpr int32_t kSortedMaxSpan = (1 << (32 - kSortedOffsetBits)) - 1; // column - anchor in the high bits
constexpr int kSortedChunk = 64;          // column-sorted entries that share one anchor column

// Everything a per-iteration kernel needs to know about one graph and its solve state.
// The single-graph kernels take one view as an argument; the batched kernels look up the
// view of each workgroup's graph in a device array.  Both run the same device functions on
// the same tiles, so a graph's results do not depend on what else shares the launch.
template <typename T>
struct GraphView {
    int64_t n;
    int32_t K, diag_one;
    const int32_t *rp, *ci;
    const T *a;
    const int32_t *lab;
    T *U, *Q;
    double *P;        // L_s U carried by linearity, FP64 for both dtypes
    uint8_t *s0, *s1;
    uint8_t *s4;      // vertices of the current iteration, two per byte (written for the sorted pass)
    uint16_t *nv;     // per CSR entry, the last evaluated vertex of its column (large-K kernels)
    Ctl *ctl;
    double *row_part, *lab_part;
    double *row_fold; // the row partials folded per label-pass block, [kRowParts][n_fold] (else null)
    unsigned int *ticket; // label-pass workgroups that have written their partials (finish_if_last)
    int32_t n_lab_blocks; // workgroups of the graph's label pass
    int32_t n_fold;   // label-pass blocks that fold: sorted tiles, or the 256-row blocks for K > 16
    int32_t nb_row;   // 256-row tiles (row kernel, plain label pass, SpMM)
    int32_t nb_big;   // blocks of the large-K row kernel (stride of its partials)
    int32_t n_tiles;  // tiles of the column-sorted label pass (0: plain pass)
    const int32_t *tile_rows;  // first row of each tile
    const int32_t *tile_chunk; // first anchor of each tile
    const int32_t *ganch;      // anchor column of each 64-entry chunk (-1: read the CSR column)
    const uint32_t *gword;     // per column-sorted entry: (column - anchor) << 17 | CSR offset
};

// workgroup -> (graph, tile) of a batched launch
struct TileRef {
    int32_t graph, tile;
};

// ---------------------------------------------------------------------------------
// Row work (see the file header): pending update, gradient, GLMO, per-row partials.
// A group of kRowBlock threads owns a 256-row block; the block's U and P rows (and Q rows,
// when they come from memory) form contiguous runs of rows*K elements, moved between HBM
// and LDS with coalesced 16-byte accesses; each thread then works on one row out of LDS.
// The pieces below are shared by the row kernel and the persistent iteration kernel, so
// that both compute every row with the same operations.
// ---------------------------------------------------------------------------------

// LDS of one 256-row block: P (FP64), U, and optionally Q (graph dtype).
template <typename T>
struct RowLds {
    double *p;
    T *u, *q;
};

template <typename T>
__device__ __forceinline__ RowLds<T> row_lds_at(unsigned char *base, int K, bool with_q)
{
    RowLds<T> l;
    l.p = reinterpret_cast<double *>(base);
    l.u = reinterpret_cast<T *>(l.p + kRowBlock * K);
    l.q = with_q ? l.u + kRowBlock * K : nullptr;
    return l;
}

// Rows of block `blk` (kRowBlock rows from r0) and how its element run is moved.
struct RowSpan {
    int64_t r0, base;
    int rows, cnt;
    bool full;
};

__device__ __forceinline__ RowSpan row_span(int64_t n, int K, int64_t blk)
{
    RowSpan sp;
    sp.r0 = blk * kRowBlock;
    sp.rows = (int)min((int64_t)kRowBlock, n - sp.r0);
    sp.cnt = sp.rows * K;
    sp.base = sp.r0 * K;
    sp.full = sp.rows == kRowBlock;
    return sp;
}

// U, P (and Q if l.q) of the block into LDS; t is the thread's index in its 256-thread group.
// The block's runs start on 16-byte boundaries (256*K*sizeof(T) is a multiple of 16); full
// blocks move them with 16-byte vectors, the ragged last block with scalars.  All loads are
// issued before the LDS stores.
template <typename T, int KB>
__device__ __forceinline__ void row_stage_in(const GraphView<T> &gv, const RowSpan &sp, const RowLds<T> &l, int t,
                                             bool want_q)
{
    constexpr int VE = 16 / sizeof(T);                                     // elements of U or Q per vector
    constexpr int VPT = (KB * kRowBlock / VE + kRowBlock - 1) / kRowBlock; // vectors per thread
    constexpr int VPTP = (KB * kRowBlock / 2 + kRowBlock - 1) / kRowBlock; // the same for P (FP64)
    const T *__restrict__ U = gv.U;
    const double *__restrict__ P = gv.P;
    const T *__restrict__ Q = gv.Q;
    if (sp.full) {
        const int nvec = sp.cnt / VE, nvecp = sp.cnt / 2;
        const v4u *gu = reinterpret_cast<const v4u *>(U + sp.base);
        const v4u *gp = reinterpret_cast<const v4u *>(P + sp.base);
        const v4u *gq = reinterpret_cast<const v4u *>(Q + sp.base);
        v4u vu[VPT], vp[VPTP], vq[VPT];
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = min(t + m * kRowBlock, nvec - 1);
            vu[m] = __builtin_nontemporal_load(gu + v);
            if (want_q) vq[m] = __builtin_nontemporal_load(gq + v);
        }
#pragma unroll
        for (int m = 0; m < VPTP; ++m) vp[m] = __builtin_nontemporal_load(gp + min(t + m * kRowBlock, nvecp - 1));
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = t + m * kRowBlock;
            if (v < nvec) {
                reinterpret_cast<v4u *>(l.u)[v] = vu[m];
                if (want_q) reinterpret_cast<v4u *>(l.q)[v] = vq[m];
            }
        }
#pragma unroll
        for (int m = 0; m < VPTP; ++m) {
            const int v = t + m * kRowBlock;
            if (v < nvecp) reinterpret_cast<v4u *>(l.p)[v] = vp[m];
        }
    } else {
        for (int q = t; q < sp.cnt; q += kRowBlock) {
            l.u[q] = U[sp.base + q];
            l.p[q] = P[sp.base + q];
            if (want_q) l.q[q] = Q[sp.base + q];
        }
    }
}

// U and P of the block back to HBM from LDS.
template <typename T, int KB>
__device__ __forceinline__ void row_stage_out(const GraphView<T> &gv, const RowSpan &sp, const RowLds<T> &l, int t)
{
    constexpr int VE = 16 / sizeof(T);
    constexpr int VPT = (KB * kRowBlock / VE + kRowBlock - 1) / kRowBlock;
    constexpr int VPTP = (KB * kRowBlock / 2 + kRowBlock - 1) / kRowBlock;
    T *__restrict__ U = gv.U;
    double *__restrict__ P = gv.P;
    if (sp.full) {
        const int nvec = sp.cnt / VE, nvecp = sp.cnt / 2;
        v4u *gu = reinterpret_cast<v4u *>(U + sp.base);
        v4u *gp = reinterpret_cast<v4u *>(P + sp.base);
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = t + m * kRowBlock;
            if (v < nvec) __builtin_nontemporal_store(reinterpret_cast<const v4u *>(l.u)[v], gu + v);
        }
#pragma unroll
        for (int m = 0; m < VPTP; ++m) {
            const int v = t + m * kRowBlock;
            if (v < nvecp) __builtin_nontemporal_store(reinterpret_cast<const v4u *>(l.p)[v], gp + v);
        }
    } else {
        for (int q = t; q < sp.cnt; q += kRowBlock) {
            U[sp.base + q] = l.u[q];
            P[sp.base + q] = l.p[q];
        }
    }
}

// Per-iteration values every row needs (read once from the control block).
struct RowStep {
    int32_t active, pending;
    double alpha;
    SolveParams sp;
};

// One row i: the pending update U, P <- (1-a)(U, P) + a (e_s_prev, q) (q = row i of
// Q_{k-1}), then, when the iteration is evaluated, the gradient (eq. gradgl_vv2g), the GLMO
// vertex (Section 4, stored to s_cur) and the row's partials.  ur / pr: the row in LDS.
template <typename T, typename ST, int KB>
__device__ __forceinline__ void row_one(const GraphView<T> &gv, const RowStep &st, const int64_t i, T *ur, double *pr,
                                        const T (&q)[KB], const int32_t sp_i, ST *__restrict__ s_cur,
                                        double (&acc)[kRowParts], int32_t &s_row)
{
    const int32_t K = gv.K;
    const double alpha = st.alpha;
    const SolveParams &sp = st.sp;
    // u is held in the graph's dtype (its values are exactly those of U) and p in FP64
    T u[KB];
    double p[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) {
        u[c] = c < K ? ur[c] : (T)0;
        p[c] = c < K ? pr[c] : 0.0;
    }
    bool binary = true;
#pragma unroll
    for (int c = 0; c < KB; ++c)
        if (c < K && !(u[c] == (T)0 || u[c] == (T)1)) binary = false;
    if (st.pending) {
        const double om = 1.0 - alpha;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < K) {
                p[c] = om * p[c] + alpha * (double)q[c];
                pr[c] = p[c];
            }
        }
        // a row whose direction d_i = e_{s_i} - u_i is zero (a binary row kept by the
        // GLMO) is left exactly as it is; every other row moves to (1-a) u + a e_s
        T at_s = (T)0;
#pragma unroll
        for (int c = 0; c < KB; ++c)
            if (c == sp_i) at_s = u[c];
        if (!(binary && at_s == (T)1)) {
#pragma unroll
            for (int c = 0; c < KB; ++c) {
                if (c < K) {
                    u[c] = (T)(om * (double)u[c] + (c == sp_i ? alpha : 0.0));
                    ur[c] = u[c];
                }
            }
            binary = true;
#pragma unroll
            for (int c = 0; c < KB; ++c)
                if (c < K && !(u[c] == (T)0 || u[c] == (T)1)) binary = false;
        }
    }
    if (!st.active) return;
    const int32_t y = gv.lab[i];
    const double om_i = y >= 0 ? sp.omega0 : 0.0;
    // gradient entry of class c (eq. gradgl_vv2g), formed where it is used
    auto grad = [&](const int c) -> double {
        const double uc = (double)u[c];
        const double uhat = (c == y) ? 1.0 : 0.0;
        const double fid = om_i != 0.0 ? om_i * (uhat - uc) : 0.0;
        return p[c] + sp.inv_eps * (1.0 - 2.0 * uc) - fid;
    };
    int32_t s = 0;
    if (binary && sp.lmo == 0) {
        // the GLMO keeps a binary row: its vertex is the position of its 1
#pragma unroll
        for (int c = KB - 1; c >= 0; --c)
            if (c < K && u[c] == (T)1) s = c;
    } else {
        double best = 0.0;
        int32_t bi = -1;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < K && (sp.lmo == 1 || u[c] != (T)0)) {
                const double gc = grad(c);
                if (bi < 0 || gc < best) {
                    best = gc;
                    bi = c;
                }
            }
        }
        s = bi < 0 ? 0 : bi;
    }
    s_cur[i] = (ST)s;
    s_row = s;
    double gap = 0.0, up = 0.0, dd = 0.0, pen = 0.0, fid = 0.0, ps = 0.0;
#pragma unroll
    for (int c = 0; c < KB; ++c) {
        if (c < K) {
            const double uc = (double)u[c];
            const double d = (c == s ? 1.0 : 0.0) - uc;
            gap -= grad(c) * d;
            up += uc * p[c];
            dd += d * d;
            pen += uc * (1.0 - uc);
            if (c == s) ps = p[c];
            if (om_i != 0.0) {
                const double e = (y == c ? 1.0 : 0.0) - uc;
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

// Vertices of rows 2m, 2m + 1 packed into byte m of s4 (low nibble = even row) for the
// column-sorted label pass; r0 is a multiple of 256, so row pairs are lane pairs.
__device__ __forceinline__ void pack_s4(uint8_t *s4, int64_t r0, int rows, int t, int32_t s_row)
{
    const int32_t s_next = __shfl_down(s_row, 1);
    if (t < rows && !(t & 1)) s4[(r0 + t) >> 1] = (uint8_t)(s_row | ((t + 1 < rows ? s_next : 0) << 4));
}

// Row kernel body: block `tile` of 256 rows, one thread per row.  Partials are stored
// transposed: row_part[j * nb_row + tile].  Dynamic LDS: kRowBlock * K * (2 sizeof(T) + 8).
template <typename T, typename ST, int KB>
__device__ __forceinline__ void row_body(const GraphView<T> &gv, const int tile, const int apply_only)
{
    const Ctl *__restrict__ ctl = gv.ctl;
    RowStep st;
    st.active = apply_only ? 0 : ctl->active;
    st.pending = ctl->pending;
    if (!st.active && !st.pending) return;
    st.alpha = ctl->alpha;
    st.sp = ctl->sp;
    // iteration k writes its vertices to s[k & 1]; the pending update is the one of the
    // last evaluated iteration
    const ST *__restrict__ s_prev = reinterpret_cast<const ST *>((ctl->last_eval & 1) ? gv.s1 : gv.s0);
    ST *__restrict__ s_cur = reinterpret_cast<ST *>((ctl->k & 1) ? gv.s1 : gv.s0);
    extern __shared__ unsigned char lds_raw[];
    const RowLds<T> l = row_lds_at<T>(lds_raw, gv.K, true);
    const int tid = threadIdx.x;
    const RowSpan sp = row_span(gv.n, gv.K, tile);
    row_stage_in<T, KB>(gv, sp, l, tid, st.pending != 0); // Q is used when an update is pending
    __syncthreads();
    double acc[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) acc[j] = 0.0;
    int32_t s_row = 0;
    if (tid < sp.rows) {
        const int64_t i = sp.r0 + tid;
        T q[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) q[c] = (st.pending && c < gv.K) ? l.q[tid * gv.K + c] : (T)0;
        const int32_t sp_i = st.pending ? (int32_t)s_prev[i] : 0;
        row_one<T, ST, KB>(gv, st, i, l.u + tid * gv.K, l.p + tid * gv.K, q, sp_i, s_cur, acc, s_row);
    }
    if (KB <= 16 && gv.n_tiles > 0 && st.active) pack_s4(gv.s4, sp.r0, sp.rows, tid, s_row);
    __syncthreads();
    if (st.pending) row_stage_out<T, KB>(gv, sp, l, tid);
    if (!st.active) return;
    block_sum_store_strided<kRowParts>(acc, gv.row_part + tile, gv.nb_row);
}

// Label pass body (plain): Q = L_s S for the one-hot S given by s (a per-row histogram of
// neighbour labels weighted by the stored values), and the per-row terms Q_{i, s_i}.
// A block owns tile `tile` (kRowBlock consecutive rows, one contiguous range of CSR
// entries), streamed through LDS in sub-tiles: all threads load column indices and values
// with coalesced accesses and gather the one-byte labels of the columns; then each thread
// sums the entries of its own row in CSR order.  Q is staged in LDS (dynamic, kRowBlock *
// K * sizeof(T)) and written back coalesced.  One partial per tile: lab_part[tile].
// LT entries per sub-tile: the single-graph launch stages 4,096 (16 gathers in flight per
// thread), the batched launch 2,048 (half the LDS, so more blocks of a mixed batch share a
// CU); the sub-tiles do not change any sum.
template <typename T, typename ST, int KB, int LT>
__device__ __forceinline__ void label_body(const GraphView<T> &gv, const int tile)
{
    const int64_t n = gv.n;
    const int32_t K = gv.K;
    const int32_t *__restrict__ rp = gv.rp;
    const int32_t *__restrict__ ci = gv.ci;
    const T *__restrict__ a = gv.a;
    const int diag_one = gv.diag_one;
    const ST *__restrict__ s0 = gv.s0;
    const ST *__restrict__ s1 = gv.s1;
    T *__restrict__ Q = gv.Q;
    const Ctl *__restrict__ ctl = gv.ctl;
    double *__restrict__ part = gv.lab_part;
    if (!ctl->active) return label_inactive(gv, tile);
    const ST *__restrict__ s = (ctl->k & 1) ? s1 : s0;
    __shared__ ST ls[LT];
    __shared__ T lv[LT];
    extern __shared__ unsigned char lds_raw[];
    T *lq = reinterpret_cast<T *>(lds_raw);
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)tile * kRowBlock;
    const int rows = (int)min((int64_t)kRowBlock, n - r0);
    const bool has_row = tid < rows;
    const int64_t i = r0 + tid;
    const int32_t b = has_row ? rp[i] : 0, e = has_row ? rp[i + 1] : 0;
    const int32_t t_begin = rp[r0], t_end = rp[r0 + rows];
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    // FP32 values: the row's entries in groups of 8 from its first, each group summed per class
    // in FP32 and added in FP64, the last (e - b) mod 8 entries added one by one in FP64 (the
    // column-sorted pass's order: both passes give the same Q bit for bit).  A group may span
    // two sub-tiles, so its partial sum lives across them.
    float grp[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) grp[c] = 0.0f;
    const int32_t full_end = b + ((e - b) & ~7);
    constexpr int PER = LT / kRowBlock;
    for (int32_t t0 = t_begin; t0 < t_end; t0 += LT) {
        const int cnt = (int)min((int32_t)LT, t_end - t0);
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
        if (has_row && sizeof(T) == 4) {
            const int32_t pb = max(b, t0), pe = min(e, t0 + cnt);
            int32_t p = pb;
            while (p < pe) {
                if (((p - b) & 7) == 0 && p + 8 <= pe && p + 8 <= full_end) {
                    int32_t sj[8];
                    float v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        sj[u] = (int32_t)ls[p + u - t0];
                        v[u] = (float)lv[p + u - t0];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int c = 0; c < KB; ++c) grp[c] += (c == sj[u]) ? v[u] : 0.0f;
#pragma unroll
                    for (int c = 0; c < KB; ++c) {
                        acc[c] += (double)grp[c];
                        grp[c] = 0.0f;
                    }
                    p += 8;
                } else if (p < full_end) {
                    const int32_t sj = (int32_t)ls[p - t0];
                    const float v = (float)lv[p - t0];
#pragma unroll
                    for (int c = 0; c < KB; ++c) grp[c] += (c == sj) ? v : 0.0f;
                    if (((p - b) & 7) == 7)
#pragma unroll
                        for (int c = 0; c < KB; ++c) {
                            acc[c] += (double)grp[c];
                            grp[c] = 0.0f;
                        }
                    ++p;
                } else {
                    const int32_t sj = (int32_t)ls[p - t0];
                    const double v = (double)lv[p - t0];
#pragma unroll
                    for (int c = 0; c < KB; ++c) acc[c] += (c == sj) ? v : 0.0;
                    ++p;
                }
            }
        } else if (has_row) {
            const int32_t pb = max(b, t0), pe = min(e, t0 + cnt);
            int32_t p = pb;
            for (; p + 4 <= pe; p += 4) {
                int32_t sj[4];
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    sj[u] = (int32_t)ls[p + u - t0];
                    v[u] = (double)lv[p + u - t0];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < KB; ++c) acc[c] += (c == sj[u]) ? v[u] : 0.0;
            }
            for (; p < pe; ++p) {
                const int32_t sj = (int32_t)ls[p - t0];
                const double v = (double)lv[p - t0];
#pragma unroll
                for (int c = 0; c < KB; ++c) acc[c] += (c == sj) ? v : 0.0;
            }
        }
    }
    double own = 0.0;
    if (has_row) {
        const int32_t si = (int32_t)s[i];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < K) {
                const T v = (T)(acc[c] + ((diag_one && c == si) ? 1.0 : 0.0));
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
    block_sum_store_strided<1, true>(v, part + tile, gv.nb_row);
    finish_if_last(gv, gv.row_part, gv.nb_row, gv.lab_part, gv.nb_row);
}

// Column-sorted label pass body: the same Q = L_s S and per-tile partial as label_body, for
// graphs whose neighbour labels are scattered (random node order).  A workgroup owns one
// tile of consecutive rows holding at most kSortedMaxEntries CSR entries.  The tile's
// entries are stored twice: in CSR order (values) and sorted by column.  A column-sorted
// entry is one 32-bit word: its offset inside the tile's CSR range (low 17 bits) and its
// column minus the anchor of its chunk (high 15 bits), where the anchor is the first column
// of each aligned run of kSortedChunk sorted entries.  A chunk whose columns span more than
// kSortedMaxSpan has anchor -1; its entries take their column from the CSR column array at
// their offset instead.
//  1. gather: consecutive threads take consecutive column-sorted entries, so the labels they
//     load lie close together and share cache lines; a wavefront's 64 entries form one
//     chunk, whose anchor is a scalar load; labels are read from the packed two-per-byte
//     copy (half the lines of the byte array) and each is written into an LDS array at the
//     entry's CSR offset.
//  2. rows: each thread sums the histogram of one row at a time in CSR order, values read
//     from global memory (a row's values are contiguous) and labels from LDS (the same
//     order, hence the same result, as label_body), and writes the row of Q directly.
// Dynamic LDS: one byte per entry of the graph's largest tile (at most kSortedMaxEntries).
// One tile runs per CU at a time, and the tiles are sized so that their count fills whole
// rounds of the CUs.  On a randomly ordered graph both phases wait on memory: the gathers of
// phase 1 cost in proportion to the distinct cache lines each gather instruction touches
// (which the column order and the packed labels reduce), and the row walks of phase 2 wait
// on their values; both keep several loads in flight per thread (16 sorted entries per
// gather batch, row values in batches of 8).
// The pieces of the column-sorted pass, shared with the persistent iteration kernel.
// Step 0: the row kernel's partials of a fixed slice of 256-row blocks, folded into this
// tile's entry of row_fold, so that the finish reads n_tiles partials instead of nb_row: the
// first wavefront loads them (lane order) and sorted_finish sums them (a wavefront tree).
template <typename T>
__device__ __forceinline__ void sorted_fold_load(const GraphView<T> &gv, const int tile, double (&fold)[kRowParts])
{
    const int nbr = gv.nb_row, ntl = gv.n_tiles;
    const int fb0 = (int)((int64_t)tile * nbr / ntl), fb1 = (int)((int64_t)(tile + 1) * nbr / ntl);
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) fold[j] = 0.0;
    if (threadIdx.x < 64)
        for (int b = fb0 + (int)threadIdx.x; b < fb1; b += 64)
#pragma unroll
            for (int j = 0; j < kRowParts; ++j) fold[j] += gv.row_part[(int64_t)j * nbr + b];
}

// Step 1: the labels of the tile's entries gathered in column order and scattered to their
// CSR offsets in LDS (llab).  G sorted entries per thread per batch.
template <typename T, int G>
__device__ __forceinline__ void sorted_gather(const GraphView<T> &gv, const int tile, uint8_t *llab)
{
    static_assert(kSortedThreads % kSortedChunk == 0 && kSortedChunk == 64, "a wavefront reads one chunk");
    const int tid = threadIdx.x;
    const int32_t r0 = gv.tile_rows[tile], r1 = gv.tile_rows[tile + 1];
    const int32_t e0 = gv.rp[r0], e1 = gv.rp[r1];
    const int E = e1 - e0;
    const uint32_t *__restrict__ gword = gv.gword;
    const int32_t *__restrict__ ci = gv.ci;
    const uint8_t *__restrict__ s4 = gv.s4;
    const int32_t *__restrict__ anch = gv.ganch + gv.tile_chunk[tile];
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63); // first entry of the wavefront's chunk
    for (int b = 0; b < E; b += G * kSortedThreads) {
        uint32_t ww[G];
        int32_t an[G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            // lanes past the end repeat the last entry, which lies in the wavefront's chunk
            const int e = min(b + tid + m * kSortedThreads, E - 1);
            ww[m] = __builtin_nontemporal_load(gword + e0 + e);
            an[m] = anch[min(b + wbase + m * kSortedThreads, E - 1) / kSortedChunk];
        }
        int32_t cc[G];
#pragma unroll
        for (int m = 0; m < G; ++m)
            cc[m] = an[m] >= 0 ? an[m] + (int32_t)(ww[m] >> kSortedOffsetBits)
                               : ci[e0 + (int32_t)(ww[m] & kSortedOffsetMask)];
        uint32_t ss[G];
#pragma unroll
        for (int m = 0; m < G; ++m) ss[m] = (uint32_t)s4[cc[m] >> 1];
#pragma unroll
        for (int m = 0; m < G; ++m)
            if (b + tid + m * kSortedThreads < E)
                llab[ww[m] & kSortedOffsetMask] = (uint8_t)((ss[m] >> ((cc[m] & 1) << 2)) & 15u);
    }
}

// Step 2 for one row (local index r in the tile): the histogram of its neighbours' labels
// weighted by the stored values, in CSR order, FP64 sums; q receives row r of Q = L_s S
// rounded to the graph's dtype (the identity's 1 added to the row's own vertex si).  The
// row's values are loaded in batches of 8, then 4, then singly (a row has about 24 entries
// on the large SBM: three batches), each batch's loads in flight together.
template <typename T, int KB>
__device__ __forceinline__ void sorted_row(const GraphView<T> &gv, const int32_t e0, const int rb, const int re,
                                           const uint8_t *llab, const int32_t si, T (&q)[KB])
{
    const T *__restrict__ a = gv.a;
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    int p = rb;
    for (; p + 8 <= re; p += 8) {
        T v[8];
        int32_t sj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v[u] = a[e0 + p + u];
            sj[u] = (int32_t)llab[p + u];
        }
        if constexpr (sizeof(T) == 4) {
            // FP32 values: each group of 8 entries summed per class in FP32, the group sums added
            // in FP64 (the plain pass sums in the same groups)
            float part[KB];
#pragma unroll
            for (int c = 0; c < KB; ++c) part[c] = 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < KB; ++c) part[c] += (c == sj[u]) ? (float)v[u] : 0.0f;
#pragma unroll
            for (int c = 0; c < KB; ++c) acc[c] += (double)part[c];
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < KB; ++c) acc[c] += (c == sj[u]) ? (double)v[u] : 0.0;
        }
    }
    for (; p + 4 <= re; p += 4) {
        T v[4];
        int32_t sj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = a[e0 + p + u];
            sj[u] = (int32_t)llab[p + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < KB; ++c) acc[c] += (c == sj[u]) ? (double)v[u] : 0.0;
    }
    for (; p < re; ++p) {
        const double v = (double)a[e0 + p];
        const int32_t sj = (int32_t)llab[p];
#pragma unroll
        for (int c = 0; c < KB; ++c) acc[c] += (c == sj) ? v : 0.0;
    }
#pragma unroll
    for (int c = 0; c < KB; ++c) q[c] = (T)(acc[c] + ((gv.diag_one && c == si) ? 1.0 : 0.0));
}

// Step 3: the tile's partial of <S, L_s S> (each thread's sum over its rows, wavefront trees,
// then the 16 wavefronts in order) to lab_part[tile], and the folded row partials to row_fold.
template <typename T>
__device__ __forceinline__ void sorted_finish(const GraphView<T> &gv, const int tile, double own,
                                              double (&fold)[kRowParts])
{
    __shared__ double red[kSortedThreads / 64];
    const int tid = threadIdx.x;
    own = wave_sum(own);
    if ((tid & 63) == 0) red[tid >> 6] = own;
    if (tid < 64) { // the whole first wavefront
#pragma unroll
        for (int j = 0; j < kRowParts; ++j) fold[j] = wave_sum(fold[j]);
        if (tid == 0)
#pragma unroll
            for (int j = 0; j < kRowParts; ++j) store_coherent(gv.row_fold + (int64_t)j * gv.n_tiles + tile, fold[j]);
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kSortedThreads / 64; ++w) t += red[w];
        store_coherent(gv.lab_part + tile, t);
    }
}

// Column-sorted label pass body: steps 0-3 for tile `tile`; Q rows go to memory.
template <typename T, typename ST, int KB>
__device__ __forceinline__ void label_sorted_body(const GraphView<T> &gv, const int tile)
{
    static_assert(KB <= 16, "packed labels hold K <= 16");
    const Ctl *__restrict__ ctl = gv.ctl;
    if (!ctl->active) return label_inactive(gv, tile);
    const ST *__restrict__ s = (ctl->k & 1) ? gv.s1 : gv.s0;
    extern __shared__ unsigned char lds_raw[];
    uint8_t *llab = lds_raw; // [entries of the tile]
    const int tid = threadIdx.x;
    const int32_t r0 = gv.tile_rows[tile], r1 = gv.tile_rows[tile + 1];
    const int32_t e0 = gv.rp[r0];
    const int rows = r1 - r0;
    double fold[kRowParts];
    sorted_fold_load<T>(gv, tile, fold);
    constexpr int G = 16; // sorted entries per thread per batch (n = 2 M SBM: 4, 8, 16 took 143, 128, 124 us)
    sorted_gather<T, G>(gv, tile, llab);
    __syncthreads();
    // one row at a time per thread: rows r0 + tid + j * kSortedThreads
    double own = 0.0;
    for (int r = tid; r < rows; r += kSortedThreads) {
        const int rb = gv.rp[r0 + r] - e0, re = gv.rp[r0 + r + 1] - e0;
        const int32_t si = (int32_t)s[r0 + r];
        T q[KB];
        sorted_row<T, KB>(gv, e0, rb, re, llab, si, q);
        T *__restrict__ qr = gv.Q + (int64_t)(r0 + r) * gv.K;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < gv.K) {
                qr[c] = q[c];
                if (c == si) own += (double)q[c];
            }
        }
    }
    sorted_finish<T>(gv, tile, own, fold);
    finish_if_last(gv, gv.row_fold, gv.n_tiles, gv.lab_part, gv.n_tiles);
}

// Finish: fixed-order reduction of the partials, gap, objective, curvature, step size,
// stop test and history entry of one graph.  row_part is [kRowParts][nb_row], lab_part is
// [nb_lab].  finish_sums reduces them in the order of kFinishThreads threads (thread v sums
// partials v, v + 512, ... four at a time; wavefront trees; the eight wavefronts in order),
// whatever the size of the workgroup running it: a workgroup of 256 threads takes the 512
// sums two per thread, one of 1024 threads leaves half its threads idle.  Every thread must
// call it (it holds a barrier); the totals land in t on thread 0.
__device__ __forceinline__ void finish_sums(const double *row_part, int nb_row, const double *lab_part, int nb_lab,
                                            double (&t)[kRowParts + 1])
{
    __shared__ double red[kFinishThreads / 64][kRowParts + 1];
    const int lane = threadIdx.x & 63;
    for (int vt = threadIdx.x; vt < kFinishThreads; vt += blockDim.x) { // uniform per wavefront
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
                    const int b = b0 + vt + c * kFinishThreads;
                    x[j][c] = b < nb_row ? load_coherent(row_part + (int64_t)j * nb_row + b) : 0.0;
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
                const int b = b0 + vt + c * kFinishThreads;
                x[c] = b < nb_lab ? load_coherent(lab_part + b) : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) v[kRowParts] += x[c];
        }
#pragma unroll
        for (int j = 0; j <= kRowParts; ++j) v[j] = wave_sum(v[j]);
        if (lane == 0)
#pragma unroll
            for (int j = 0; j <= kRowParts; ++j) red[vt >> 6][j] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j <= kRowParts; ++j) {
            double x = 0.0;
            for (int w = 0; w < kFinishThreads / 64; ++w) x += red[w][j];
            t[j] = x;
        }
}

// The decision of iteration k from the totals: g_k, E(U_k), q_k, the step size and whether
// a step is taken (no step: g_k <= tol, or a NaN).
struct Decision {
    double g, E, q, alpha;
    bool step;
    int32_t stop_reason; // when no step: 1 tol, 2 numeric
};

__device__ __forceinline__ Decision finish_decide(const double (&t)[kRowParts + 1], const SolveParams &sp,
                                                  int32_t one_shot)
{
    Decision d;
    d.g = t[PART_GAP];
    d.E = t[PART_E];
    // q = <D, L D> - (2/eps)||D||^2 + sum omega_i ||d_i||^2 with
    // <D, L D> = <S, L S> - 2 <S, L U> + <U, L U> (L symmetric).  ||D||^2 is exactly 0 iff
    // D = 0, and then q is exactly 0 (the assembled form would leave a rounding residue).
    d.q = t[PART_DD] == 0.0 ? 0.0 : t[kRowParts] + t[PART_CURV];
    d.alpha = __builtin_nan("");
    d.step = true;
    d.stop_reason = 0;
    if (!(d.g == d.g) || !(d.E == d.E)) {
        d.stop_reason = 2;
        d.step = false;
    } else if (sp.tol >= 0.0 && d.g <= sp.tol) {
        d.stop_reason = 1;
        d.step = false;
    }
    if (d.step) {
        if (one_shot) {
            d.alpha = 1.0;
        } else if (sp.ls == 0) {
            double alpha = 1.0;
            for (int j = 0; j <= 1074; ++j) {
                const double dec = alpha * d.g - 0.5 * alpha * alpha * d.q;
                if (dec >= sp.gamma * alpha * d.g) break;
                alpha *= sp.delta;
            }
            d.alpha = alpha;
        } else if (sp.ls == 1) {
            d.alpha = d.q <= 0.0 ? 1.0 : fmin(1.0, d.g / d.q);
        } else {
            d.alpha = fmin(1.0, d.g / (sp.lipschitz * t[PART_DD]));
        }
    }
    return d;
}

// The control block and history after the decision of iteration k (one thread).
__device__ __forceinline__ void finish_commit(Ctl *ctl, const int k, const Decision &d, const double nonbinary)
{
    double *hist = ctl->hist;
    const int hist_stride = ctl->hist_stride;
    ctl->last_eval = k;
    ctl->gap = d.g;
    ctl->E_last = d.E;
    if (!d.step) ctl->stop_reason = d.stop_reason;
    if (hist) {
        hist[0 * hist_stride + k] = d.E;
        hist[1 * hist_stride + k] = d.g;
        hist[2 * hist_stride + k] = d.step ? d.q : __builtin_nan("");
        hist[3 * hist_stride + k] = d.alpha;
        hist[4 * hist_stride + k] = nonbinary;
    }
    if (d.step) {
        ctl->alpha = d.alpha;
        ctl->alpha_last = d.alpha;
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

// The finish folded into a label pass: every workgroup of the graph's pass, once its partials
// are in memory, takes a ticket; the one that takes the last ticket (all partials of the
// iteration written) makes the finish of the iteration and resets the counter for the next.
// The label-pass partials are written through to memory (store_coherent) by the thread that
// takes the ticket, which waits for its stores to complete first; the finish reads every
// partial from memory (load_coherent), past the caches of its XCD, so the partials of
// workgroups on other XCDs are seen without a cache-wide fence.  (The row kernel's partials
// come from an earlier launch.)  Every thread of the workgroup must call it.  The result does
// not depend on which workgroup is last.
template <typename T>
__device__ __forceinline__ void finish_if_last(const GraphView<T> &gv, const double *row_part, int nb_row,
                                               const double *lab_part, int nb_lab)
{
    __shared__ int last;
    __syncthreads(); // the workgroup's partials are written
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0); // this thread's partial stores have completed
        const unsigned int ticket = atomicAdd(gv.ticket, 1u);
        last = ticket + 1u == (unsigned int)gv.n_lab_blocks;
    }
    __syncthreads();
    if (!last) return;
    double t[kRowParts + 1];
    finish_sums(row_part, nb_row, lab_part, nb_lab, t);
    if (threadIdx.x != 0) return;
    Ctl *ctl = gv.ctl;
    const Decision d = finish_decide(t, ctl->sp, ctl->one_shot);
    finish_commit(ctl, ctl->k, d, t[PART_NB]);
    *gv.ticket = 0u;
}

// A label pass of an iteration that is not evaluated (the solve has stopped): the update of
// the last evaluated iteration has just been made by the row kernel, so nothing is pending.
template <typename T>
__device__ __forceinline__ void label_inactive(const GraphView<T> &gv, const int tile)
{
    if (tile == 0 && threadIdx.x == 0) gv.ctl->pending = 0;
}

// U_0 = Uhat (labelled rows one-hot, others 1/K; Section 5.1), or a copy of U0, for the rows
// of tile `tile`.
template <typename T>
__device__ __forceinline__ void init_body(const GraphView<T> &gv, const T *__restrict__ U0, const int tile)
{
    const int32_t K = gv.K;
    const int64_t r0 = (int64_t)tile * kRowBlock;
    const int rows = (int)min((int64_t)kRowBlock, gv.n - r0);
    const T invK = (T)(1.0 / (double)K);
    for (int q = threadIdx.x; q < rows * K; q += kRowBlock) {
        const int64_t t = r0 * K + q;
        if (U0) {
            gv.U[t] = U0[t];
            continue;
        }
        const int64_t i = r0 + q / K;
        const int32_t c = q % K;
        const int32_t y = gv.lab[i];
        gv.U[t] = y >= 0 ? (c == y ? (T)1 : (T)0) : invK;
    }
}

// Row i of L U for the rows of tile `tile` (kRowBlock consecutive rows), FP64 sums.  L is
// I + A (kind W: A the stored scaled values, the identity implicit) or A itself (kind L).
// kSpmmLanes lanes share a row: lane l of the row holds classes l, l + 4, l + 8, l + 12, so
// that the lanes of a row gather one contiguous run of its neighbour's row of U.  Every lane
// walks all of the row's entries in CSR order (index and value read by the row's lanes
// together), with the identity's term u_i taken at the diagonal's place in that order (where
// a self-loop's entry a_ii stands, as (1 + a_ii) u_i; else before the first larger column):
// the order of a CSR loop over the explicit operator, so each class's sum rounds as that loop
// does.  UN entries are loaded before they are summed.  The result depends on nothing but the
// row.  K <= KB.
constexpr int kSpmmLanes = 4;
constexpr int kSpmmThreads = kRowBlock * kSpmmLanes;

// Row i of L U (lane l of the row's kSpmmLanes holds classes l, l + kSpmmLanes, ...); i < 0 or
// i >= n gives zeros.
template <typename T, int KB>
__device__ __forceinline__ void spmm_row(const GraphView<T> &gv, const T *__restrict__ Uin, const int64_t i,
                                         double (&acc)[KB / kSpmmLanes])
{
    constexpr int MC = KB / kSpmmLanes; // classes per lane
    constexpr int UN = 4;
    const int32_t K = gv.K;
    const int l = threadIdx.x % kSpmmLanes;
#pragma unroll
    for (int m = 0; m < MC; ++m) acc[m] = 0.0;
    if (i < 0 || i >= gv.n) return;
    const T *__restrict__ ui = Uin + i * K;
    bool diag_due = gv.diag_one != 0; // the identity's term is still to be added
    auto take = [&](const int32_t j, const double v, const T (&uj)[MC]) {
        if (diag_due && j >= (int32_t)i) {
            diag_due = false;
            if (j == (int32_t)i) { // a self-loop: (1 + a_ii) u_i
                const double w = 1.0 + v;
#pragma unroll
                for (int m = 0; m < MC; ++m) acc[m] += w * (double)uj[m];
                return;
            }
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = l + kSpmmLanes * m;
                if (c < K) acc[m] += (double)ui[c];
            }
        }
#pragma unroll
        for (int m = 0; m < MC; ++m) acc[m] += v * (double)uj[m];
    };
    const int32_t e0 = gv.rp[i], e1 = gv.rp[i + 1];
    int32_t e = e0;
    for (; e + UN <= e1; e += UN) {
        int32_t j[UN];
        double v[UN];
        T uu[UN][MC];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            j[u] = gv.ci[e + u];
            v[u] = (double)gv.a[e + u];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u)
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = l + kSpmmLanes * m;
                uu[u][m] = c < K ? Uin[(int64_t)j[u] * K + c] : (T)0;
            }
#pragma unroll
        for (int u = 0; u < UN; ++u) take(j[u], v[u], uu[u]);
    }
    for (; e < e1; ++e) {
        const int32_t j = gv.ci[e];
        T uj[MC];
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = l + kSpmmLanes * m;
            uj[m] = c < K ? Uin[(int64_t)j * K + c] : (T)0;
        }
        take(j, (double)gv.a[e], uj);
    }
    if (diag_due) // every column of the row precedes i
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = l + kSpmmLanes * m;
            if (c < K) acc[m] += (double)ui[c];
        }
}

template <typename T, int KB>
__device__ __forceinline__ void spmm_rows(const GraphView<T> &gv, const T *__restrict__ Uin, const int tile,
                                          double (&acc)[KB / kSpmmLanes])
{
    spmm_row<T, KB>(gv, Uin, (int64_t)tile * kRowBlock + threadIdx.x / kSpmmLanes, acc);
}

// P = L U for the rows of tile `tile`, stored as PT.  kSpmmThreads threads.
template <typename T, int KB, typename PT>
__device__ __forceinline__ void spmm_body(const GraphView<T> &gv, const T *__restrict__ Uin, PT *__restrict__ Pout,
                                          const int tile)
{
    constexpr int MC = KB / kSpmmLanes;
    double acc[MC];
    spmm_rows<T, KB>(gv, Uin, tile, acc);
    const int l = threadIdx.x % kSpmmLanes;
    const int64_t i = (int64_t)tile * kRowBlock + threadIdx.x / kSpmmLanes;
    if (i < gv.n)
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = l + kSpmmLanes * m;
            if (c < gv.K) Pout[i * gv.K + c] = (PT)acc[m];
        }
}

template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_init_u(GraphView<T> gv, const T *__restrict__ U0)
{
    init_body<T>(gv, U0, blockIdx.x);
}

template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_init_u_batch(const GraphView<T> *__restrict__ views,
                                                             const TileRef *__restrict__ refs,
                                                             const T *const *__restrict__ U0s)
{
    const TileRef r = refs[blockIdx.x];
    init_body<T>(views[r.graph], U0s ? U0s[r.graph] : nullptr, r.tile);
}

template <typename T, int KB, typename PT>
static __global__ void __launch_bounds__(kSpmmThreads) k_spmm(GraphView<T> gv, const T *__restrict__ Uin, PT *__restrict__ Pout)
{
    spmm_body<T, KB, PT>(gv, Uin, Pout, blockIdx.x);
}

// batched L_s U_0 -> P at the start of a batched solve
template <typename T, int KB>
static __global__ void __launch_bounds__(kSpmmThreads) k_spmm_batch(const GraphView<T> *__restrict__ views,
                                                           const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    const GraphView<T> &gv = views[r.graph];
    spmm_body<T, KB, double>(gv, gv.U, gv.P, r.tile);
}

// ---------------------------------------------------------------------------------
// single-graph and batched entry points
// ---------------------------------------------------------------------------------
template <typename T, typename ST, int KB>
static __global__ void __launch_bounds__(kRowBlock) k_row(GraphView<T> gv, int apply_only)
{
    row_body<T, ST, KB>(gv, blockIdx.x, apply_only);
}

template <typename T, typename ST, int KB>
static __global__ void __launch_bounds__(kRowBlock) k_row_batch(const GraphView<T> *__restrict__ views,
                                                          const TileRef *__restrict__ refs, int apply_only)
{
    const TileRef r = refs[blockIdx.x];
    row_body<T, ST, KB>(views[r.graph], r.tile, apply_only);
}

template <typename T, typename ST, int KB>
static __global__ void __launch_bounds__(kRowBlock) k_label(GraphView<T> gv)
{
    label_body<T, ST, KB, kLabelTileSingle>(gv, blockIdx.x);
}

// LT: CSR entries staged per sub-tile (1,024, 2,048 or 4,096, chosen per batch by measurement;
// the sub-tiles change no sum)
template <typename T, typename ST, int KB, int LT>
static __global__ void __launch_bounds__(kRowBlock) k_label_batch(const GraphView<T> *__restrict__ views,
                                                            const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    label_body<T, ST, KB, LT>(views[r.graph], r.tile);
}

// The label-pass ticket of every graph of a batch set to `value` (a preset that no pass
// completes keeps timing launches from making a finish; 0 restores it).
template <typename T>
static __global__ void k_set_tickets_batch(const GraphView<T> *__restrict__ views, int32_t count, unsigned int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) *views[i].ticket = value;
}

template <typename T, typename ST, int KB>
static __global__ void __launch_bounds__(kSortedThreads) k_label_sorted(GraphView<T> gv)
{
    label_sorted_body<T, ST, KB>(gv, blockIdx.x);
}

template <typename T, typename ST, int KB>
static __global__ void __launch_bounds__(kSortedThreads) k_label_sorted_batch(const GraphView<T> *__restrict__ views,
                                                                        const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    label_sorted_body<T, ST, KB>(views[r.graph], r.tile);
}

// Terms of E(U) (eq. gl_vv2) from their definitions for the rows of tile `tile`: row i of
// P = L U is formed in FP64 (spmm_rows, kSpmmLanes lanes per row) and used at once, never
// stored; then <u_i, P_i>, sum u(1-u) and omega_i ||uhat_i - u_i||^2; block sums (fixed order:
// wavefront trees, then wavefronts in order) stored at part[j * stride + tile].
template <typename T, int KB>
__device__ __forceinline__ void energy_body(const GraphView<T> &gv, const T *__restrict__ U, double omega0,
                                            double *__restrict__ part, int64_t stride, const int tile)
{
    constexpr int MC = KB / kSpmmLanes;
    double p[MC];
    spmm_rows<T, KB>(gv, U, tile, p);
    double acc[3] = {0.0, 0.0, 0.0};
    const int l = threadIdx.x % kSpmmLanes;
    const int64_t i = (int64_t)tile * kRowBlock + threadIdx.x / kSpmmLanes;
    if (i < gv.n) {
        const int32_t y = gv.lab[i];
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = l + kSpmmLanes * m;
            if (c < gv.K) {
                const double u = (double)U[i * gv.K + c];
                acc[0] += u * p[m];
                acc[1] += u * (1.0 - u);
                if (y >= 0) {
                    const double e = (c == y ? 1.0 : 0.0) - u;
                    acc[2] += omega0 * e * e;
                }
            }
        }
    }
    __shared__ double red[kSpmmThreads / 64][3];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = wave_sum(acc[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) red[wid][j] = acc[j];
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < kSpmmThreads / 64; ++w) t += red[w][threadIdx.x];
        part[threadIdx.x * stride + tile] = t;
    }
}

// E = 1/2 <U, L U> + (1/eps) sum u(1-u) + 1/2 sum omega ||uhat - u||^2 from the tile partials.
__device__ __forceinline__ void energy_sum_body(const double *__restrict__ part, int nb, double inv_eps,
                                                double *__restrict__ out)
{
    __shared__ double red[kFinishThreads / 64][3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kFinishThreads)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j] += part[(int64_t)j * nb + b];
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = wave_sum(v[j]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) red[threadIdx.x >> 6][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < kFinishThreads / 64; ++w)
#pragma unroll
            for (int j = 0; j < 3; ++j) t[j] += red[w][j];
        *out = 0.5 * t[0] + inv_eps * t[1] + 0.5 * t[2];
    }
}

template <typename T, int KB>
static __global__ void __launch_bounds__(kSpmmThreads) k_energy(GraphView<T> gv, const T *__restrict__ U, double omega0,
                                                       double *__restrict__ part)
{
    energy_body<T, KB>(gv, U, omega0, part, gv.nb_row, blockIdx.x);
}

static __global__ void __launch_bounds__(kFinishThreads) k_energy_sum(const double *__restrict__ part, int nb,
                                                               double inv_eps, double *__restrict__ out)
{
    energy_sum_body(part, nb, inv_eps, out);
}

// batched objective of the final iterates: tile partials of E to row_part
template <typename T, int KB>
static __global__ void __launch_bounds__(kSpmmThreads) k_energy_batch(const GraphView<T> *__restrict__ views,
                                                             const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    const GraphView<T> &gv = views[r.graph];
    energy_body<T, KB>(gv, gv.U, gv.ctl->sp.omega0, gv.row_part, gv.nb_row, r.tile);
}

// one workgroup per graph: objective and a copy of the control block
template <typename T>
static __global__ void __launch_bounds__(kFinishThreads) k_collect_batch(const GraphView<T> *__restrict__ views,
                                                                  double *__restrict__ E, Ctl *__restrict__ ctls)
{
    const GraphView<T> &gv = views[blockIdx.x];
    energy_sum_body(gv.row_part, gv.nb_big > 0 ? gv.nb_big : gv.nb_row, gv.ctl->sp.inv_eps, E + blockIdx.x);
    if (threadIdx.x == 0) ctls[blockIdx.x] = *gv.ctl;
}

// writes the initial control blocks of a batch
template <typename T>
static __global__ void k_set_ctl_batch(const GraphView<T> *__restrict__ views, const Ctl *__restrict__ src, int count)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < count; g += gridDim.x * blockDim.x) *views[g].ctl = src[g];
}

// labels (lowest-index argmax of each row of U) for the rows of a tile
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_labels_batch(const GraphView<T> *__restrict__ views,
                                                             const TileRef *__restrict__ refs,
                                                             int32_t *const *__restrict__ outs)
{
    const TileRef r = refs[blockIdx.x];
    const GraphView<T> &gv = views[r.graph];
    int32_t *out = outs[r.graph];
    const int64_t i = (int64_t)r.tile * kRowBlock + threadIdx.x;
    if (!out || i >= gv.n) return;
    const T *u = gv.U + i * gv.K;
    int32_t at = 0;
    T best = u[0];
    for (int32_t c = 1; c < gv.K; ++c)
        if (u[c] > best) {
            best = u[c];
            at = c;
        }
    out[i] = at;
}

// 1 while some graph of the batch still has an iteration to evaluate or an update to commit
template <typename T>
static __global__ void k_any_active(const GraphView<T> *__restrict__ views, int count, int32_t *__restrict__ flag)
{
    int a = 0;
    for (int g = threadIdx.x; g < count; g += blockDim.x) a |= views[g].ctl->active | views[g].ctl->pending;
    a = __syncthreads_or(a);
    if (threadIdx.x == 0) *flag = a;
}

template <typename T>
static __global__ void k_clear_pending_batch(const GraphView<T> *__restrict__ views, int count)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < count; g += gridDim.x * blockDim.x)
        views[g].ctl->pending = 0;
}

template <typename T>
static __global__ void k_ctl_gather_batch(const GraphView<T> *__restrict__ views, Ctl *__restrict__ out, int count)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < count; g += gridDim.x * blockDim.x) out[g] = *views[g].ctl;
}

// labels_i = lowest-index argmax_c U_ic; s_out = vertex indices of the last GLMO output
// (-1 when no iteration was evaluated).
template <typename T, typename ST>
static __global__ void k_outputs(int64_t n, int32_t K, const T *__restrict__ U, const ST *__restrict__ s0,
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

static __global__ void k_clear_pending(Ctl *ctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->pending = 0;
}

// Largest of n non-negative values over all blocks of the grid.  A non-negative IEEE double
// orders like its bit pattern as an unsigned integer, so the block maxima are combined with
// an integer atomic max (the result does not depend on the order).  *out must hold 0 first.
static __global__ void k_max_nonneg(const double *__restrict__ v, int64_t n, unsigned long long *__restrict__ out)
{
    __shared__ double red[256 / 64];
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, v[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
        atomicMax(out, (unsigned long long)__double_as_longlong(s));
    }
}

// Streaming copy of n16 16-byte vectors (the achievable HBM rate the roofline is compared
// with): each thread moves CU vectors per step, all loads issued before the stores,
// non-temporal both ways, grid-stride over the array.
static __global__ void __launch_bounds__(256) k_stream_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                            int64_t n16)
{
    constexpr int CU = 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n16; b += stride * CU) {
        v4u x[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int64_t q = b + u * stride;
            if (q < n16) x[u] = __builtin_nontemporal_load(src + q);
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int64_t q = b + u * stride;
            if (q < n16) __builtin_nontemporal_store(x[u], dst + q);
        }
    }
}

} // namespace gfw
