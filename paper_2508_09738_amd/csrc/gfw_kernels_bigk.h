// ---------------------------------------------------------------------------------
// Kernels for many classes (16 < K <= 1024), the regime of the paper's LFR networks
// (Section 5.2: hundreds of communities, average degree about 5).
//
// With K this large a row of U, P or Q is K wide and no longer fits one thread's
// registers, while the CSR row is short.  The iteration keeps the structure of the
// small-K path (row kernel, label pass, finish) with three changes:
//  * a wavefront owns a row: lane l holds classes l, l + 64, l + 128, ... (MC per lane),
//    so every row of U and P is read and written with coalesced accesses, and the
//    GLMO's lowest-index argmin and the per-row sums are wavefront reductions;
//  * Q = L_s S is never stored: S is one-hot, so the row (L_s S_{k-1})_i has at most
//    deg_i + 1 non-zeros, and the row kernel of iteration k rebuilds it (FP64 sums, rounded
//    to the graph's dtype as the small-K label pass stores Q) from the row's values and its
//    neighbours' vertices s_{k-1} just before the update P_k = (1 - a) P_{k-1} + a Q_{k-1}
//    (P in FP64).  That saves writing and reading an n x K array;
//  * the label pass forms the per-row term Q_{i,s_i} of <S, L_s S> (the sum of the row's
//    values over neighbours that share its vertex, plus the diagonal), which does not
//    depend on K, and stores each entry's neighbour vertex (nv, 2 bytes per entry), so
//    that the row kernel reads the vertices it needs with plain loads instead of a
//    dependent gather.
// Vertices are 16-bit (K up to 1024).  Every sum over a row runs in a fixed order, so
// the results are deterministic; the sums over a row's classes are wavefront trees and
// differ from a sequential sum by rounding only.
// ---------------------------------------------------------------------------------
#pragma once

#include "gfw_kernels.h"

#include <limits.h>

namespace gfw {

constexpr int kBigThreads = 256;                             // 4 wavefronts per block
constexpr int kBigRowsPerWave = 1;                           // rows a wavefront takes in turn
constexpr int kBigRowsPerBlock = kBigRowsPerWave * (kBigThreads / 64);

// Wavefront minimum (the DPP steps of wave_sum).
__device__ __forceinline__ int wave_min_int(int v)
{
    v = min(v, dpp_i32<kDppQuadSwap1>(v, INT_MAX));
    v = min(v, dpp_i32<kDppQuadSwap2>(v, INT_MAX));
    v = min(v, dpp_i32<kDppRowHalfMirror>(v, INT_MAX));
    v = min(v, dpp_i32<kDppRowMirror>(v, INT_MAX));
    v = min(v, dpp_i32<kDppRowBcast15, 0xa>(v, INT_MAX));
    v = min(v, dpp_i32<kDppRowBcast31, 0xc>(v, INT_MAX));
    return __builtin_amdgcn_readlane(v, 63);
}

// One step of the lowest-index minimum: take the pair (ov, oi) read from another lane if it
// is a candidate that precedes (v, idx).
__device__ __forceinline__ void argmin_take(double &v, int &idx, const double ov, const int oi)
{
    const bool take = oi != INT_MAX && (idx == INT_MAX || ov < v || (ov == v && oi < idx));
    if (take) {
        v = ov;
        idx = oi;
    }
}

// Lowest-index minimum over the wavefront of (value, index) pairs; index INT_MAX marks a
// lane without a candidate.  The pairs are totally ordered, so the result does not depend on
// the order of the steps; every lane ends with it.
__device__ __forceinline__ void wave_argmin(double &v, int &idx)
{
    argmin_take(v, idx, dpp_f64<kDppQuadSwap1>(v, v), dpp_i32<kDppQuadSwap1>(idx, INT_MAX));
    argmin_take(v, idx, dpp_f64<kDppQuadSwap2>(v, v), dpp_i32<kDppQuadSwap2>(idx, INT_MAX));
    argmin_take(v, idx, dpp_f64<kDppRowHalfMirror>(v, v), dpp_i32<kDppRowHalfMirror>(idx, INT_MAX));
    argmin_take(v, idx, dpp_f64<kDppRowMirror>(v, v), dpp_i32<kDppRowMirror>(idx, INT_MAX));
    argmin_take(v, idx, dpp_f64<kDppRowBcast15, 0xa>(v, v), dpp_i32<kDppRowBcast15, 0xa>(idx, INT_MAX));
    argmin_take(v, idx, dpp_f64<kDppRowBcast31, 0xc>(v, v), dpp_i32<kDppRowBcast31, 0xc>(idx, INT_MAX));
    v = readlane_f64(v, 63);
    idx = __builtin_amdgcn_readlane(idx, 63);
}

// Row kernel for large K: pending update (with the Q row rebuilt from s_{k-1}), gradient,
// GLMO, per-row partials.  Block `tile` owns rows [tile * kBigRowsPerBlock, +kBigRowsPerBlock);
// partials are stored transposed with stride nb_big: row_part[j * nb_big + tile].
template <typename T, int MC>
__device__ __forceinline__ void row_big_body(const GraphView<T> &gv, const int tile, const int apply_only)
{
    const int64_t n = gv.n;
    const int32_t K = gv.K;
    const Ctl *__restrict__ ctl = gv.ctl;
    const int32_t active = apply_only ? 0 : ctl->active, pending = ctl->pending;
    if (!active && !pending) return;
    const uint16_t *__restrict__ s_prev = reinterpret_cast<const uint16_t *>((ctl->last_eval & 1) ? gv.s1 : gv.s0);
    uint16_t *__restrict__ s_cur = reinterpret_cast<uint16_t *>((ctl->k & 1) ? gv.s1 : gv.s0);
    const int32_t *__restrict__ rp = gv.rp;
    const T *__restrict__ a = gv.a;
    const double alpha = ctl->alpha;
    const SolveParams sp = ctl->sp;
    const uint16_t *__restrict__ nv = gv.nv;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double wacc[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) wacc[j] = 0.0;
    const int64_t rbase = (int64_t)tile * kBigRowsPerBlock + (int64_t)wid * kBigRowsPerWave;
    // row pointers, label and previous vertex of the wavefront's rows, one row per lane
    int32_t md_b = 0, md_e = 0, md_y = -1, md_sp = 0;
    if (lane < kBigRowsPerWave && rbase + lane < n) {
        md_b = rp[rbase + lane];
        md_e = rp[rbase + lane + 1];
        md_y = gv.lab[rbase + lane];
        md_sp = pending ? (int32_t)s_prev[rbase + lane] : 0;
    }
    for (int t = 0; t < kBigRowsPerWave; ++t) {
        const int64_t i = rbase + t;
        if (i >= n) break; // uniform across the wavefront
        T *__restrict__ Ui = gv.U + i * K;
        double *__restrict__ Pi = gv.P + i * K;
        // u is held at storage precision (every value is rounded to T anyway) and widened to
        // FP64 where it is used; p is FP64 (the carried L_s U)
        T u[MC];
        double p[MC];
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = lane + 64 * m;
            u[m] = c < K ? __builtin_nontemporal_load(Ui + c) : (T)0;
            p[m] = c < K ? __builtin_nontemporal_load(Pi + c) : 0.0;
        }
        bool bl = true;
#pragma unroll
        for (int m = 0; m < MC; ++m)
            if (lane + 64 * m < K && !(u[m] == (T)0 || u[m] == (T)1)) bl = false;
        bool binary = __all(bl);
        if (pending) {
            const int32_t spi = __shfl(md_sp, t, 64);
            // Q_{k-1} row i: values of the row summed per neighbour vertex, in CSR order.  The
            // row's entries are loaded one per lane (64 at a time) with their vertices, then
            // taken in order from the lanes that hold them.
            double q[MC];
#pragma unroll
            for (int m = 0; m < MC; ++m) q[m] = 0.0;
            const int32_t e0 = __shfl(md_b, t, 64), e1 = __shfl(md_e, t, 64);
            for (int32_t c0 = e0; c0 < e1; c0 += 64) {
                const int cnt = min(64, e1 - c0);
                int32_t sj_l = 0;
                T v_l = (T)0;
                if (lane < cnt) {
                    sj_l = (int32_t)nv[c0 + lane];
                    v_l = a[c0 + lane];
                }
                for (int x = 0; x < cnt; ++x) {
                    const int32_t sj = __shfl(sj_l, x, 64);
                    const double v = (double)__shfl(v_l, x, 64);
                    if ((sj & 63) == lane) {
#pragma unroll
                        for (int m = 0; m < MC; ++m)
                            if (m == (sj >> 6)) q[m] += v;
                    }
                }
            }
            if (gv.diag_one && (spi & 63) == lane) {
#pragma unroll
                for (int m = 0; m < MC; ++m)
                    if (m == (spi >> 6)) q[m] += 1.0;
            }
            const double om = 1.0 - alpha;
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = lane + 64 * m;
                if (c < K) {
                    // Q_{k-1} rounded to the graph's dtype, as the small-K label pass stores it
                    p[m] = om * p[m] + alpha * (double)(T)q[m];
                    __builtin_nontemporal_store(p[m], Pi + c);
                }
            }
            // a row whose direction e_{s_i} - u_i is zero (binary, kept by the GLMO) stays as it is
            double us = 0.0;
#pragma unroll
            for (int m = 0; m < MC; ++m)
                if (m == (spi >> 6)) us = (double)u[m];
            const double at_s = __shfl(us, spi & 63, 64);
            if (!(binary && at_s == 1.0)) {
                bl = true;
#pragma unroll
                for (int m = 0; m < MC; ++m) {
                    const int c = lane + 64 * m;
                    if (c < K) {
                        u[m] = (T)(om * (double)u[m] + (c == spi ? alpha : 0.0));
                        __builtin_nontemporal_store(u[m], Ui + c);
                        if (!(u[m] == (T)0 || u[m] == (T)1)) bl = false;
                    }
                }
                binary = __all(bl);
            }
        }
        if (active) {
            const int32_t y = __shfl(md_y, t, 64);
            const double om_i = y >= 0 ? sp.omega0 : 0.0;
            // gradient entry of class c (eq. gradgl_vv2g), formed where it is used
            auto grad = [&](const int m, const int c) -> double {
                const double uc = (double)u[m];
                const double fid = om_i != 0.0 ? om_i * (((c == y) ? 1.0 : 0.0) - uc) : 0.0;
                return p[m] + sp.inv_eps * (1.0 - 2.0 * uc) - fid;
            };
            int32_t s;
            if (binary && sp.lmo == 0) {
                // the GLMO keeps a binary row: its vertex is the position of its 1
                int cand = INT_MAX;
#pragma unroll
                for (int m = 0; m < MC; ++m) {
                    const int c = lane + 64 * m;
                    if (c < K && u[m] == (T)1) cand = min(cand, c);
                }
                cand = wave_min_int(cand);
                s = cand == INT_MAX ? 0 : cand;
            } else {
                double best = 0.0;
                int bi = INT_MAX;
#pragma unroll
                for (int m = 0; m < MC; ++m) {
                    const int c = lane + 64 * m;
                    if (c < K && (sp.lmo == 1 || u[m] != (T)0)) {
                        const double gm = grad(m, c);
                        if (bi == INT_MAX || gm < best) {
                            best = gm;
                            bi = c;
                        }
                    }
                }
                wave_argmin(best, bi);
                s = bi == INT_MAX ? 0 : bi;
            }
            if (lane == 0) s_cur[i] = (uint16_t)s;
            double gap = 0.0, up = 0.0, dd = 0.0, pen = 0.0, fid = 0.0, ps = 0.0;
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = lane + 64 * m;
                if (c < K) {
                    const double uc = (double)u[m], pc = p[m];
                    const double d = (c == s ? 1.0 : 0.0) - uc;
                    gap -= grad(m, c) * d;
                    up += uc * pc;
                    dd += d * d;
                    pen += uc * (1.0 - uc);
                    if (c == s) ps = pc;
                    if (om_i != 0.0) {
                        const double e = (y == c ? 1.0 : 0.0) - uc;
                        fid += e * e;
                    }
                }
            }
            gap = wave_sum(gap);
            up = wave_sum(up);
            dd = wave_sum(dd);
            pen = wave_sum(pen);
            fid = wave_sum(fid);
            ps = wave_sum(ps);
            wacc[PART_GAP] += gap;
            wacc[PART_E] += 0.5 * up + sp.inv_eps * pen + 0.5 * (om_i * fid);
            wacc[PART_CURV] += up - 2.0 * ps - 2.0 * sp.inv_eps * dd + om_i * dd;
            wacc[PART_DD] += dd;
            wacc[PART_NB] += binary ? 0.0 : 1.0;
        }
    }
    if (!active) return; // uniform across the block
    __shared__ double red[kBigThreads / 64][kRowParts];
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < kRowParts; ++j) red[wid][j] = wacc[j];
    }
    __syncthreads();
    if (threadIdx.x < kRowParts) {
        double s = 0.0;
        for (int w = 0; w < kBigThreads / 64; ++w) s += red[w][threadIdx.x];
        gv.row_part[(int64_t)threadIdx.x * gv.nb_big + tile] = s;
    }
}

// Label pass for large K: the per-row term Q_{i,s_i} = sum of the row's values over
// neighbours with vertex s_i (CSR order) + the diagonal, and each entry's neighbour vertex
// nv[e] = s_{ci[e]} for the next row kernel; one thread per row, 256-row blocks; partial
// lab_part[tile].
template <typename T>
__device__ __forceinline__ void label_big_body(const GraphView<T> &gv, const int tile)
{
    const Ctl *__restrict__ ctl = gv.ctl;
    if (!ctl->active) return label_inactive(gv, tile);
    const uint16_t *__restrict__ s = reinterpret_cast<const uint16_t *>((ctl->k & 1) ? gv.s1 : gv.s0);
    const int64_t i = (int64_t)tile * kRowBlock + threadIdx.x;
    // the row kernel's partials of a fixed slice of its blocks, folded into this block's entry
    // of row_fold (loaded here by the first wavefront, summed at the end), so that the finish
    // reads nb_row partials instead of nb_big
    const int nbb = gv.nb_big, nbr = gv.nb_row;
    const int fb0 = (int)((int64_t)tile * nbb / nbr), fb1 = (int)((int64_t)(tile + 1) * nbb / nbr);
    double fold[kRowParts];
#pragma unroll
    for (int j = 0; j < kRowParts; ++j) fold[j] = 0.0;
    if (threadIdx.x < 64)
        for (int b = fb0 + (int)threadIdx.x; b < fb1; b += 64)
#pragma unroll
            for (int j = 0; j < kRowParts; ++j) fold[j] += gv.row_part[(int64_t)j * nbb + b];
    double own = 0.0;
    if (i < gv.n) {
        const int32_t si = (int32_t)s[i];
        double acc = 0.0;
        const int32_t e0 = gv.rp[i], e1 = gv.rp[i + 1];
        for (int32_t e = e0; e < e1; ++e) {
            const uint16_t sj = s[gv.ci[e]];
            gv.nv[e] = sj;
            if ((int32_t)sj == si) acc += (double)gv.a[e];
        }
        own = (double)(T)(acc + (gv.diag_one ? 1.0 : 0.0));
    }
    if (threadIdx.x < 64) { // the whole first wavefront
#pragma unroll
        for (int j = 0; j < kRowParts; ++j) fold[j] = wave_sum(fold[j]);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < kRowParts; ++j) store_coherent(gv.row_fold + (int64_t)j * nbr + tile, fold[j]);
    }
    double v[1] = {own};
    block_sum_store_strided<1, true>(v, gv.lab_part + tile, gv.nb_row);
    finish_if_last(gv, gv.row_fold, gv.nb_row, gv.lab_part, gv.nb_row);
}

// Row i of L U for large K, one wavefront per row, each lane accumulating its classes over
// the row's entries in CSR order in FP64, with the identity's term at the diagonal's place
// (the order and arithmetic of spmm_rows).  Four neighbour rows (two for more than four
// classes per lane) are loaded before they are summed.  `fn(i, acc)` receives each finished row (acc[m] is class lane + 64 m).
template <typename T, int MC, typename Fn>
__device__ __forceinline__ void spmm_big_rows(const GraphView<T> &gv, const T *__restrict__ Uin, const int tile,
                                              Fn &&fn)
{
    const int32_t K = gv.K;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t rbase = (int64_t)tile * kBigRowsPerBlock + (int64_t)wid * kBigRowsPerWave;
    for (int t = 0; t < kBigRowsPerWave; ++t) {
        const int64_t i = rbase + t;
        if (i >= gv.n) break; // uniform across the wavefront
        double acc[MC];
#pragma unroll
        for (int m = 0; m < MC; ++m) acc[m] = 0.0;
        const T *__restrict__ ui = Uin + i * K;
        bool diag_due = gv.diag_one != 0;
        auto take = [&](const int32_t j, const double v, const T (&uj)[MC]) {
            if (diag_due && j >= (int32_t)i) {
                diag_due = false;
                if (j == (int32_t)i) {
                    const double w = 1.0 + v;
#pragma unroll
                    for (int m = 0; m < MC; ++m) acc[m] += w * (double)uj[m];
                    return;
                }
#pragma unroll
                for (int m = 0; m < MC; ++m) {
                    const int c = lane + 64 * m;
                    acc[m] += c < K ? (double)ui[c] : 0.0;
                }
            }
#pragma unroll
            for (int m = 0; m < MC; ++m) acc[m] += v * (double)uj[m];
        };
        const int32_t e0 = gv.rp[i], e1 = gv.rp[i + 1];
        int32_t e = e0;
        constexpr int UN = MC <= 4 ? 4 : 2;
        for (; e + UN <= e1; e += UN) {
            int32_t j[UN];
            T uu[UN][MC];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                j[u] = gv.ci[e + u];
#pragma unroll
                for (int m = 0; m < MC; ++m) {
                    const int c = lane + 64 * m;
                    uu[u][m] = c < K ? Uin[(int64_t)j[u] * K + c] : (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < UN; ++u) take(j[u], (double)gv.a[e + u], uu[u]);
        }
        for (; e < e1; ++e) {
            const int32_t j = gv.ci[e];
            T uj[MC];
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = lane + 64 * m;
                uj[m] = c < K ? Uin[(int64_t)j * K + c] : (T)0;
            }
            take(j, (double)gv.a[e], uj);
        }
        if (diag_due)
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                const int c = lane + 64 * m;
                acc[m] += c < K ? (double)ui[c] : 0.0;
            }
        fn(i, acc);
    }
}

// P = L U for large K, stored as PT.
template <typename T, int MC, typename PT>
__device__ __forceinline__ void spmm_big_body(const GraphView<T> &gv, const T *__restrict__ Uin, PT *__restrict__ Pout,
                                              const int tile)
{
    const int lane = threadIdx.x & 63;
    spmm_big_rows<T, MC>(gv, Uin, tile, [&](const int64_t i, const double (&acc)[MC]) {
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = lane + 64 * m;
            if (c < gv.K) Pout[i * gv.K + c] = (PT)acc[m];
        }
    });
}

// Terms of E(U) for large K (the quantities of energy_body): each wavefront forms its rows of
// L U (spmm_big_rows) and sums the row's terms across lanes; block sums stored at
// part[j * stride + tile], with the blocks of the large-K row kernel.
template <typename T, int MC>
__device__ __forceinline__ void energy_big_body(const GraphView<T> &gv, const T *__restrict__ U, double omega0,
                                                double *__restrict__ part, int64_t stride, const int tile)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double wacc[3] = {0.0, 0.0, 0.0};
    spmm_big_rows<T, MC>(gv, U, tile, [&](const int64_t i, const double (&p)[MC]) {
        const int32_t y = gv.lab[i];
        double t[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < MC; ++m) {
            const int c = lane + 64 * m;
            if (c < gv.K) {
                const double u = (double)U[i * gv.K + c];
                t[0] += u * p[m];
                t[1] += u * (1.0 - u);
                if (y >= 0) {
                    const double e = (c == y ? 1.0 : 0.0) - u;
                    t[2] += omega0 * e * e;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) wacc[j] += wave_sum(t[j]);
    });
    __shared__ double red[kBigThreads / 64][3];
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) red[wid][j] = wacc[j];
    __syncthreads();
    if (threadIdx.x < 3) {
        double v = 0.0;
        for (int w = 0; w < kBigThreads / 64; ++w) v += red[w][threadIdx.x];
        part[threadIdx.x * stride + tile] = v;
    }
}

template <typename T, int MC>
static __global__ void __launch_bounds__(kBigThreads) k_energy_big(GraphView<T> gv, const T *__restrict__ U,
                                                                   double omega0, double *__restrict__ part)
{
    energy_big_body<T, MC>(gv, U, omega0, part, gv.nb_big, blockIdx.x);
}

template <typename T, int MC>
static __global__ void __launch_bounds__(kBigThreads) k_energy_big_batch(const GraphView<T> *__restrict__ views,
                                                                         const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    const GraphView<T> &gv = views[r.graph];
    energy_big_body<T, MC>(gv, gv.U, gv.ctl->sp.omega0, gv.row_part, gv.nb_big, r.tile);
}

template <typename T, int MC>
static __global__ void __launch_bounds__(kBigThreads) k_row_big(GraphView<T> gv, int apply_only)
{
    row_big_body<T, MC>(gv, blockIdx.x, apply_only);
}

template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_label_big(GraphView<T> gv)
{
    label_big_body<T>(gv, blockIdx.x);
}

template <typename T, int MC, typename PT>
static __global__ void __launch_bounds__(kBigThreads) k_spmm_big(GraphView<T> gv, const T *__restrict__ Uin,
                                                                 PT *__restrict__ Pout)
{
    spmm_big_body<T, MC, PT>(gv, Uin, Pout, blockIdx.x);
}

// Batched forms: workgroup -> (graph, tile) through the TileRef table, the same bodies on
// the same tiles as the single-graph kernels.  A graph's results do not depend on MC as long
// as 64 * MC >= K (the slots past K take no part in any sum), so a batch groups graphs into
// a few MC buckets.
template <typename T, int MC>
static __global__ void __launch_bounds__(kBigThreads) k_row_big_batch(const GraphView<T> *__restrict__ views,
                                                                      const TileRef *__restrict__ refs, int apply_only)
{
    const TileRef r = refs[blockIdx.x];
    row_big_body<T, MC>(views[r.graph], r.tile, apply_only);
}

template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_label_big_batch(const GraphView<T> *__restrict__ views,
                                                                      const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    label_big_body<T>(views[r.graph], r.tile);
}

// P = L_s U at the start of a batched solve
template <typename T, int MC>
static __global__ void __launch_bounds__(kBigThreads) k_spmm_big_batch(const GraphView<T> *__restrict__ views,
                                                                       const TileRef *__restrict__ refs)
{
    const TileRef r = refs[blockIdx.x];
    const GraphView<T> &gv = views[r.graph];
    spmm_big_body<T, MC, double>(gv, gv.U, gv.P, r.tile);
}

} // namespace gfw
