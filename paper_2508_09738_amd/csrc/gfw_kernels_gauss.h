// ---------------------------------------------------------------------------------
// Fully connected Gaussian graphs (the image setting of Section 5.1): nodes are feature
// vectors x_i in R^d, w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) for i != j (eq. of the
// Gaussian similarity in Section 1), no self-loops.  The n x n matrix is never formed: every
// product R = W V (V n x K) is summed from the features, by one of two methods.
//
//  * exact: R_i = sum_{j != i} w_ij V_j, the weights formed where they are used (in the
//    graph's dtype, summed in FP64); O(n^2 K), the reference operator and the right one for
//    images of a few 10^4 pixels.
//  * grid (d <= 3): a fast summation in the spirit of the NFFT-based one the paper uses.
//    With unnormalised Gaussians g_w(r) = exp(-r^2 / (2 w^2)) and sigma^2 = 2 tau^2 + s^2,
//    the convolution g_tau * g_s * g_tau is (2 pi tau^2 s / sigma) g_sigma per dimension, so
//        w(x - y) = c^d sum_a sum_b g_tau(x - a) g_s(a - b) g_tau(b - y),
//    c = h^2 sigma / (2 pi tau^2 s), is exact in the limit of grid spacing h -> 0 (a, b grid
//    points).  The three factors are three passes: gather the points onto the grid with the
//    window g_tau (each grid cell sums the points binned in the cells around it, in a fixed
//    order: deterministic, no atomics), convolve the grid with g_s one axis at a time, and
//    interpolate back at every point with g_tau.  tau^2 = (1 - 1/sqrt 2) sigma^2 makes the
//    narrowest Gaussian summed on the grid as wide as it can be (0.414 sigma).  The grid
//    spacing h = sigma / 2 and windows cut at 5 widths leave a relative error of about 1e-7
//    per product (trapezoid rule on a Gaussian of width w: about 2 exp(-2 pi^2 w^2 / h^2),
//    cut tails exp(-12.5)).  Since h, tau and s are fixed multiples of sigma, so are the
//    half-widths in cells: kGridRW for the window, kGridRC for the convolution.
//    The self term (w_ii = 0) is removed by subtracting V_i (the sum gives it weight 1).
//  For both, L_s V = V - D^{-1/2} W D^{-1/2} V with the degrees d = W 1.  The n x K blocks
//  summed (V, R = W V, the grid's G) are stored with a padded row stride KP (1, 4, 8 or 16,
//  the padding columns zero), so that every kernel's class loop has a compile-time length.
// ---------------------------------------------------------------------------------
#pragma once

#include "gfw_kernels.h"

namespace gfw {

constexpr int kGaussMaxDim = 8;   // feature dimensions of the exact method
constexpr int kGridMaxDim = 3;    // feature dimensions of the grid method
constexpr double kGridSpacing = 0.5; // h / sigma
constexpr double kGridCut = 5.0;     // widths at which the window and the convolution stop
constexpr int kGridRW = 6;        // ceil(kGridCut tau / h): the window reaches cells c - 6 .. c + 7
constexpr int kGridRC = 7;        // ceil(kGridCut s / h): the convolution's taps -7 .. 7
constexpr int kGridWin = 2 * kGridRW + 2; // grid points per dimension in a point's window

struct GaussView {
    int64_t n;
    int32_t d;
    double inv2s2;               // 1 / (2 sigma^2)
    const double *x;             // n x d features
    const float *xf;             // the features in FP32 (FP32 graphs: their weights are FP32)
    const double *dinv;          // d_i^{-1/2} (0 for an isolated node)
    // grid method
    int32_t gdim[kGridMaxDim];   // cells per dimension (1 past d)
    int64_t gstride[kGridMaxDim];// linear stride of each dimension
    int64_t ncells;
    double g0[kGridMaxDim];      // coordinate of cell 0 per dimension
    double h;                    // grid spacing
    double inv2t2, inv2s2g;      // 1 / (2 tau^2), 1 / (2 s^2)
    double cnorm;                // c^d
    double ctap[kGridRC + 1];    // g_s(t h), t = 0 .. kGridRC
    const int32_t *cell_start;   // ncells + 1: the points of cell a are cell_pts[cell_start[a] ..)
    const int32_t *cell_pts;
    const double *xs;            // n x d: the features in binned order (xs[pp] = x[cell_pts[pp]])
    const int32_t *pt_cell;      // n: the linear cell of each point in binned order (pt_cell[pp] = cell of cell_pts[pp])
    const struct GatherPart *parts; // the gather's work list (grid method)
    const int32_t *part_first;   // per gather task, its first part (tasks + 1 entries)
    int64_t nparts;
};

// One wavefront's share of the grid gather: `count` consecutive points of task `task`'s union
// box, starting `off` points into its union row `row`.
struct GatherPart {
    int32_t task, row, off, count;
};

// ---- exact method -------------------------------------------------------------------

// R_i = sum_{j != i} w_ij V_j, one thread per row i, V and R n x KP.  The points j are split
// into gridDim.y chunks of `chunk` points, so that a few 10^4 rows still fill the chip;
// chunk y sums its points in increasing order into Rp[y], and k_gauss_chunks_sum adds the
// chunks in increasing order.  Every thread of a workgroup visits the same point j at the
// same time, so x_j and V_j are uniform: they are read with scalar loads and broadcast from
// scalar registers (no LDS staging).  D = d for d <= 3, else D = 0 (any d <= 8).  W: the
// type each weight is formed in — the graph's dtype (an FP32 graph forms its weights from the
// FP32 features with the FP32 exponential, as an FP32 CSR graph stores its values in FP32); the
// sums are FP64 either way.
template <int D, int KP, typename W>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_exact(GaussView gv, int64_t chunk,
                                                                   const double *__restrict__ V,
                                                                   double *__restrict__ Rp, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    constexpr int DM = D > 0 ? D : kGaussMaxDim;
    const int d = D > 0 ? D : gv.d;
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    const int64_t ii = i < gv.n ? i : gv.n - 1; // rows past n compute row n - 1 and store nothing
    const W *__restrict__ x;
    if constexpr (sizeof(W) == 4) x = gv.xf;
    else x = gv.x;
    W xi[DM];
#pragma unroll
    for (int q = 0; q < DM; ++q) xi[q] = q < d ? x[ii * d + q] : (W)0;
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    const W nscale = (W)(-gv.inv2s2);
    const int64_t jb = (int64_t)blockIdx.y * chunk, je = min(gv.n, jb + chunk);
#pragma unroll 2
    for (int64_t j = jb; j < je; ++j) {
        W r2 = (W)0;
#pragma unroll
        for (int q = 0; q < DM; ++q)
            if (q < d) {
                const W df = xi[q] - x[j * d + q];
                r2 = fma(df, df, r2);
            }
        double w = (double)exp(r2 * nscale);
        w = j == ii ? 0.0 : w;
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] = fma(w, V[j * KP + c], acc[c]);
    }
    if (i < gv.n) {
        double *out = Rp + ((int64_t)blockIdx.y * gv.n + i) * KP;
#pragma unroll
        for (int c = 0; c < KP; ++c) out[c] = acc[c];
    }
}

// R = sum over the chunks y = 0, 1, ... of Rp[y] (in that order); count = n KP.
static __global__ void k_gauss_chunks_sum(int64_t count, int32_t chunks, const double *__restrict__ Rp,
                                          double *__restrict__ R, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
        double acc = Rp[t];
        for (int32_t y = 1; y < chunks; ++y) acc += Rp[(int64_t)y * count + t];
        R[t] = acc;
    }
}

// ---- grid method --------------------------------------------------------------------

// coordinate of grid index a along dimension q
__device__ __forceinline__ double grid_coord(const GaussView &gv, int q, int a) { return gv.g0[q] + gv.h * (double)a; }

// Vs[pp] = V[cell_pts[pp]] (stride KP): the gather's right-hand side in binned order.
template <int KP>
static __global__ void __launch_bounds__(kRowBlock) k_grid_bin_v(GaussView gv, const double *__restrict__ V,
                                                                  double *__restrict__ Vs, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < gv.n * KP; t += (int64_t)gridDim.x * kRowBlock) {
        const int64_t pp = t / KP;
        Vs[t] = V[(int64_t)gv.cell_pts[pp] * KP + (t - pp * KP)];
    }
}

// G0[a] = sum over the points p binned in the cells b with a - kGridRW - 1 <= b <= a + kGridRW
// of g_tau(a - x_p) V_p (Vs: V in binned order, stride KP): the mirror of the grid points k_grid_interp visits
// around a point's cell, so that both truncate the window on the same point-grid pairs.
// The cells are taken in blocks of 64 (4 x 4 x 4, 8 x 8 or 64 of them by dimension), and the
// box of a cell is cut into its kGridWin slices along the last dimension L.  A task is a (block,
// last-dimension index bl) pair: the union of the block's boxes on that slice, whose rows (the
// cells with the same coordinates past dimension 0, consecutive in the linear order) hold
// consecutive ranges of the binned order.  Image colours crowd into a few clusters, so the
// tasks' point counts differ by orders of magnitude: each task is cut into parts of at most a
// fixed number of points (the work list, planned when the graph is made), one wavefront per part.
// All 64 lanes visit the same point at the same time, so the point's V (and, for d < 3, its
// features) are uniform (scalar loads, broadcast from scalar registers), and each lane adds the
// point only if it lies in its own cell's box; in 3-D the window is formed from per-dimension
// factors (gather_row_3d).  Part p writes its 64 lane sums to Tp[p] (64 x KP); k_grid_parts_sum
// adds, for each cell, its slices in increasing order and each slice's parts in increasing order.
template <int D> struct GridBlock {
    static constexpr int b0 = D == 1 ? 64 : D == 2 ? 8 : 4, b1 = D == 1 ? 1 : D == 2 ? 8 : 4, b2 = D == 3 ? 4 : 1;
    static constexpr int bl = D == 1 ? b0 : D == 2 ? b1 : b2; // block extent along the last dimension
    static constexpr int slices = bl + kGridWin - 1;          // last-dimension indices a block's boxes reach
};

// The geometry of gather task `task` for lane `lane` of its wavefront: the lane's cell (valid
// when inside the grid), its slice index y (mine: the cell's box reaches bl), the union of the
// block's boxes (ulo..uhi, the same for every lane) and the lane's own box (llo..lhi), both
// clipped to the grid, along L both the one index bl.  The host plans the parts with it, the
// gather kernel walks them with it.
struct GatherTask {
    int ai[kGridMaxDim], ulo[kGridMaxDim], uhi[kGridMaxDim], llo[kGridMaxDim], lhi[kGridMaxDim];
    int bl, y;
    int64_t a;
    bool valid, mine, in_grid;
};

template <int D>
__host__ __device__ inline GatherTask gather_task(const int32_t (&gdim)[kGridMaxDim], const int64_t (&gstride)[kGridMaxDim],
                                                  int64_t task, int lane)
{
    using B = GridBlock<D>;
    constexpr int L = D - 1;
    GatherTask g{};
    const int64_t blk = task / B::slices;
    const int ys = (int)(task - blk * B::slices);
    const int nb0 = (gdim[0] + B::b0 - 1) / B::b0, nb1 = (gdim[1] + B::b1 - 1) / B::b1;
    const int bk[kGridMaxDim] = {(int)(blk % nb0), (int)((blk / nb0) % nb1), (int)(blk / ((int64_t)nb0 * nb1))};
    const int bsz[kGridMaxDim] = {B::b0, B::b1, B::b2};
    const int off[kGridMaxDim] = {lane % B::b0, (lane / B::b0) % B::b1, lane / (B::b0 * B::b1)};
    g.bl = bk[L] * bsz[L] - kGridRW - 1 + ys;
    g.in_grid = g.bl >= 0 && g.bl < gdim[L];
    g.valid = true;
    g.a = 0;
    for (int q = 0; q < kGridMaxDim; ++q) {
        g.ai[q] = 0;
        g.ulo[q] = g.uhi[q] = g.llo[q] = g.lhi[q] = 0;
    }
    for (int q = 0; q < D; ++q) {
        g.ai[q] = bk[q] * bsz[q] + off[q];
        g.valid = g.valid && g.ai[q] < gdim[q];
        g.a += (int64_t)g.ai[q] * gstride[q];
        if (q == L) {
            g.ulo[q] = g.uhi[q] = g.llo[q] = g.lhi[q] = g.bl;
        } else {
            g.ulo[q] = bk[q] * bsz[q] - kGridRW - 1 > 0 ? bk[q] * bsz[q] - kGridRW - 1 : 0;
            g.uhi[q] = bk[q] * bsz[q] + bsz[q] - 1 + kGridRW < gdim[q] - 1 ? bk[q] * bsz[q] + bsz[q] - 1 + kGridRW
                                                                          : gdim[q] - 1;
            g.llo[q] = g.ai[q] - kGridRW - 1 > 0 ? g.ai[q] - kGridRW - 1 : 0;
            g.lhi[q] = g.ai[q] + kGridRW < gdim[q] - 1 ? g.ai[q] + kGridRW : gdim[q] - 1;
        }
    }
    g.y = g.bl - (g.ai[L] - kGridRW - 1);
    g.mine = g.valid && g.y >= 0 && g.y < kGridWin;
    return g;
}

// Union rows of a task: for d = 3 the rows b1 = ulo[1] .. uhi[1] of slice b2 = bl; otherwise the
// one row of the slice.  row_lin is the linear index of the row's cell 0.
template <int D> __host__ __device__ inline int gather_rows(const GatherTask &g) { return D == 3 ? g.uhi[1] - g.ulo[1] + 1 : 1; }

template <int D>
__host__ __device__ inline void gather_row(const GatherTask &g, const int64_t (&gstride)[kGridMaxDim], int r, int &b1, int &b2,
                                           int64_t &row_lin)
{
    b1 = D == 3 ? g.ulo[1] + r : D == 2 ? g.bl : 0;
    b2 = D == 3 ? g.bl : 0;
    row_lin = (int64_t)b1 * gstride[1] + (int64_t)b2 * gstride[2];
}

template <int D> __host__ __device__ inline int64_t grid_tasks(const int32_t (&gdim)[kGridMaxDim])
{
    using B = GridBlock<D>;
    return (int64_t)((gdim[0] + B::b0 - 1) / B::b0) * ((gdim[1] + B::b1 - 1) / B::b1) * ((gdim[2] + B::b2 - 1) / B::b2) *
           B::slices;
}

// acc += g_tau(a - x) v when `in` (the arithmetic of one point's term of the gather)
template <int D, int KP>
__device__ __forceinline__ void gather_term(const double (&ac)[kGridMaxDim], const double (&x)[D], const double (&v)[KP],
                                            double inv2t2, bool in, double (&acc)[KP])
{
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const double df = ac[q] - x[q];
        r2 = fma(df, df, r2);
    }
    const double w = exp(-r2 * inv2t2);
#pragma unroll
    for (int c = 0; c < KP; ++c) {
        const double t = fma(w, v[c], acc[c]);
        acc[c] = in ? t : acc[c];
    }
}

// The per-lane constants of the 3-D gather's factored window (see k_grid_gather).
struct GatherFactor {
    int u, q;       // the point of the batch and the dimension of the factor this lane forms
    double coord;   // the grid coordinate the factor is taken at
    int src[kGridMaxDim]; // per dimension, the lane (within a point's 12) holding this lane's factor
};

// One union row's points [P0, P1) for d = 3, in batches of 5: lanes 0..59 form the batch's 12
// window factors per point g_tau(c - x_q) (c the block's 4 coordinates per dimension), each
// lane's weight is the product of its three factors (read from the lanes that formed them), and
// a lane adds w V_p only for the points of its own box [p0, p1).  Every lane of the wavefront
// runs this (the shuffles read all lanes).
template <int KP>
__device__ __forceinline__ void gather_row_3d(const GaussView &gv, const double *__restrict__ Vs, const GatherFactor &fx,
                                              int32_t P0, int32_t P1, int32_t p0, int32_t p1, double (&acc)[KP])
{
    constexpr int NB = 5;
    const double *__restrict__ xs = gv.xs;
    // the batch's feature is loaded one batch ahead; its V rows and the factors' shuffles are
    // issued together (points past P1 repeat the last one, and add nothing)
    double xq = xs[(int64_t)min(P0 + fx.u, P1 - 1) * 3 + fx.q];
    for (int32_t pp = P0; pp < P1; pp += NB) {
        const double xn = xs[(int64_t)min(pp + NB + fx.u, P1 - 1) * 3 + fx.q];
        const double df = fx.coord - xq;
        const double f = exp(-df * df * gv.inv2t2);
        double vb[NB][KP];
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int c = 0; c < KP; ++c) vb[u][c] = Vs[(int64_t)min(pp + u, P1 - 1) * KP + c];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double f0 = __shfl(f, 12 * u + fx.src[0]);
            const double f1 = __shfl(f, 12 * u + fx.src[1]);
            const double f2 = __shfl(f, 12 * u + fx.src[2]);
            const double w = f0 * f1 * f2;
            const bool in = pp + u < P1 && pp + u >= p0 && pp + u < p1;
#pragma unroll
            for (int c = 0; c < KP; ++c) {
                const double t = fma(w, vb[u][c], acc[c]);
                acc[c] = in ? t : acc[c];
            }
        }
        xq = xn;
    }
}

template <int D, int KP>
static __global__ void __launch_bounds__(kRowBlock) k_grid_gather(GaussView gv, const double *__restrict__ Vs,
                                                                   double *__restrict__ Tp, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    const int64_t p = (int64_t)blockIdx.x * (kRowBlock / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    if (p >= gv.nparts) return;
    const GatherPart part = gv.parts[p];
    const int lane = (int)threadIdx.x & 63;
    const GatherTask g = gather_task<D>(gv.gdim, gv.gstride, part.task, lane);
    double ac[kGridMaxDim] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < D; ++q) ac[q] = grid_coord(gv, q, g.ai[q]);
    const double *__restrict__ xs = gv.xs;
    const int32_t *__restrict__ cs = gv.cell_start;
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    // d = 3: the window factors over the dimensions, and the block's 64 cells take only 4
    // coordinates per dimension: lane l < 60 forms factor (l % 12) / 4 (the dimension q), l % 4
    // (the block's q-th coordinate) of point l / 12 of a batch of 5
    GatherFactor fx{};
    if constexpr (D == 3) {
        const int offs[kGridMaxDim] = {lane % 4, (lane / 4) % 4, lane / 16};
        const int fq = (lane % 12) / 4, fo = lane % 4;
        fx.u = lane / 12;
        fx.q = fq;
        fx.coord = grid_coord(gv, fq, g.ai[fq] - offs[fq] + fo);
#pragma unroll
        for (int q = 0; q < 3; ++q) fx.src[q] = 4 * q + offs[q];
    }
    const int nrows = gather_rows<D>(g);
    int32_t left = part.count, skip = part.off;
    for (int r = part.row; r < nrows && left > 0; ++r) {
        int b1, b2;
        int64_t row;
        gather_row<D>(g, gv.gstride, r, b1, b2, row);
        const int32_t P0 = cs[row + g.ulo[0]] + skip;
        const int32_t P1 = (int32_t)min((int64_t)cs[row + g.uhi[0] + 1], (int64_t)P0 + left);
        skip = 0;
        if (P0 >= P1) continue;
        left -= P1 - P0;
        const bool on = g.mine && b1 >= g.llo[1] && b1 <= g.lhi[1] && b2 >= g.llo[2] && b2 <= g.lhi[2];
        const int32_t p0 = on ? cs[row + g.llo[0]] : 0, p1 = on ? cs[row + g.lhi[0] + 1] : 0;
        if constexpr (D == 3) {
            gather_row_3d<KP>(gv, Vs, fx, P0, P1, p0, p1, acc);
            continue;
        }
        // the points' data are loaded for batches of 4 points ahead of their use (every lane
        // computes every point's term; a lane keeps it only for the points of its own box)
        int32_t pp = P0;
        for (; pp + 4 <= P1; pp += 4) {
            double xb[4][D], vb[4][KP];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int q = 0; q < D; ++q) xb[u][q] = xs[(int64_t)(pp + u) * D + q];
#pragma unroll
                for (int c = 0; c < KP; ++c) vb[u][c] = Vs[(int64_t)(pp + u) * KP + c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) gather_term<D, KP>(ac, xb[u], vb[u], gv.inv2t2, pp + u >= p0 && pp + u < p1, acc);
        }
        for (; pp < P1; ++pp) {
            double xb[D], vb[KP];
#pragma unroll
            for (int q = 0; q < D; ++q) xb[q] = xs[(int64_t)pp * D + q];
#pragma unroll
            for (int c = 0; c < KP; ++c) vb[c] = Vs[(int64_t)pp * KP + c];
            gather_term<D, KP>(ac, xb, vb, gv.inv2t2, pp >= p0 && pp < p1, acc);
        }
    }
    double *__restrict__ out = Tp + (p * 64 + lane) * KP;
#pragma unroll
    for (int c = 0; c < KP; ++c) out[c] = acc[c];
}

// G0[a] = sum over the slices y = 0 .. kGridWin - 1 of cell a (in that order) of the parts of the
// slice's task (in order).  One thread per cell.
template <int D, int KP>
static __global__ void __launch_bounds__(kRowBlock) k_grid_parts_sum(GaussView gv, const double *__restrict__ Tp,
                                                                      double *__restrict__ G0, const Ctl *__restrict__ ctl)
{
    using B = GridBlock<D>;
    constexpr int L = D - 1;
    if (ctl && !ctl->active) return;
    const int64_t a = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (a >= gv.ncells) return;
    int ai[kGridMaxDim] = {0, 0, 0};
    int64_t rem = a;
#pragma unroll
    for (int q = D - 1; q >= 0; --q) {
        ai[q] = (int)(rem / gv.gstride[q]);
        rem -= (int64_t)ai[q] * gv.gstride[q];
    }
    const int bsz[kGridMaxDim] = {B::b0, B::b1, B::b2};
    const int nb0 = (gv.gdim[0] + B::b0 - 1) / B::b0, nb1 = (gv.gdim[1] + B::b1 - 1) / B::b1;
    const int bk[kGridMaxDim] = {ai[0] / B::b0, ai[1] / B::b1, ai[2] / B::b2};
    const int lane = ai[0] % B::b0 + B::b0 * (ai[1] % B::b1 + B::b1 * (ai[2] % B::b2));
    const int64_t blk = bk[0] + (int64_t)nb0 * (bk[1] + (int64_t)nb1 * bk[2]);
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    for (int y = 0; y < kGridWin; ++y) {
        const int ys = (ai[L] - kGridRW - 1 + y) - (bk[L] * bsz[L] - kGridRW - 1);
        const int64_t t = blk * B::slices + ys;
        for (int32_t q = gv.part_first[t]; q < gv.part_first[t + 1]; ++q)
#pragma unroll
            for (int c = 0; c < KP; ++c) acc[c] += Tp[((int64_t)q * 64 + lane) * KP + c];
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) G0[a * KP + c] = acc[c];
}

// out[a] = sum_{t = -kGridRC..kGridRC} g_s(t h) in[a + t e_axis] (zero past the grid), stored as
// OT.  One thread per cell.
template <int KP, typename OT>
static __global__ void __launch_bounds__(kRowBlock) k_grid_conv(GaussView gv, int axis, const double *__restrict__ in,
                                                                 OT *__restrict__ out, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    const int64_t a = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (a >= gv.ncells) return;
    const int64_t st = gv.gstride[axis];
    const int ai = (int)((a / st) % gv.gdim[axis]);
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    const int t0 = max(-kGridRC, -ai), t1 = min(kGridRC, gv.gdim[axis] - 1 - ai);
    for (int t = t0; t <= t1; ++t) {
        const double w = gv.ctap[t < 0 ? -t : t];
        const double *src = in + (a + (int64_t)t * st) * KP;
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] = fma(w, src[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < KP; ++c) out[a * KP + c] = (OT)acc[c];
}

// R_i = c^d sum over the grid points a with c_i - kGridRW <= a <= c_i + kGridRW + 1 (c_i the
// cell of x_i; inside the grid, which keeps kGridRW + 2 cells to spare) of g_tau(x_i - a)
// G1[a], minus V_i (the self term).  A workgroup takes 64 consecutive points of the binned
// order (neighbouring points read overlapping windows of G1) with kGridWin wavefronts:
// wavefront t sums, for each of the 64 points (one per lane), the window's slice at index t
// along the last dimension (the window factors over the dimensions: the weights along
// dimension 0 are formed once per lane, in registers, those along dimension 1 once per row),
// and the first wavefront adds the kGridWin slice sums in increasing order.  Splitting the
// window keeps the chip busy for images of a few 10^4 pixels.  The reads of G1 bound the kernel
// (L1 bandwidth): GT is the type G1 is stored in (FP32 for an FP32 graph, half the bytes; the
// sums stay FP64).
constexpr int kInterpThreads = 64 * kGridWin;

template <int D, int KP, typename GT>
static __global__ void __launch_bounds__(kInterpThreads) k_grid_interp(GaussView gv, const GT *__restrict__ G1,
                                                                        const double *__restrict__ V,
                                                                        double *__restrict__ R, const Ctl *__restrict__ ctl)
{
    constexpr int CW = KP < 4 ? KP : 4; // classes reduced through LDS per pass
    __shared__ double part[kGridWin][64][CW];
    if (ctl && !ctl->active) return;
    const int t = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int64_t pp = (int64_t)blockIdx.x * 64 + lane;
    const bool pt = pp < gv.n;
    double acc[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = 0.0;
    if (pt) {
        int ci[kGridMaxDim] = {0, 0, 0};
        double xi[kGridMaxDim] = {0.0, 0.0, 0.0};
        int64_t rem = gv.pt_cell[pp];
#pragma unroll
        for (int q = D - 1; q >= 0; --q) {
            ci[q] = (int)(rem / gv.gstride[q]);
            rem -= (int64_t)ci[q] * gv.gstride[q];
            xi[q] = gv.xs[pp * D + q];
        }
        // this wavefront's slice: index t along the last dimension
        const double dfl = xi[D - 1] - grid_coord(gv, D - 1, ci[D - 1] - kGridRW + t);
        const double wl = exp(-dfl * dfl * gv.inv2t2);
        if constexpr (D == 1) {
            const GT *__restrict__ src = G1 + (int64_t)(ci[0] - kGridRW + t) * KP;
#pragma unroll
            for (int c = 0; c < KP; ++c) acc[c] = fma(wl, (double)src[c], acc[c]);
        } else {
            double w0[kGridWin];
#pragma unroll
            for (int t0 = 0; t0 < kGridWin; ++t0) {
                const double df = xi[0] - grid_coord(gv, 0, ci[0] - kGridRW + t0);
                w0[t0] = exp(-df * df * gv.inv2t2);
            }
            constexpr int N1 = D >= 3 ? kGridWin : 1;
            for (int t1 = 0; t1 < N1; ++t1) {
                double w1 = wl;
                int64_t base = (int64_t)(ci[0] - kGridRW) + (int64_t)(ci[D - 1] - kGridRW + t) * gv.gstride[D - 1];
                if (D >= 3) {
                    const double df = xi[1] - grid_coord(gv, 1, ci[1] - kGridRW + t1);
                    w1 = wl * exp(-df * df * gv.inv2t2);
                    base += (int64_t)(ci[1] - kGridRW + t1) * gv.gstride[1];
                }
                const GT *__restrict__ src = G1 + base * KP;
#pragma unroll
                for (int t0 = 0; t0 < kGridWin; ++t0) {
                    const double w = w1 * w0[t0];
#pragma unroll
                    for (int c = 0; c < KP; ++c) acc[c] = fma(w, (double)src[t0 * KP + c], acc[c]);
                }
            }
        }
    }
    const int64_t i = pt ? gv.cell_pts[pp] : 0;
#pragma unroll
    for (int c0 = 0; c0 < KP; c0 += CW) {
        if (c0 > 0) __syncthreads(); // the previous pass has read part
#pragma unroll
        for (int c = 0; c < CW; ++c) part[t][lane][c] = acc[c0 + c];
        __syncthreads();
        if (t == 0 && pt)
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                double sum = 0.0;
                for (int u = 0; u < kGridWin; ++u) sum += part[u][lane][c];
                R[i * KP + c0 + c] = gv.cnorm * sum - V[i * KP + c0 + c];
            }
    }
}

// ---- the pieces of the iteration around R = W V ----------------------------------------

// V = D^{-1/2} U (stride KP, the padding zero), for P = L_s U and the objective.
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_scale_u(int64_t n, int32_t K, int32_t KP,
                                                                    const double *__restrict__ dinv,
                                                                    const T *__restrict__ U, double *__restrict__ V)
{
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * KP; t += (int64_t)gridDim.x * kRowBlock) {
        const int64_t i = t / KP;
        const int32_t c = (int32_t)(t - i * KP);
        V[t] = c < K ? dinv[i] * (double)U[i * K + c] : 0.0;
    }
}

// V = D^{-1/2} S_k (stride KP), the one-hot rows of the iteration's vertices, for its label pass.
static __global__ void __launch_bounds__(kRowBlock) k_gauss_scale_s(int64_t n, int32_t KP, const double *__restrict__ dinv,
                                                                    const uint8_t *__restrict__ s0,
                                                                    const uint8_t *__restrict__ s1,
                                                                    const Ctl *__restrict__ ctl, double *__restrict__ V)
{
    if (!ctl->active) return;
    const uint8_t *__restrict__ s = (ctl->k & 1) ? s1 : s0;
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * KP; t += (int64_t)gridDim.x * kRowBlock) {
        const int64_t i = t / KP;
        V[t] = (int32_t)(t - i * KP) == (int32_t)s[i] ? dinv[i] : 0.0;
    }
}

static __global__ void k_gauss_fill(int64_t n, double v, double *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = v;
}

// P = U - D^{-1/2} R (R = W D^{-1/2} U, stride KP), stored as PT.
template <typename T, typename PT>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_p(int64_t n, int32_t K, int32_t KP,
                                                              const double *__restrict__ dinv, const T *__restrict__ U,
                                                              const double *__restrict__ R, PT *__restrict__ P)
{
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kRowBlock) {
        const int64_t i = t / K;
        P[t] = (PT)((double)U[t] - dinv[i] * R[i * KP + (t - i * K)]);
    }
}

// Label pass of a Gaussian graph: Q_k = S_k - D^{-1/2} R with R = W D^{-1/2} S_k (stride KP),
// rounded to the graph's dtype; the per-row term Q_{i, s_i} summed per 256-row block; the
// finish of the iteration by the last block (finish_if_last).
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_label(GraphView<T> view, int32_t KP,
                                                                  const double *__restrict__ dinv,
                                                                  const double *__restrict__ R)
{
    const Ctl *__restrict__ ctl = view.ctl;
    const int tile = blockIdx.x;
    if (!ctl->active) return label_inactive(view, tile);
    const uint8_t *__restrict__ s = (ctl->k & 1) ? view.s1 : view.s0;
    const int32_t K = view.K;
    const int64_t i = (int64_t)tile * kRowBlock + threadIdx.x;
    double own = 0.0;
    if (i < view.n) {
        const int32_t si = (int32_t)s[i];
        const double di = dinv[i];
        for (int32_t c = 0; c < K; ++c) {
            const T q = (T)((c == si ? 1.0 : 0.0) - di * R[i * KP + c]);
            view.Q[i * K + c] = q;
            if (c == si) own = (double)q;
        }
    }
    double v[1] = {own};
    block_sum_store_strided<1, true>(v, view.lab_part + tile, view.nb_row);
    finish_if_last(view, view.row_part, view.nb_row, view.lab_part, view.nb_row);
}

// Terms of E(U) of a Gaussian graph from U and R = W D^{-1/2} U (stride KP; P = U - D^{-1/2}
// R): block sums of <u_i, P_i>, sum u(1-u), omega_i ||uhat_i - u_i||^2 at part[j * nb + tile].
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_energy(GraphView<T> view, int32_t KP,
                                                                   const double *__restrict__ dinv,
                                                                   const T *__restrict__ U, const double *__restrict__ R,
                                                                   double omega0, double *__restrict__ part)
{
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (i < view.n) {
        const int32_t y = view.lab[i];
        const double di = dinv[i];
        for (int32_t c = 0; c < view.K; ++c) {
            const double u = (double)U[i * view.K + c];
            const double p = u - di * R[i * KP + c];
            acc[0] += u * p;
            acc[1] += u * (1.0 - u);
            if (y >= 0) {
                const double e = (c == y ? 1.0 : 0.0) - u;
                acc[2] += omega0 * e * e;
            }
        }
    }
    block_sum_store_strided<3>(acc, part + blockIdx.x, view.nb_row);
}

// d_i^{-1/2} from R = W 1; a degree at or below `floor` makes node i isolated (d_i^{-1/2} = 0,
// its row of L_s the identity's).  The grid method takes floor = 1e-6: there the degree is
// the grid sum minus the self term 1, and about 1e-7 of it is the method's error.
static __global__ void k_gauss_dinv(int64_t n, double floor_, const double *__restrict__ R, double *__restrict__ dinv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dinv[i] = R[i] > floor_ ? 1.0 / sqrt(R[i]) : 0.0;
}

// The Gershgorin radius 1 + d_i^{-1/2} (W D^{-1/2} 1)_i of row i of L_s (R2 = W dinv).
static __global__ void k_gauss_rho(int64_t n, const double *__restrict__ dinv, const double *__restrict__ R2,
                                   double *__restrict__ rho)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rho[i] = 1.0 + dinv[i] * R2[i];
}

} // namespace gfw
