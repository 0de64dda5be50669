// ---------------------------------------------------------------------------------
// Fully connected Gaussian graphs (the image setting of Section 5.1): nodes are feature
// vectors x_i in R^d, w_ij = exp(-||x_i - x_j||^2 / (2 sigma^2)) for i != j (eq. of the
// Gaussian similarity in Section 1), no self-loops.  The n x n matrix is never formed: every
// product R = W V (V n x K) is summed from the features, by one of two methods.
//
//  * exact: R_i = sum_{j != i} w_ij V_j, the weights formed where they are used (FP64);
//    O(n^2 K), the reference operator and the right one for images of a few 10^4 pixels.
//  * grid (d <= 3): a fast summation in the spirit of the NFFT-based one the paper uses.
//    With unnormalised Gaussians g_w(r) = exp(-r^2 / (2 w^2)) and sigma^2 = 2 tau^2 + s^2,
//    the convolution g_tau * g_s * g_tau is (2 pi tau^2 s / sigma) g_sigma per dimension, so
//        w(x - y) = c^d sum_a sum_b g_tau(x - a) g_s(a - b) g_tau(b - y),
//    c = h^2 sigma / (2 pi tau^2 s), is exact in the limit of grid spacing h -> 0 (a, b grid
//    points).  The three factors are three passes: gather the points onto the grid with the
//    window g_tau (each grid cell sums the points binned in the cells around it, in a fixed
//    order: deterministic, no atomics), convolve the grid with g_s one axis at a time, and
//    interpolate back at every point with g_tau.  tau^2 = (1 - 1/sqrt 2) sigma^2 makes the
//    narrowest Gaussian summed on the grid as wide as it can be (0.414 sigma); h = 0.4 sigma
//    keeps the sampling error of every sum below 1e-9 (trapezoid rule on a Gaussian of width
//    w: about 2 exp(-2 pi^2 w^2 / h^2)); the windows stop at 6 widths (exp(-18) = 1.5e-8).
//    The self term (w_ii = 0) is removed by subtracting V_i (the sum gives it weight 1).
//  For both, L_s V = V - D^{-1/2} W D^{-1/2} V with the degrees d = W 1.
// ---------------------------------------------------------------------------------
#pragma once

#include "gfw_kernels.h"

namespace gfw {

constexpr int kGaussMaxDim = 8;   // feature dimensions of the exact method
constexpr int kGridMaxDim = 3;    // feature dimensions of the grid method
constexpr int kGaussTile = 128;   // points staged in LDS per step of the exact method

struct GaussView {
    int64_t n;
    int32_t d;
    double inv2s2;               // 1 / (2 sigma^2)
    const double *x;             // n x d features
    const double *dinv;          // d_i^{-1/2} (0 for an isolated node)
    // grid method
    int32_t gdim[kGridMaxDim];   // cells per dimension (1 past d)
    int64_t gstride[kGridMaxDim];// linear stride of each dimension
    int64_t ncells;
    double g0[kGridMaxDim];      // coordinate of cell 0 per dimension
    double h;                    // grid spacing
    double inv2t2, inv2s2g;      // 1 / (2 tau^2), 1 / (2 s^2)
    double cnorm;                // c^d
    int32_t rw, rc;              // half-widths in cells of the window and of the convolution
    const int32_t *cell_start;   // ncells + 1: the points of cell a are cell_pts[cell_start[a] ..)
    const int32_t *cell_pts;
    const int32_t *pt_cell;      // n: the linear cell of each point (the binning above, point-wise)
};

// ---- exact method -------------------------------------------------------------------

// R_i = sum_{j != i} w_ij V_j, one thread per row i.  The points j are split into gridDim.y
// chunks of `chunk` points (a multiple of kGaussTile), so that a few 10^4 rows still fill the
// chip; chunk y sums its points in increasing order, staged in LDS kGaussTile at a time, into
// Rp[y] (n x K).  k_gauss_chunks_sum adds the chunks in increasing order.  K <= KB.
template <int KB>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_exact(GaussView gv, int32_t K, int64_t chunk,
                                                                   const double *__restrict__ V, double *__restrict__ Rp,
                                                                   const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    __shared__ double lx[kGaussTile * kGaussMaxDim];
    __shared__ double lv[kGaussTile * KB];
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    const bool has = i < gv.n;
    const int d = gv.d;
    double xi[kGaussMaxDim];
#pragma unroll
    for (int q = 0; q < kGaussMaxDim; ++q) xi[q] = (has && q < d) ? gv.x[i * d + q] : 0.0;
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    const int64_t jb = (int64_t)blockIdx.y * chunk, je = min(gv.n, jb + chunk);
    for (int64_t j0 = jb; j0 < je; j0 += kGaussTile) {
        const int cnt = (int)min((int64_t)kGaussTile, je - j0);
        __syncthreads(); // the previous tile has been consumed
        for (int q = threadIdx.x; q < cnt * d; q += kRowBlock) lx[q] = gv.x[j0 * d + q];
        for (int q = threadIdx.x; q < cnt * K; q += kRowBlock) lv[(q / K) * KB + q % K] = V[j0 * K + q];
        __syncthreads();
        if (!has) continue;
        for (int t = 0; t < cnt; ++t) {
            if (j0 + t == i) continue;
            double r2 = 0.0;
#pragma unroll
            for (int q = 0; q < kGaussMaxDim; ++q)
                if (q < d) {
                    const double df = xi[q] - lx[t * d + q];
                    r2 += df * df;
                }
            const double w = exp(-r2 * gv.inv2s2);
#pragma unroll
            for (int c = 0; c < KB; ++c)
                if (c < K) acc[c] += w * lv[t * KB + c];
        }
    }
    if (has) {
        double *out = Rp + (int64_t)blockIdx.y * gv.n * K + i * K;
#pragma unroll
        for (int c = 0; c < KB; ++c)
            if (c < K) out[c] = acc[c];
    }
}

// R = sum over the chunks y = 0, 1, ... of Rp[y] (in that order); count = n K.
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

// G0[a] = sum over points p in the cells within rw of a (cells in increasing linear order,
// points in their binned order) of g_tau(a - x_p) V_p.  One thread per cell.
template <int KB>
static __global__ void __launch_bounds__(kRowBlock) k_grid_gather(GaussView gv, int32_t K, const double *__restrict__ V,
                                                                   double *__restrict__ G0, const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    const int64_t a = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (a >= gv.ncells) return;
    int ai[kGridMaxDim];
    double ac[kGridMaxDim];
    int64_t rem = a;
#pragma unroll
    for (int q = kGridMaxDim - 1; q >= 0; --q) {
        ai[q] = (int)(rem / gv.gstride[q]);
        rem -= (int64_t)ai[q] * gv.gstride[q];
        ac[q] = q < gv.d ? grid_coord(gv, q, ai[q]) : 0.0;
    }
    // the cells whose points the window of grid point a reaches: the mirror of the grid points
    // k_grid_interp visits around a point's cell (cell - rw .. cell + rw + 1), so that the gather
    // and the interpolation truncate the window on the same point-grid pairs
    int lo[kGridMaxDim], hi[kGridMaxDim];
#pragma unroll
    for (int q = 0; q < kGridMaxDim; ++q) {
        lo[q] = q < gv.d ? max(ai[q] - gv.rw - 1, 0) : 0;
        hi[q] = q < gv.d ? min(ai[q] + gv.rw, gv.gdim[q] - 1) : 0;
    }
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    for (int b2 = lo[2]; b2 <= hi[2]; ++b2)
        for (int b1 = lo[1]; b1 <= hi[1]; ++b1)
            for (int b0 = lo[0]; b0 <= hi[0]; ++b0) {
                const int64_t cb = (int64_t)b0 * gv.gstride[0] + (int64_t)b1 * gv.gstride[1] + (int64_t)b2 * gv.gstride[2];
                const int32_t p0 = gv.cell_start[cb], p1 = gv.cell_start[cb + 1];
                for (int32_t pp = p0; pp < p1; ++pp) {
                    const int32_t p = gv.cell_pts[pp];
                    double r2 = 0.0;
#pragma unroll
                    for (int q = 0; q < kGridMaxDim; ++q)
                        if (q < gv.d) {
                            const double df = ac[q] - gv.x[(int64_t)p * gv.d + q];
                            r2 += df * df;
                        }
                    const double w = exp(-r2 * gv.inv2t2);
#pragma unroll
                    for (int c = 0; c < KB; ++c)
                        if (c < K) acc[c] += w * V[(int64_t)p * K + c];
                }
            }
#pragma unroll
    for (int c = 0; c < KB; ++c)
        if (c < K) G0[a * K + c] = acc[c];
}

// out[a] = sum_{t = -rc..rc} g_s(t h) in[a + t e_axis] (zero past the grid).  One thread per cell.
template <int KB>
static __global__ void __launch_bounds__(kRowBlock) k_grid_conv(GaussView gv, int32_t K, int axis,
                                                                 const double *__restrict__ in, double *__restrict__ out,
                                                                 const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    const int64_t a = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (a >= gv.ncells) return;
    const int64_t st = gv.gstride[axis];
    const int ai = (int)((a / st) % gv.gdim[axis]);
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    const int t0 = max(-gv.rc, -ai), t1 = min(gv.rc, gv.gdim[axis] - 1 - ai);
    for (int t = t0; t <= t1; ++t) {
        const double dt = gv.h * (double)t;
        const double w = exp(-dt * dt * gv.inv2s2g);
        const double *src = in + (a + (int64_t)t * st) * K;
#pragma unroll
        for (int c = 0; c < KB; ++c)
            if (c < K) acc[c] += w * src[c];
    }
#pragma unroll
    for (int c = 0; c < KB; ++c)
        if (c < K) out[a * K + c] = acc[c];
}

// R_i = c^d sum over cells a within rw of x_i of g_tau(x_i - a) G1[a], minus V_i (the self
// term).  One thread per point.
template <int KB>
static __global__ void __launch_bounds__(kRowBlock) k_grid_interp(GaussView gv, int32_t K, const double *__restrict__ G1,
                                                                   const double *__restrict__ V, double *__restrict__ R,
                                                                   const Ctl *__restrict__ ctl)
{
    if (ctl && !ctl->active) return;
    const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
    if (i >= gv.n) return;
    double xi[kGridMaxDim];
    int lo[kGridMaxDim], hi[kGridMaxDim];
    int64_t rem = gv.pt_cell[i];
#pragma unroll
    for (int q = kGridMaxDim - 1; q >= 0; --q) {
        const int ci = (int)(rem / gv.gstride[q]);
        rem -= (int64_t)ci * gv.gstride[q];
        xi[q] = q < gv.d ? gv.x[i * gv.d + q] : 0.0;
        lo[q] = q < gv.d ? max(ci - gv.rw, 0) : 0;
        hi[q] = q < gv.d ? min(ci + gv.rw + 1, gv.gdim[q] - 1) : 0;
    }
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    for (int b2 = lo[2]; b2 <= hi[2]; ++b2)
        for (int b1 = lo[1]; b1 <= hi[1]; ++b1)
            for (int b0 = lo[0]; b0 <= hi[0]; ++b0) {
                const int bb[kGridMaxDim] = {b0, b1, b2};
                double r2 = 0.0;
#pragma unroll
                for (int q = 0; q < kGridMaxDim; ++q)
                    if (q < gv.d) {
                        const double df = xi[q] - grid_coord(gv, q, bb[q]);
                        r2 += df * df;
                    }
                const double w = exp(-r2 * gv.inv2t2);
                const double *src =
                    G1 + ((int64_t)b0 * gv.gstride[0] + (int64_t)b1 * gv.gstride[1] + (int64_t)b2 * gv.gstride[2]) * K;
#pragma unroll
                for (int c = 0; c < KB; ++c)
                    if (c < K) acc[c] += w * src[c];
            }
#pragma unroll
    for (int c = 0; c < KB; ++c)
        if (c < K) R[i * K + c] = gv.cnorm * acc[c] - V[i * K + c];
}

// ---- the pieces of the iteration around R = W V ----------------------------------------

// V = D^{-1/2} U, for P = L_s U and the objective.
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_scale_u(int64_t n, int32_t K, const double *__restrict__ dinv,
                                                                    const T *__restrict__ U, double *__restrict__ V)
{
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kRowBlock)
        V[t] = dinv[t / K] * (double)U[t];
}

// V = D^{-1/2} S_k, the one-hot rows of the iteration's vertices, for its label pass.
static __global__ void __launch_bounds__(kRowBlock) k_gauss_scale_s(int64_t n, int32_t K, const double *__restrict__ dinv,
                                                                    const uint8_t *__restrict__ s0,
                                                                    const uint8_t *__restrict__ s1,
                                                                    const Ctl *__restrict__ ctl, double *__restrict__ V)
{
    if (!ctl->active) return;
    const uint8_t *__restrict__ s = (ctl->k & 1) ? s1 : s0;
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kRowBlock) {
        const int64_t i = t / K;
        V[t] = (int32_t)(t - i * K) == (int32_t)s[i] ? dinv[i] : 0.0;
    }
}

static __global__ void k_gauss_fill(int64_t n, double v, double *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = v;
}

// P = U - D^{-1/2} R (R = W D^{-1/2} U), stored as PT.
template <typename T, typename PT>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_p(int64_t n, int32_t K, const double *__restrict__ dinv,
                                                              const T *__restrict__ U, const double *__restrict__ R,
                                                              PT *__restrict__ P)
{
    for (int64_t t = (int64_t)blockIdx.x * kRowBlock + threadIdx.x; t < n * K; t += (int64_t)gridDim.x * kRowBlock)
        P[t] = (PT)((double)U[t] - dinv[t / K] * R[t]);
}

// Label pass of a Gaussian graph: Q_k = S_k - D^{-1/2} R with R = W D^{-1/2} S_k, rounded to
// the graph's dtype; the per-row term Q_{i, s_i} summed per 256-row block; the finish of the
// iteration by the last block (finish_if_last).
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_label(GraphView<T> view, const double *__restrict__ dinv,
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
            const T q = (T)((c == si ? 1.0 : 0.0) - di * R[i * K + c]);
            view.Q[i * K + c] = q;
            if (c == si) own = (double)q;
        }
    }
    double v[1] = {own};
    block_sum_store_strided<1, true>(v, view.lab_part + tile, view.nb_row);
    finish_if_last(view, view.row_part, view.nb_row, view.lab_part, view.nb_row);
}

// Terms of E(U) of a Gaussian graph from U and R = W D^{-1/2} U (P = U - D^{-1/2} R): block
// sums of <u_i, P_i>, sum u(1-u), omega_i ||uhat_i - u_i||^2 at part[j * nb + tile].
template <typename T>
static __global__ void __launch_bounds__(kRowBlock) k_gauss_energy(GraphView<T> view, const double *__restrict__ dinv,
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
            const double p = u - di * R[i * view.K + c];
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
// the grid sum minus the self term 1, and a few 1e-8 of it are the method's error.
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
