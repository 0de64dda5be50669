// Fully connected Gaussian graphs: creation (features, degrees, the grid of the fast method)
// and the products with L_s that the iteration, the objective and gfw_spmm make on them.
// The kernels are in gfw_kernels_gauss.h; the iteration's row kernel is the one of every
// graph (it reads only U, P and Q).

#include "gfw_internal.h"
#include "gfw_kernels_gauss.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace gfw {

struct GaussGraph {
    int method = GFW_GAUSS_EXACT;
    GaussView view{};
    int32_t kp = 4;              // padded row stride of V, R and the grids: 4, 8 or 16
    int32_t chunks = 1;          // exact method: chunks of the points summed apart
    int64_t chunk = 0;           // points per chunk
    double *x = nullptr;         // n x d features (FP64)
    float *xf = nullptr;         // the same in FP32, for an FP32 graph's exact sums
    double *dinv = nullptr;      // n
    int32_t *cell_start = nullptr, *cell_pts = nullptr, *pt_cell = nullptr;
    double *V = nullptr, *R = nullptr; // n x kp
    double *Rp = nullptr;        // chunks x n x kp (exact method, chunks > 1)
    double *G0 = nullptr, *G1 = nullptr; // ncells x kp (grid method)
    float *G1f = nullptr;        // the convolved grid in FP32 (grid method, FP32 graph)
    double *Tp = nullptr;        // nparts x 64 x kp: the gather's part sums (grid method)
    GatherPart *parts = nullptr; // the gather's work list
    int32_t *part_first = nullptr; // per gather task, its first part
    double *xs = nullptr, *Vs = nullptr; // n x d features and n x kp V in binned order (grid method)
};

int gauss_method(const GaussGraph *gg) { return gg->method; }

void gauss_free(GaussGraph *gg)
{
    if (!gg) return;
    dfree(gg->x);
    dfree(gg->xf);
    dfree(gg->dinv);
    dfree(gg->cell_start);
    dfree(gg->cell_pts);
    dfree(gg->pt_cell);
    dfree(gg->V);
    dfree(gg->R);
    dfree(gg->Rp);
    dfree(gg->G0);
    dfree(gg->G1);
    dfree(gg->Tp);
    dfree(gg->G1f);
    dfree(gg->parts);
    dfree(gg->part_first);
    dfree(gg->xs);
    dfree(gg->Vs);
    delete gg;
}

template <int D, int KP>
static void apply_exact(const GaussGraph &gg, const double *V, double *R, const Ctl *ctl, hipStream_t st)
{
    const GaussView &v = gg.view;
    double *out = gg.chunks > 1 ? gg.Rp : R;
    const dim3 grid((unsigned)cdiv(v.n, kRowBlock), gg.chunks);
    if (gg.xf) k_gauss_exact<D, KP, float><<<grid, kRowBlock, 0, st>>>(v, gg.chunk, V, out, ctl);
    else k_gauss_exact<D, KP, double><<<grid, kRowBlock, 0, st>>>(v, gg.chunk, V, out, ctl);
    if (gg.chunks > 1)
        k_gauss_chunks_sum<<<grid_for(v.n * KP, 256, 4096), 256, 0, st>>>(v.n * KP, gg.chunks, gg.Rp, R, ctl);
}

template <int D, int KP>
static void apply_grid(const GaussGraph &gg, const double *V, double *R, const Ctl *ctl, hipStream_t st)
{
    const GaussView &v = gg.view;
    const unsigned nc = (unsigned)cdiv(v.ncells, kRowBlock);
    k_grid_bin_v<KP><<<grid_for(v.n * KP, kRowBlock, 4096), kRowBlock, 0, st>>>(v, V, gg.Vs, ctl);
    if (v.nparts > 0) // one wavefront per part
        k_grid_gather<D, KP><<<(unsigned)cdiv(v.nparts, kRowBlock / 64), kRowBlock, 0, st>>>(v, gg.Vs, gg.Tp, ctl);
    k_grid_parts_sum<D, KP><<<nc, kRowBlock, 0, st>>>(v, gg.Tp, gg.G0, ctl);
    // the convolution one axis at a time; an FP32 graph's last pass stores the grid in FP32
    const double *in = gg.G0;
    double *out = gg.G1;
    for (int q = 0; q < D; ++q) {
        if (q == D - 1 && gg.G1f) {
            k_grid_conv<KP, float><<<nc, kRowBlock, 0, st>>>(v, q, in, gg.G1f, ctl);
            break;
        }
        k_grid_conv<KP, double><<<nc, kRowBlock, 0, st>>>(v, q, in, out, ctl);
        double *done = out;
        out = const_cast<double *>(in);
        in = done;
    }
    const unsigned ni = (unsigned)cdiv(v.n, 64);
    if (gg.G1f) k_grid_interp<D, KP, float><<<ni, kInterpThreads, 0, st>>>(v, gg.G1f, V, R, ctl);
    else k_grid_interp<D, KP, double><<<ni, kInterpThreads, 0, st>>>(v, in, V, R, ctl);
}

template <int KP>
static void apply_w_kp(const GaussGraph &gg, const double *V, double *R, const Ctl *ctl, hipStream_t st)
{
    const GaussView &v = gg.view;
    if (gg.method == GFW_GAUSS_EXACT) {
        switch (v.d) {
        case 1: apply_exact<1, KP>(gg, V, R, ctl, st); break;
        case 2: apply_exact<2, KP>(gg, V, R, ctl, st); break;
        case 3: apply_exact<3, KP>(gg, V, R, ctl, st); break;
        default: apply_exact<0, KP>(gg, V, R, ctl, st); break;
        }
        return;
    }
    switch (v.d) {
    case 1: apply_grid<1, KP>(gg, V, R, ctl, st); break;
    case 2: apply_grid<2, KP>(gg, V, R, ctl, st); break;
    default: apply_grid<3, KP>(gg, V, R, ctl, st); break;
    }
}

// R = W V for V n x KP (FP64, KP = 1 or the graph's padded class count).  ctl: the launches
// do nothing once the solve has stopped (null: they always run).
static void apply_w(const GaussGraph &gg, int32_t KP, const double *V, double *R, const Ctl *ctl, hipStream_t st)
{
    switch (KP) {
    case 1: apply_w_kp<1>(gg, V, R, ctl, st); break;
    case 4: apply_w_kp<4>(gg, V, R, ctl, st); break;
    case 8: apply_w_kp<8>(gg, V, R, ctl, st); break;
    default: apply_w_kp<16>(gg, V, R, ctl, st); break;
    }
}

template <typename T, typename PT>
void gauss_spmm(const gfw_graph_s *g, const T *U, PT *P, hipStream_t st)
{
    const GaussGraph &gg = *g->gauss;
    const int32_t KP = gg.kp;
    k_gauss_scale_u<T><<<grid_for(g->n * KP, kRowBlock, 4096), kRowBlock, 0, st>>>(g->n, g->K, KP, gg.dinv, U, gg.V);
    apply_w(gg, KP, gg.V, gg.R, nullptr, st);
    k_gauss_p<T, PT><<<grid_for(g->n * g->K, kRowBlock, 4096), kRowBlock, 0, st>>>(g->n, g->K, KP, gg.dinv, U, gg.R, P);
}

template <typename T>
void gauss_label(const gfw_graph_s *g, hipStream_t st)
{
    const GaussGraph &gg = *g->gauss;
    const Workspace &w = g->ws;
    const int32_t KP = gg.kp;
    k_gauss_scale_s<<<grid_for(g->n * KP, kRowBlock, 4096), kRowBlock, 0, st>>>(g->n, KP, gg.dinv, w.s0, w.s1, w.ctl,
                                                                                 gg.V);
    apply_w(gg, KP, gg.V, gg.R, w.ctl, st);
    k_gauss_label<T><<<g->shape.nb_row, kRowBlock, 0, st>>>(make_view<T>(g), KP, gg.dinv, gg.R);
}

template <typename T>
int gauss_energy(const gfw_graph_s *g, const T *U, double omega0, double *part, hipStream_t st)
{
    const GaussGraph &gg = *g->gauss;
    const int32_t KP = gg.kp;
    k_gauss_scale_u<T><<<grid_for(g->n * KP, kRowBlock, 4096), kRowBlock, 0, st>>>(g->n, g->K, KP, gg.dinv, U, gg.V);
    apply_w(gg, KP, gg.V, gg.R, nullptr, st);
    k_gauss_energy<T><<<g->shape.nb_row, kRowBlock, 0, st>>>(make_view<T>(g), KP, gg.dinv, U, gg.R, omega0, part);
    return g->shape.nb_row;
}

template void gauss_spmm<float, float>(const gfw_graph_s *, const float *, float *, hipStream_t);
template void gauss_spmm<float, double>(const gfw_graph_s *, const float *, double *, hipStream_t);
template void gauss_spmm<double, double>(const gfw_graph_s *, const double *, double *, hipStream_t);
template void gauss_label<float>(const gfw_graph_s *, hipStream_t);
template void gauss_label<double>(const gfw_graph_s *, hipStream_t);
template int gauss_energy<float>(const gfw_graph_s *, const float *, double, double *, hipStream_t);
template int gauss_energy<double>(const gfw_graph_s *, const double *, double, double *, hipStream_t);

// ---- set-up ----------------------------------------------------------------------------

namespace {

// Grid geometry of the fast method for features xh (n x d, d <= 3) and width sigma: the
// widths of the window and of the convolution (sigma^2 = 2 tau^2 + s^2), the spacing, the
// convolution's taps, cells covering every point with kGridRW + 2 cells to spare on each side,
// and the work estimate of one product (point and cell visits by a thread).
struct GridPlan {
    GaussView v{};
    double work = 0.0;
};

GridPlan plan_grid(const std::vector<double> &xh, int64_t n, int d, double sigma)
{
    GridPlan gp;
    GaussView &v = gp.v;
    const double tau2 = (1.0 - 1.0 / std::sqrt(2.0)) * sigma * sigma;
    const double s2 = sigma * sigma - 2.0 * tau2;
    const double s = std::sqrt(s2);
    v.h = kGridSpacing * sigma;
    v.inv2t2 = 1.0 / (2.0 * tau2);
    v.inv2s2g = 1.0 / (2.0 * s2);
    const double c = v.h * v.h * sigma / (2.0 * M_PI * tau2 * s);
    v.cnorm = std::pow(c, d);
    for (int t = 0; t <= kGridRC; ++t) {
        const double dt = v.h * t;
        v.ctap[t] = std::exp(-dt * dt * v.inv2s2g);
    }
    for (int q = 0; q < kGridMaxDim; ++q) {
        if (q < d) {
            double lo = xh[(size_t)q], hi = lo;
            for (int64_t i = 1; i < n; ++i) {
                lo = std::min(lo, xh[(size_t)(i * d + q)]);
                hi = std::max(hi, xh[(size_t)(i * d + q)]);
            }
            v.g0[q] = lo - (kGridRW + 2) * v.h;
            const double span = std::floor((hi - v.g0[q]) / v.h) + kGridRW + 4;
            v.gdim[q] = span < 2e9 ? (int32_t)span : INT32_MAX;
        } else {
            v.g0[q] = 0.0;
            v.gdim[q] = 1;
        }
    }
    v.gstride[0] = 1;
    v.gstride[1] = v.gdim[0];
    v.gstride[2] = (int64_t)v.gdim[0] * v.gdim[1];
    const double cells = (double)v.gdim[0] * (double)v.gdim[1] * (double)v.gdim[2];
    v.ncells = cells < 9e18 ? (int64_t)cells : INT64_MAX;
    const double win = std::pow((double)kGridWin, d);
    gp.work = cells * win / kGridWin + 2.0 * (double)n * win + cells * d * (2.0 * kGridRC + 1.0);
    return gp;
}

// The grid gather's work list: every task's union points (its rows in order, each row's points
// in binned order) cut into parts of at most `cap` points; first[t] is task t's first part.
// cap is at least 256 and large enough that the parts number about 16 wavefronts per SIMD.
template <int D>
void plan_gather(const GaussView &v, const std::vector<int32_t> &start, int num_cu, std::vector<GatherPart> &parts,
                 std::vector<int32_t> &first)
{
    const int64_t tasks = grid_tasks<D>(v.gdim);
    int64_t total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t cap = std::max<int64_t>(256, total / (16LL * 4 * std::max(num_cu, 1)));
        if (pass == 1) first.assign((size_t)tasks + 1, 0);
        for (int64_t t = 0; t < tasks; ++t) {
            if (pass == 1) first[(size_t)t] = (int32_t)parts.size();
            const GatherTask g = gather_task<D>(v.gdim, v.gstride, t, 0);
            if (!g.in_grid) continue;
            GatherPart cur{(int32_t)t, 0, 0, 0};
            bool open = false;
            for (int r = 0; r < gather_rows<D>(g); ++r) {
                int b1, b2;
                int64_t row;
                gather_row<D>(g, v.gstride, r, b1, b2, row);
                int64_t c = (int64_t)start[(size_t)(row + g.uhi[0] + 1)] - start[(size_t)(row + g.ulo[0])];
                if (pass == 0) {
                    total += c;
                    continue;
                }
                int64_t off = 0;
                while (c > 0) {
                    if (!open) {
                        cur = GatherPart{(int32_t)t, r, (int32_t)off, 0};
                        open = true;
                    }
                    const int64_t take = std::min(c, cap - cur.count);
                    cur.count += (int32_t)take;
                    c -= take;
                    off += take;
                    if (cur.count == cap) {
                        parts.push_back(cur);
                        open = false;
                    }
                }
            }
            if (open) parts.push_back(cur);
        }
        if (pass == 1) first[(size_t)tasks] = (int32_t)parts.size();
    }
}

template <typename T>
void features_to_f64(const void *src, int64_t count, std::vector<double> &out)
{
    const T *p = (const T *)src;
    for (int64_t t = 0; t < count; ++t) out[(size_t)t] = (double)p[t];
}

} // namespace

// The largest grid the fast method takes: ncells * KP doubles per grid buffer (the gather's
// slices take kGridWin such buffers).
constexpr int64_t kGridMaxElems = int64_t(1) << 26;

gfw_status_t gauss_graph_create(gfw_context_s *ctx, const gfw_gaussian_problem_t *p, gfw_graph_s **out, hipStream_t st)
{
    if (!p) return fail(GFW_E_INVALID_ARG, "problem is NULL");
    if (p->n < 1 || p->n > INT32_MAX) return fail(GFW_E_INVALID_ARG, "n = %lld out of [1, 2^31)", (long long)p->n);
    if (p->K < 2) return fail(GFW_E_INVALID_ARG, "K must be >= 2");
    if (p->K > 16) return fail(GFW_E_UNSUPPORTED, "Gaussian graphs take K <= 16 (K = %d)", p->K);
    if (p->dtype != GFW_F32 && p->dtype != GFW_F64) return fail(GFW_E_INVALID_ARG, "bad dtype");
    if (p->location != GFW_HOST && p->location != GFW_DEVICE) return fail(GFW_E_INVALID_ARG, "bad location");
    if (!p->features) return fail(GFW_E_INVALID_ARG, "features is NULL");
    if (!(p->sigma > 0.0) || !std::isfinite(p->sigma)) return fail(GFW_E_INVALID_ARG, "sigma must be > 0 and finite");
    if (p->method < GFW_GAUSS_AUTO || p->method > GFW_GAUSS_GRID) return fail(GFW_E_INVALID_ARG, "bad method");
    if (p->d < 1) return fail(GFW_E_INVALID_ARG, "d must be >= 1");
    if (p->n_labelled < 0 || p->n_labelled > p->n) return fail(GFW_E_LABELS, "n_labelled out of [0, n]");
    if (p->n_labelled > 0 && (!p->labelled_idx || !p->labels)) return fail(GFW_E_INVALID_ARG, "label arrays are NULL");
    const int d = p->d;
    if (p->method == GFW_GAUSS_GRID && d > kGridMaxDim)
        return fail(GFW_E_UNSUPPORTED, "the grid method takes d <= %d (d = %d)", kGridMaxDim, d);
    if (p->method == GFW_GAUSS_EXACT && d > kGaussMaxDim)
        return fail(GFW_E_UNSUPPORTED, "the exact method takes d <= %d (d = %d)", kGaussMaxDim, d);
    if (d > kGaussMaxDim) return fail(GFW_E_UNSUPPORTED, "feature dimension %d above %d", d, kGaussMaxDim);
    GFW_HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = p->n;
    const int32_t K = p->K;

    // the features, on the host in FP64 (the grid is planned and the points binned there)
    const size_t vs = dsize(p->dtype);
    std::vector<double> xh((size_t)(n * d));
    {
        std::vector<unsigned char> raw;
        const void *src = p->features;
        if (p->location == GFW_DEVICE) {
            raw.resize(vs * (size_t)(n * d));
            GFW_HIP_TRY(hipMemcpyAsync(raw.data(), p->features, raw.size(), hipMemcpyDeviceToHost, st));
            GFW_HIP_TRY(hipStreamSynchronize(st));
            src = raw.data();
        }
        if (p->dtype == GFW_F32) features_to_f64<float>(src, n * d, xh);
        else features_to_f64<double>(src, n * d, xh);
    }
    for (double v : xh)
        if (!std::isfinite(v)) return fail(GFW_E_GRAPH, "a feature is not finite");

    // method: exact, grid, or the one of smaller modelled time.  Rates measured on gfx950 at K <= 4
    // (both methods scale alike with KP): the grid about 1.8 ps per unit of its work estimate plus
    // about 20 us of fixed launches; the exact sums 0.8 ps per pair with FP32 weights, 1.3 ps with
    // FP64 ones.
    int method = p->method;
    GridPlan gp;
    if (method != GFW_GAUSS_EXACT && d <= kGridMaxDim) gp = plan_grid(xh, n, d, p->sigma);
    const int32_t KP = K <= 4 ? 4 : K <= 8 ? 8 : 16;
    const bool grid_fits = d <= kGridMaxDim && gp.v.ncells <= kGridMaxElems / KP;
    if (method == GFW_GAUSS_GRID && !grid_fits)
        return fail(GFW_E_UNSUPPORTED, "the grid for sigma = %g over these features has %lld cells (at most %lld for K "
                    "= %d); use the exact method or a larger sigma", p->sigma, (long long)gp.v.ncells,
                    (long long)(kGridMaxElems / KP), K);
    if (method == GFW_GAUSS_AUTO) {
        const double grid_ps = 1.8 * gp.work + 2e7;
        const double exact_ps = (p->dtype == GFW_F32 ? 0.8 : 1.3) * (double)n * (double)n;
        method = (grid_fits && grid_ps < exact_ps) ? GFW_GAUSS_GRID : GFW_GAUSS_EXACT;
    }

    gfw_graph_s *g = new (std::nothrow) gfw_graph_s();
    if (!g) return fail(GFW_E_NOMEM, "host allocation failed");
    struct Guard {
        gfw_graph_s *g;
        ~Guard() { if (g) free_graph(g); }
    } guard{g};
    g->ctx = ctx;
    g->n = n;
    g->nnz = 0; // no stored entries
    g->K = K;
    g->dtype = p->dtype;
    g->kind = GFW_GRAPH_W;
    g->n_labelled = p->n_labelled;
    g->diag_one = 1;
    g->label_path = 0;
    g->gauss = new (std::nothrow) GaussGraph();
    if (!g->gauss) return fail(GFW_E_NOMEM, "host allocation failed");
    GaussGraph &gg = *g->gauss;
    gg.method = method;
    gg.kp = KP;
    size_t bytes = 0;
    auto dalloc = [&](void **ptr, size_t b) -> gfw_status_t {
        hipError_t e = hipMalloc(ptr, std::max<size_t>(b, 16));
        if (e != hipSuccess) return fail(GFW_E_NOMEM, "device allocation of %zu bytes failed", b);
        bytes += b;
        return GFW_OK;
    };
    gfw_status_t s;
    const size_t nK = (size_t)n * KP;
    if ((s = dalloc((void **)&g->lab, 4 * (size_t)n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&gg.x, 8 * xh.size())) != GFW_OK) return s;
    if ((s = dalloc((void **)&gg.dinv, 8 * (size_t)n)) != GFW_OK) return s;
    if ((s = dalloc((void **)&gg.V, 8 * nK)) != GFW_OK) return s;
    if ((s = dalloc((void **)&gg.R, 8 * nK)) != GFW_OK) return s;
    GFW_HIP_TRY(hipMemcpyAsync(gg.x, xh.data(), 8 * xh.size(), hipMemcpyHostToDevice, st));
    std::vector<float> xfh;
    if (method == GFW_GAUSS_EXACT && p->dtype == GFW_F32) {
        // the FP32 features the caller gave (an FP32 graph forms its weights in FP32)
        xfh.resize(xh.size());
        for (size_t t = 0; t < xh.size(); ++t) xfh[t] = (float)xh[t];
        if ((s = dalloc((void **)&gg.xf, 4 * xfh.size())) != GFW_OK) return s;
        GFW_HIP_TRY(hipMemcpyAsync(gg.xf, xfh.data(), 4 * xfh.size(), hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipStreamSynchronize(st)); // before xfh can go out of scope
    }

    GaussView &v = gg.view;
    if (method == GFW_GAUSS_GRID) {
        v = gp.v;
        // bin the points: counting sort by linear cell, points in increasing index per cell
        std::vector<int32_t> pc((size_t)n), start((size_t)v.ncells + 1, 0), pts((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            int64_t lin = 0;
            for (int q = 0; q < d; ++q) {
                const int cq = (int)std::floor((xh[(size_t)(i * d + q)] - v.g0[q]) / v.h);
                // every point's window lies inside the grid (the interpolation does not clamp)
                if (cq - kGridRW < 0 || cq + kGridRW + 1 > v.gdim[q] - 1)
                    return fail(GFW_E_HIP, "internal: point %lld binned outside the grid", (long long)i);
                lin += (int64_t)cq * v.gstride[q];
            }
            pc[(size_t)i] = (int32_t)lin;
            ++start[(size_t)lin + 1];
        }
        for (int64_t a = 0; a < v.ncells; ++a) start[(size_t)a + 1] += start[(size_t)a];
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) pts[(size_t)fill[(size_t)pc[(size_t)i]]++] = (int32_t)i;
        if ((s = dalloc((void **)&gg.cell_start, 4 * start.size())) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.cell_pts, 4 * (size_t)n)) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.pt_cell, 4 * (size_t)n)) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.G0, 8 * (size_t)v.ncells * KP)) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.G1, 8 * (size_t)v.ncells * KP)) != GFW_OK) return s;
        if (p->dtype == GFW_F32 && (s = dalloc((void **)&gg.G1f, 4 * (size_t)v.ncells * KP)) != GFW_OK) return s;
        std::vector<GatherPart> parts;
        std::vector<int32_t> first;
        if (d == 1) plan_gather<1>(v, start, ctx->num_cu, parts, first);
        else if (d == 2) plan_gather<2>(v, start, ctx->num_cu, parts, first);
        else plan_gather<3>(v, start, ctx->num_cu, parts, first);
        v.nparts = (int64_t)parts.size();
        if ((s = dalloc((void **)&gg.parts, sizeof(GatherPart) * parts.size())) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.part_first, 4 * first.size())) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.Tp, 8 * (size_t)v.nparts * 64 * KP)) != GFW_OK) return s;
        GFW_HIP_TRY(hipMemcpyAsync(gg.parts, parts.data(), sizeof(GatherPart) * parts.size(), hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipMemcpyAsync(gg.part_first, first.data(), 4 * first.size(), hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipStreamSynchronize(st)); // parts and first go out of scope
        if ((s = dalloc((void **)&gg.xs, 8 * xh.size())) != GFW_OK) return s;
        if ((s = dalloc((void **)&gg.Vs, 8 * nK)) != GFW_OK) return s;
        std::vector<double> xsh(xh.size());
        for (int64_t pp = 0; pp < n; ++pp)
            for (int q = 0; q < d; ++q) xsh[(size_t)(pp * d + q)] = xh[(size_t)((int64_t)pts[(size_t)pp] * d + q)];
        GFW_HIP_TRY(hipMemcpyAsync(gg.xs, xsh.data(), 8 * xsh.size(), hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipStreamSynchronize(st));
        GFW_HIP_TRY(hipMemcpyAsync(gg.cell_start, start.data(), 4 * start.size(), hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipMemcpyAsync(gg.cell_pts, pts.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        // the points' cells in binned order
        std::vector<int32_t> pcb((size_t)n);
        for (int64_t pp = 0; pp < n; ++pp) pcb[(size_t)pp] = pc[(size_t)pts[(size_t)pp]];
        GFW_HIP_TRY(hipMemcpyAsync(gg.pt_cell, pcb.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
        GFW_HIP_TRY(hipStreamSynchronize(st)); // the host vectors go out of scope
    } else {
        // chunks of the points summed apart: about 8 waves per SIMD over the rows, each chunk
        // at least 128 points
        const int64_t row_waves = cdiv(n, 64);
        const int64_t want = cdiv(8LL * 4 * std::max(ctx->num_cu, 1), row_waves);
        const int64_t chunks = std::min<int64_t>(std::max<int64_t>(want, 1), 64);
        gg.chunk = std::max<int64_t>(cdiv(n, chunks), 128);
        gg.chunks = (int32_t)cdiv(n, gg.chunk);
        if (gg.chunks > 1 && (s = dalloc((void **)&gg.Rp, 8 * nK * (size_t)gg.chunks)) != GFW_OK) return s;
    }
    v.n = n;
    v.d = d;
    v.inv2s2 = 1.0 / (2.0 * p->sigma * p->sigma);
    v.x = gg.x;
    v.xf = gg.xf;
    v.dinv = gg.dinv;
    v.cell_start = gg.cell_start;
    v.cell_pts = gg.cell_pts;
    v.xs = gg.xs;
    v.pt_cell = gg.pt_cell;
    v.parts = gg.parts;
    v.part_first = gg.part_first;

    // labels (checked on the device: range, repeats, classes)
    unsigned int *flags = nullptr;
    if ((s = dalloc((void **)&flags, sizeof(unsigned int))) != GFW_OK) return s;
    bytes -= sizeof(unsigned int);
    const unsigned int zero = 0;
    GFW_HIP_TRY(hipMemcpyAsync(flags, &zero, sizeof(zero), hipMemcpyHostToDevice, st));
    k_fill_i32<<<grid_for(n, 256), 256, 0, st>>>(n, g->lab, -1);
    int32_t *ti = nullptr, *tl = nullptr;
    if (p->n_labelled) {
        const int32_t *di = p->labelled_idx, *dl = p->labels;
        if (p->location == GFW_HOST) {
            if ((s = dalloc((void **)&ti, 4 * (size_t)p->n_labelled)) != GFW_OK) { dfree(flags); return s; }
            if ((s = dalloc((void **)&tl, 4 * (size_t)p->n_labelled)) != GFW_OK) { dfree(flags); dfree(ti); return s; }
            bytes -= 8 * (size_t)p->n_labelled;
            GFW_HIP_TRY(hipMemcpyAsync(ti, p->labelled_idx, 4 * p->n_labelled, hipMemcpyHostToDevice, st));
            GFW_HIP_TRY(hipMemcpyAsync(tl, p->labels, 4 * p->n_labelled, hipMemcpyHostToDevice, st));
            di = ti;
            dl = tl;
        }
        k_scatter_labels<<<grid_for(p->n_labelled, 256), 256, 0, st>>>(n, p->n_labelled, K, di, dl, g->lab, flags);
    }
    unsigned int hf = 0;
    GFW_HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));
    dfree(flags);
    dfree(ti);
    dfree(tl);
    if (hf) return fail(GFW_E_LABELS, "labelled set invalid (range, repeat or class)");

    // degrees d = W 1, then the Gershgorin bound max_i 1 + d_i^{-1/2} (W D^{-1/2} 1)_i
    k_gauss_fill<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, 1.0, gg.V);
    apply_w(gg, 1, gg.V, gg.R, nullptr, st);
    k_gauss_dinv<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, method == GFW_GAUSS_GRID ? 1e-6 : 0.0, gg.R, gg.dinv);
    apply_w(gg, 1, gg.dinv, gg.R, nullptr, st);
    k_gauss_rho<<<grid_for(n, 256, 4096), 256, 0, st>>>(n, gg.dinv, gg.R, gg.V);
    double *rmax = gg.R + n; // R holds n KP >= 4n doubles
    const unsigned long long zero64 = 0; // the bit pattern of +0.0
    GFW_HIP_TRY(hipMemcpyAsync(rmax, &zero64, sizeof(zero64), hipMemcpyHostToDevice, st));
    k_max_nonneg<<<(unsigned)std::min<int64_t>(std::max<int64_t>(cdiv(n, 1024), 1), 1024), 256, 0, st>>>(
        gg.V, n, (unsigned long long *)rmax);
    GFW_HIP_TRY(hipGetLastError());
    GFW_HIP_TRY(hipMemcpyAsync(&g->rho_max, rmax, sizeof(double), hipMemcpyDeviceToHost, st));
    GFW_HIP_TRY(hipStreamSynchronize(st));

    g->shape.kmax = K <= 4 ? 4 : K <= 8 ? 8 : 16;
    g->shape.nb_row = (int)cdiv(n, kRowBlock);
    g->shape.nb_big = 0;
    g->graph_bytes = bytes;
    refresh_solve_bytes(g);
    guard.g = nullptr;
    *out = g;
    return GFW_OK;
}

} // namespace gfw

extern "C" {

gfw_status_t gfw_graph_create_gaussian(gfw_context_t ctx, const gfw_gaussian_problem_t *p, gfw_graph_t *out,
                                       void *stream)
{
    if (!ctx || !out) return gfw::fail(GFW_E_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    return gfw::gauss_graph_create(ctx, p, out, (hipStream_t)stream);
}

} // extern "C"
