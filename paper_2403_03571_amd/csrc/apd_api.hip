// apd_api.hip -- the C ABI of libapd (include/apd.h): validation, scratch,
// the evaluation pass, the L-BFGS weight solver (Algorithm 2 of
// arXiv 2403.03571) and the generalised Lloyd step (Algorithm 3).
#include "../../include/apd.h"
#include "apd_batch.h"
#include "apd_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

struct apd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // device scratch, grown on demand
    int64_t cap_n = 0, cap_J = 0;
    uint64_t *mom = nullptr;          // [cap_n][10]
    unsigned *queue = nullptr;        // [cap_J]
    apd::Scalars *sc = nullptr;       // one per ctx
    apd::BlockParts *parts = nullptr; // partials of the prep and finalize kernels
    double *wbuf = nullptr;           // [cap_n] trial weights of the solver
    double *gbuf = nullptr;           // [cap_n] gradient of the solver
    double *cbuf = nullptr;           // [cap_n][3] centroids of the Lloyd step
    double *eig = nullptr;            // [cap_n][2] eigenvalue range of every A_i (culling)
    int *ord = nullptr;               // [cap_n] the hybrid kernel's seed order
    int *ws_nb = nullptr;             // [cap_n][16] nearest seeds (warm-start features)
    int *tile_lists = nullptr;        // [cap_tiles][kCullCap] candidate seeds per tile
    int *tile_count = nullptr;        // [cap_tiles]
    double *tile_U = nullptr;         // [cap_tiles] cost bound of the seeds left out of each list
    double *cost_part = nullptr;      // [cap_parts] per-block cost sums (costs other than |.|^2_A)
    int64_t cap_parts = 0;
    apd::QSeg *segs = nullptr;        // [cap_tiles] segments of the re-check queue
    int64_t cap_tiles = 0;
    int *super_lists = nullptr;       // [cap_super][kSuperCap] candidate seeds per super-tile
    int *super_count = nullptr;       // [cap_super]
    int64_t cap_super = 0;
    bool need_qtotal = false;          // sum the pixel weights in the next pass (validation)
    int vec_p = 0;                     // pixels per lane of the vector kernel (0: automatic)
    // pinned host staging
    apd::Scalars *h_sc = nullptr;
    unsigned published = 0;           // graph passes published by the finalize (its seq)
    double *h_grad = nullptr;         // [cap_n]
    double *h_w = nullptr;            // [cap_n] staging of the solver's trial weights
    apd_pass_stats stats{0, 0, 0, 0.0, 0.0, 0, 0, 0};
    // HIP-event timing of the passes
    bool profiling = false;
    int variant = 2;  // single-precision kernel over every seed: 0 = matrix cores, 1 = vector ALU,
                      // 2 = hybrid from kHybMinSeeds seeds and kHybMinTiles tiles, else vector (default), 3 = hybrid
    bool culling = true;  // per-tile candidate lists in the vector kernel
    bool adaptive = true; // single-candidate tiles credited whole (with the lists)
    // batched solver: scratch and its own capture stream
    void *batch_buf = nullptr;
    size_t batch_bytes = 0;
    hipStream_t batch_stream = nullptr;
    hipStream_t fit_stream = nullptr;  // captures and replays the evaluation of a fit
    int batch_poll = 4;  // graph replays between polls of the active count
    int batch_kernel = -1;  // kernel of the batched pass (kb_assign's V); -1: by tier
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

namespace {

// The hybrid kernel pays for its per-wave winner search and staging from
// about 1 500 seeds (measured over every seed against the vector kernel: 2D
// 1024^2 at N = 1 000 0.121 / 0.114 ms, 1 500 0.160 / 0.167, 3 000 0.272 /
// 0.316; 3D 128^3 at N = 1 000 0.235 / 0.232, 1 500 0.296 / 0.336; 3D 64^3,
// 128 tiles, at N = 4 000 0.267 / 0.321); on very small grids its larger
// tiles leave compute units idle, so it needs at least 128 of them.
constexpr int64_t kHybMinSeeds = 1536;
constexpr int64_t kHybMinTiles = 128;

bool hyb_by_default(const apd_problem *p) {
    if (p->n < kHybMinSeeds) return false;
    const int64_t m0 = p->grid[0], m1 = p->grid[1];
    const int64_t tiles = p->dim == 3
        ? ((m0 + apd::kHybRows3 - 1) / apd::kHybRows3) * ((m1 + 15) / 16) * ((p->grid[2] + 7) / 8)
        : ((m0 + apd::kHybRows2 - 1) / apd::kHybRows2) * ((m1 + 31) / 32);
    return tiles >= kHybMinTiles;
}

apd_status fail(apd_ctx *c, apd_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
apd_status fail(apd_ctx *c, apd_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    if (st == APD_ERR_DEVICE || st == APD_ERR_OOM) (void)hipGetLastError();  // leave no stale error behind
    return st;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, APD_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

int64_t num_pixels(const apd_problem *p) {
    int64_t J = 1;
    for (int d = 0; d < p->dim; ++d) J *= p->grid[d];
    return J;
}

double box_measure(const apd_problem *p) {
    double m = 1.0;
    for (int d = 0; d < p->dim; ++d) m *= (p->hi[d] - p->lo[d]);
    return m;
}

apd_status check_problem(apd_ctx *c, const apd_problem *p, bool need_v) {
    if (!p) return fail(c, APD_ERR_INVALID_ARG, "problem is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(c, APD_ERR_INVALID_ARG, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->power < 0 || p->power > 4)
        return fail(c, APD_ERR_INVALID_ARG, "power must be 0 (= 2), 1, 2, 3 or 4 (got %d)", p->power);
    if (p->n < 1 || p->n > 0x7fffffffLL) return fail(c, APD_ERR_INVALID_ARG, "n must be in [1, 2^31) (got %lld)", (long long)p->n);
    for (int d = 0; d < p->dim; ++d) {
        if (p->grid[d] < 1) return fail(c, APD_ERR_INVALID_ARG, "grid[%d] must be >= 1", d);
        if (!(p->hi[d] > p->lo[d]) || !isfinite(p->lo[d]) || !isfinite(p->hi[d]))
            return fail(c, APD_ERR_INVALID_ARG, "box axis %d needs finite lo < hi", d);
    }
    const int64_t J = num_pixels(p);
    if (J >= (int64_t)0xffffffffLL) return fail(c, APD_ERR_INVALID_ARG, "too many pixels (%lld >= 2^32 - 1)", (long long)J);
    if (!p->x || !p->A) return fail(c, APD_ERR_INVALID_ARG, "x and A must be device pointers");
    if (need_v && !p->v) return fail(c, APD_ERR_INVALID_ARG, "target volumes v are required");
    if (p->mass) {
        // the weighted second moments must fit in 64 bits
        int32_t mmax = 1;
        for (int d = 0; d < p->dim; ++d) mmax = std::max(mmax, p->grid[d]);
        const double bound = 255.0 * (double)J * (2.0 * mmax + 1.0) * (2.0 * mmax + 1.0);
        if (!(bound < 1.8e19))
            return fail(c, APD_ERR_INVALID_ARG, "grid too large for pixel weights (255 J (2M)^2 >= 2^64)");
    }
    return APD_OK;
}

apd::Geo make_geo(const apd_problem *p) {
    apd::Geo g{};
    g.dim = p->dim;
    g.n = (int)p->n;
    g.pixvol = 1.0;
    for (int d = 0; d < 3; ++d) {
        g.grid[d] = d < p->dim ? p->grid[d] : 1;
        g.lo[d] = d < p->dim ? p->lo[d] : 0.0;
        g.s[d] = d < p->dim ? (p->hi[d] - p->lo[d]) / (double)p->grid[d] : 1.0;
        if (d < p->dim) g.pixvol *= g.s[d];
    }
    g.mass = p->mass;
    g.munit = p->mass ? g.pixvol / 255.0 : g.pixvol;
    g.power = p->power == 0 ? 2 : p->power;
    return g;
}

apd_status ensure_scratch(apd_ctx *c, int64_t n, int64_t J) {
    if (n > c->cap_n) {
        (void)hipFree(c->mom); c->mom = nullptr;
        (void)hipFree(c->wbuf); c->wbuf = nullptr;
        (void)hipFree(c->gbuf); c->gbuf = nullptr;
        (void)hipFree(c->cbuf); c->cbuf = nullptr;
        (void)hipFree(c->eig); c->eig = nullptr;
        (void)hipFree(c->ord); c->ord = nullptr;
        (void)hipFree(c->ws_nb); c->ws_nb = nullptr;
        (void)hipHostFree(c->h_grad); c->h_grad = nullptr;
        (void)hipHostFree(c->h_w); c->h_w = nullptr;
        c->cap_n = 0;
        const int64_t nn = std::max<int64_t>(n, 1024);
        if (hipMalloc(&c->mom, (size_t)nn * 10 * sizeof(uint64_t)) != hipSuccess ||
            hipMalloc(&c->wbuf, (size_t)nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gbuf, (size_t)nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->cbuf, (size_t)nn * 3 * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->eig, (size_t)nn * 2 * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->ord, (size_t)nn * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->ws_nb, (size_t)nn * 16 * sizeof(int)) != hipSuccess ||
            hipHostMalloc(&c->h_grad, (size_t)nn * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&c->h_w, (size_t)nn * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(c, APD_ERR_OOM, "cannot allocate seed scratch for n = %lld", (long long)n);
        c->cap_n = nn;
    }
    if (J > c->cap_J) {
        (void)hipFree(c->queue); c->queue = nullptr;
        c->cap_J = 0;
        if (hipMalloc(&c->queue, (size_t)J * sizeof(unsigned)) != hipSuccess)
            return fail(c, APD_ERR_OOM, "cannot allocate the re-check queue for %lld pixels", (long long)J);
        c->cap_J = J;
    }
    return APD_OK;
}

apd_status decode_bad(apd_ctx *c, int bad, bool need_v) {
    if (bad & apd::kBadX) return fail(c, APD_ERR_NONFINITE, "non-finite seed coordinate");
    if (bad & apd::kBadA) return fail(c, APD_ERR_NONFINITE, "non-finite anisotropy matrix entry");
    if (bad & apd::kBadW) return fail(c, APD_ERR_NONFINITE, "non-finite weight");
    if (bad & apd::kBadSPD) return fail(c, APD_ERR_NOT_SPD, "an anisotropy matrix is not symmetric positive definite");
    if (need_v && (bad & apd::kBadV)) return fail(c, APD_ERR_VOLUMES, "target volumes must be positive and finite");
    return APD_OK;
}

// Device buffers of one pass.  The context's own (grown on demand) or, for
// apd_dual_objective_grad_noalloc, regions of the static scratch array.
struct PassBufs {
    uint64_t *mom = nullptr;       // [n][K]
    unsigned *queue = nullptr;     // [J]
    double *eig = nullptr;         // [n][2]
    int *ord = nullptr;            // [n] seed order of the hybrid kernel
    int *tile_lists = nullptr;     // [tiles][list_cap]
    int *tile_count = nullptr;     // [tiles]
    double *tile_U = nullptr;      // [tiles]
    apd::QSeg *segs = nullptr;     // [tiles]
    int64_t cap_tiles = 0;
    int list_cap = apd::kCullCap;
    int *super_lists = nullptr;    // [super-tiles][super_cap]
    int *super_count = nullptr;    // [super-tiles]
    int64_t cap_super = 0;
    int super_cap = apd::kSuperCap;
    apd::Scalars *sc = nullptr;
    apd::BlockParts *parts = nullptr;
    double *cost_part = nullptr;   // [FP64 blocks], costs other than the squared norm
    int64_t cap_parts = 0;
};

// Tiles of the candidate-list kernels of a pass and their super-tiles
// (about three cell diameters across, (J / n)^(1/D) pixels, whole tiles per
// axis, at most 8 per axis).
struct ListGeometry {
    int tp = 0;
    int ntile[3] = {1, 1, 1};
    int sf[3] = {1, 1, 1};
    int nst[3] = {1, 1, 1};
    int64_t tiles = 0, nsuper = 0;
};

ListGeometry list_geometry(const apd_problem *p, const apd::Geo &g, apd_precision prec) {
    ListGeometry L;
    L.tp = prec == APD_BF16 ? apd::bf16_pixels_per_lane(g) : apd::vec_pixels_per_lane(g, true);
    const int ext[3] = {apd::tile_ext(p->dim, L.tp, 0), apd::tile_ext(p->dim, L.tp, 1),
                        apd::tile_ext(p->dim, L.tp, 2)};
    for (int d = 0; d < 3; ++d) L.ntile[d] = d < p->dim ? (g.grid[d] + ext[d] - 1) / ext[d] : 1;
    L.tiles = (int64_t)L.ntile[0] * L.ntile[1] * L.ntile[2];
    const double diam = pow((double)num_pixels(p) / (double)p->n, 1.0 / p->dim);
    L.nsuper = 1;
    for (int d = 0; d < 3; ++d) {
        const int f = d < p->dim ? (int)lround(3.0 * diam / ext[d]) : 1;
        L.sf[d] = std::max(1, std::min(8, f));
        L.nst[d] = (L.ntile[d] + L.sf[d] - 1) / L.sf[d];
        L.nsuper *= L.nst[d];
    }
    return L;
}

// Enqueue one evaluation pass: prep, assignment (+ re-check), optional
// finalize.  With `fixed`, every buffer comes from it and nothing is
// allocated (the caller has checked its capacities).
apd_status enqueue_pass(apd_ctx *c, const apd_problem *p, const double *x, const double *w,
                        int32_t *labels, bool moments, bool finalize, const apd::FinalOut &fo,
                        apd_precision prec, const double *w_host = nullptr, float *rel_gap = nullptr,
                        const PassBufs *fixed = nullptr) {
    apd::Geo g = make_geo(p);
    g.vec_p = c->vec_p;
    const int64_t J = num_pixels(p);
    PassBufs b;
    if (fixed) {
        b = *fixed;
    } else {
        apd_status st = ensure_scratch(c, p->n, J);
        if (st != APD_OK) return st;
        b.mom = c->mom;
        b.queue = c->queue;
        b.eig = c->eig;
        b.ord = c->ord;
        b.sc = c->sc;
        b.parts = c->parts;
    }
    apd::Seeds sd{x, p->A, w, p->v};
    uint64_t *mom = moments ? b.mom : nullptr;
    if (prec != APD_FP64 && prec != APD_FP32 && prec != APD_BF16)
        return fail(c, APD_ERR_INVALID_ARG, "precision %d is not available", (int)prec);
    const bool cull = c->culling && ((prec == APD_FP32 && c->variant >= 1) || prec == APD_BF16);
    const bool timing = c->profiling && !fixed;
    if (timing) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, apd::launch_prep(g, sd, b.sc, mom, cull ? b.eig : nullptr, b.parts, c->stream, w_host));
    if (g.mass && c->need_qtotal) HIP_TRY(c, apd::launch_mass_total(g, b.sc, c->stream));
    if (timing) HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    apd::PassOut out{labels, mom, nullptr};
    out.rel_gap = rel_gap;
    if (g.power != 2 && prec != APD_FP64)
        return fail(c, APD_ERR_INVALID_ARG, "costs of power %d run in APD_FP64 only", g.power);
    if (prec == APD_FP64) {
        if (g.power != 2 && finalize) {
            // the objective of such costs is summed pixel by pixel
            const int64_t nb = apd::fp64_blocks(g);
            if (fixed) {
                if (nb > b.cap_parts) return fail(c, APD_ERR_INVALID_ARG, "cost sums exceed the fixed scratch");
            } else if (nb > c->cap_parts) {
                (void)hipFree(c->cost_part);
                c->cost_part = nullptr;
                c->cap_parts = 0;
                if (hipMalloc(&c->cost_part, (size_t)nb * sizeof(double)) != hipSuccess)
                    return fail(c, APD_ERR_OOM, "cannot allocate the cost sums of %lld blocks", (long long)nb);
                c->cap_parts = nb;
            }
            out.cost_part = fixed ? b.cost_part : c->cost_part;
        }
        HIP_TRY(c, apd::launch_assign_fp64(g, sd, b.sc, out, c->stream));
        if (timing) HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
        c->stats.kernel = APD_KERNEL_FP64;
        c->stats.pixels_per_lane = 0;
    } else {
        out.queue = b.queue;
        if (prec == APD_BF16 && !cull) {
            HIP_TRY(c, apd::launch_assign_bf16(g, sd, b.sc, nullptr, out, c->stream));
            c->stats.kernel = APD_KERNEL_BF16_MATRIX;
            c->stats.pixels_per_lane = apd::bf16_pixels_per_lane(g);
        } else if (cull) {
            const ListGeometry L = list_geometry(p, g, prec);
            out.tp = L.tp;
            for (int d = 0; d < 3; ++d) out.ntile[d] = L.ntile[d];
            if (fixed) {
                if (L.tiles > b.cap_tiles || L.nsuper > b.cap_super)
                    return fail(c, APD_ERR_INVALID_ARG, "candidate lists exceed the fixed scratch");
            } else {
                if (L.tiles > c->cap_tiles) {
                    (void)hipFree(c->tile_lists);
                    (void)hipFree(c->tile_count);
                    (void)hipFree(c->tile_U);
                    (void)hipFree(c->segs);
                    c->tile_lists = nullptr;
                    c->tile_count = nullptr;
                    c->tile_U = nullptr;
                    c->segs = nullptr;
                    c->cap_tiles = 0;
                    if (hipMalloc(&c->tile_lists, (size_t)L.tiles * apd::kCullCap * sizeof(int)) != hipSuccess ||
                        hipMalloc(&c->tile_count, (size_t)L.tiles * sizeof(int)) != hipSuccess ||
                        hipMalloc(&c->tile_U, (size_t)L.tiles * sizeof(double)) != hipSuccess ||
                        hipMalloc(&c->segs, (size_t)L.tiles * sizeof(apd::QSeg)) != hipSuccess)
                        return fail(c, APD_ERR_OOM, "cannot allocate candidate lists for %lld tiles",
                                    (long long)L.tiles);
                    c->cap_tiles = L.tiles;
                }
                b.tile_lists = c->tile_lists;
                b.tile_count = c->tile_count;
                b.tile_U = c->tile_U;
                b.segs = c->segs;
                if (L.nsuper > c->cap_super) {
                    (void)hipFree(c->super_lists);
                    (void)hipFree(c->super_count);
                    c->super_lists = nullptr;
                    c->super_count = nullptr;
                    c->cap_super = 0;
                    if (hipMalloc(&c->super_lists, (size_t)L.nsuper * apd::kSuperCap * sizeof(int)) != hipSuccess ||
                        hipMalloc(&c->super_count, (size_t)L.nsuper * sizeof(int)) != hipSuccess)
                        return fail(c, APD_ERR_OOM, "cannot allocate candidate lists for %lld super-tiles",
                                    (long long)L.nsuper);
                    c->cap_super = L.nsuper;
                }
                b.super_lists = c->super_lists;
                b.super_count = c->super_count;
            }
            out.tile_lists = b.tile_lists;
            out.tile_count = b.tile_count;
            out.list_cap = b.list_cap;
            out.adaptive = c->adaptive;
            out.credited = &b.sc->credited;
            if (rel_gap) out.tile_U = b.tile_U;
            out.segs = b.segs;
            for (int d = 0; d < 3; ++d) {
                out.sf[d] = L.sf[d];
                out.nst[d] = L.nst[d];
            }
            if (L.sf[0] * L.sf[1] * L.sf[2] > 1) {
                out.super_cap = b.super_cap;
                HIP_TRY(c, apd::launch_super_cull(g, sd, b.sc, b.eig, out, b.super_lists, b.super_count,
                                                  c->stream));
                out.super_list = b.super_lists;
                out.super_count = b.super_count;
            }
            if (prec == APD_BF16) HIP_TRY(c, apd::launch_assign_bf16(g, sd, b.sc, b.eig, out, c->stream));
            else HIP_TRY(c, apd::launch_assign_cull(g, sd, b.sc, b.eig, out, c->stream));
            c->stats.kernel = prec == APD_BF16 ? APD_KERNEL_BF16_LISTS : APD_KERNEL_FP32_LISTS;
            c->stats.pixels_per_lane = L.tp;
        } else if (c->variant == 3 || (c->variant == 2 && hyb_by_default(p))) {
            HIP_TRY(c, apd::launch_seed_order(g, sd, b.ord, c->stream));
            out.seed_order = b.ord;
            HIP_TRY(c, apd::launch_assign_hyb(g, sd, b.sc, out, c->stream));
            c->stats.kernel = APD_KERNEL_FP32_HYBRID;
            c->stats.pixels_per_lane = g.dim == 3 ? 16 : 8;  // pixels a lane evaluates
        } else if (c->variant >= 1) {
            HIP_TRY(c, apd::launch_assign_fp32(g, sd, b.sc, out, c->stream));
            c->stats.kernel = APD_KERNEL_FP32_VECTOR;
            c->stats.pixels_per_lane = apd::vec_pixels_per_lane(g, false);
        } else {
            HIP_TRY(c, apd::launch_assign_mfma(g, sd, b.sc, out, c->stream));
            c->stats.kernel = APD_KERNEL_FP32_MATRIX;
            c->stats.pixels_per_lane = 0;
        }
        if (timing) HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
        HIP_TRY(c, apd::launch_recheck(g, sd, b.sc, out, c->stream));
    }
    if (finalize) HIP_TRY(c, apd::launch_finalize(g, sd, b.mom, b.sc, fo, b.parts, c->stream));
    c->stats.pixels = J;
    c->stats.pairs = J * p->n;
    return APD_OK;
}

// Copy the scalars back and wait for the stream.
apd_status sync_scalars(apd_ctx *c) {
    HIP_TRY(c, hipMemcpyAsync(c->h_sc, c->sc, sizeof(apd::Scalars), hipMemcpyDeviceToHost, c->stream));
    hipEvent_t end = nullptr;
    if (c->profiling) {
        HIP_TRY(c, hipEventCreate(&end));
        HIP_TRY(c, hipEventRecord(end, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->stats.rechecked = c->h_sc->qcount;
    c->stats.tiles_credited = c->h_sc->credited;
    if (c->profiling) {
        float a = 0.0f, t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&a, c->ev[1], c->ev[2]));
        HIP_TRY(c, hipEventElapsedTime(&t, c->ev[0], end));
        (void)hipEventDestroy(end);
        c->stats.assign_ms = a;
        c->stats.pass_ms = t;
    }
    return APD_OK;
}

// Wait until the finalize of the pass enqueued on `stream` has published
// pass number `want` in the pinned scalars (their seq field, written after
// the gradient and the other scalars), checking the stream now and then so
// that a failed pass ends the wait.  Cheaper than the stream's completion
// signal; the kernel's tail may still be running on return.
// A pass that has neither published nor finished after kPublishTimeout
// seconds is reported as a device error (the stream may still be running).
constexpr double kPublishTimeout = 300.0;

apd_status wait_published(apd_ctx *c, hipStream_t stream, unsigned want) {
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned k = 1; __atomic_load_n(&c->h_sc->seq, __ATOMIC_ACQUIRE) != want; ++k) {
        if ((k & 1023u) != 0) continue;
        const hipError_t q = hipStreamQuery(stream);
        if (q == hipErrorNotReady) {
            if ((k & 0xfffffu) == 0 &&
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > kPublishTimeout)
                return fail(c, APD_ERR_DEVICE, "an evaluation did not publish its result within %.0f s",
                            kPublishTimeout);
            continue;
        }
        if (q != hipSuccess) return fail(c, APD_ERR_DEVICE, "evaluation: %s", hipGetErrorString(q));
        if (__atomic_load_n(&c->h_sc->seq, __ATOMIC_ACQUIRE) != want)
            return fail(c, APD_ERR_DEVICE, "an evaluation ended without publishing its result");
    }
    c->stats.rechecked = c->h_sc->qcount;
    c->stats.tiles_credited = c->h_sc->credited;
    return APD_OK;
}

// The pass number the next publishing pass will write; the pinned seq is
// reset first so that a stale value cannot match.
unsigned next_published(apd_ctx *c) {
    const unsigned want = ++c->published;
    __atomic_store_n(&c->h_sc->seq, want - 1u, __ATOMIC_RELEASE);
    return want;
}

apd_status check_volumes(apd_ctx *c, const apd_problem *p) {
    // the domain measure: |Omega|, or sum_j |P_j| with pixel weights
    const double om = p->mass ? (double)c->h_sc->qtotal * make_geo(p).munit : box_measure(p);
    if (fabs(c->h_sc->vsum - om) > 1e-12 * om)
        return fail(c, APD_ERR_VOLUMES, "target volumes sum to %.17g, the box measure is %.17g", c->h_sc->vsum, om);
    return APD_OK;
}

// One evaluation at device weights w: returns g~, max rel error; gradient in
// c->gbuf (device) and optionally on the host.
apd_status evaluate(apd_ctx *c, const apd_problem *p, const double *x, const double *w,
                    apd_precision prec, bool host_grad, double *g, double *maxrel,
                    const apd::FinalOut *extra, bool validate) {
    apd::FinalOut fo{c->gbuf, nullptr, nullptr};
    if (extra) {
        if (extra->grad) fo.grad = extra->grad;
        fo.counts = extra->counts;
        fo.centroids = extra->centroids;
    }
    c->need_qtotal = validate;
    // without per-pass timing or a host copy of the gradient, the finalize
    // publishes the scalars in pinned memory and the host waits for that
    // instead of the stream
    const bool publish = !host_grad && !c->profiling;
    unsigned want = 0;
    if (publish) {
        fo.host_sc = c->h_sc;
        want = next_published(c);
    }
    apd_status st = enqueue_pass(c, p, x, w, nullptr, true, true, fo, prec);
    c->need_qtotal = false;
    if (st != APD_OK) {
        if (publish) --c->published;  // its finalize was never enqueued
        return st;
    }
    if (host_grad)
        HIP_TRY(c, hipMemcpyAsync(c->h_grad, fo.grad, (size_t)p->n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    st = publish ? wait_published(c, c->stream, want) : sync_scalars(c);
    if (st != APD_OK) return st;
    if (validate || c->h_sc->bad) {
        st = decode_bad(c, c->h_sc->bad, true);
        if (st != APD_OK) return st;
        st = check_volumes(c, p);
        if (st != APD_OK) return st;
    }
    *g = c->h_sc->g;
    if (maxrel) *maxrel = c->h_sc->maxrel;
    return APD_OK;
}

double default_gamma0(int dim, int64_t n) { return dim == 2 ? 0.3 : 0.2 * cbrt((double)n); }

// ---------------------------------------------------------------- L-BFGS
//
// Minimises f = -g~ (grad f = m|P| - v), the specification shared with the
// CPU reference: evaluate at the start and stop as soon as any evaluation
// meets max_i |grad_i| / v_i < eps; gradients are projected on sum = 0;
// direction by the two-loop recursion over at most `history` pairs with
// H0 = (s.y / y.y) I of the newest pair, or -gamma0 grad with no pairs;
// Armijo backtracking (c1 = 1e-4) from the unit step, halving up to 30
// times; a pair is stored only when s.y > 1e-10 |s| |y|; a non-descent
// direction or a failed search clears the history and retries with the
// scaled steepest step, whose own failure ends the solve.
// sum_i a_i b_i with eight running partial sums combined in a fixed order
// (deterministic; a single running sum is a chain of dependent additions,
// about 0.26 ms per direction at n = 10^4)
double dotn(const double *a, const double *b, int64_t n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = 0;
    for (; i + 8 <= n; i += 8)
        for (int k = 0; k < 8; ++k) s[k] += a[i + k] * b[i + k];
    for (int k = 0; i < n; ++i, ++k) s[k] += a[i] * b[i];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// sum_i a_i in dotn's order (dotn(a, ones) without the ones)
double sumn(const double *a, int64_t n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = 0;
    for (; i + 8 <= n; i += 8)
        for (int k = 0; k < 8; ++k) s[k] += a[i + k];
    for (int k = 0; i < n; ++i, ++k) s[k] += a[i];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// q_i += a y_i (the product a y_i added), returning dotn(z, q) of the
// updated values
double axpy_dot(double *__restrict__ q, double a, const double *__restrict__ y, const double *__restrict__ z,
                int64_t n) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = 0;
    for (; i + 8 <= n; i += 8)
        for (int k = 0; k < 8; ++k) {
            const double v = q[i + k] + a * y[i + k];
            q[i + k] = v;
            s[k] += z[i + k] * v;
        }
    for (int k = 0; i < n; ++i, ++k) {
        const double v = q[i] + a * y[i];
        q[i] = v;
        s[k] += z[i] * v;
    }
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

struct Lbfgs {
    int64_t n;
    int m;
    std::vector<std::vector<double>> S, Y;  // m slots, a circular buffer of pairs
    std::vector<double> rho;
    int count = 0, head = 0;  // stored pairs; slot of the oldest
    std::vector<double> q, alpha;

    Lbfgs(int64_t n_, int m_)
        : n(n_), m(m_), S(m_, std::vector<double>(n_)), Y(m_, std::vector<double>(n_)), rho(m_),
          q(n_), alpha(m_) {}
    static double dot(const std::vector<double> &a, const std::vector<double> &b) {
        return dotn(a.data(), b.data(), (int64_t)a.size());
    }
    bool empty() const { return count == 0; }
    void clear() { count = head = 0; }
    int slot(int t) const { return (head + t) % m; }  // t-th oldest pair
    // store (s, y), dropping the oldest pair when full; s and y are taken
    // by swapping storage (the caller's vectors then hold stale values)
    void push(std::vector<double> &s, std::vector<double> &y, double sy) {
        int j;
        if (count == m) {
            j = head;
            head = (head + 1) % m;
        } else {
            j = slot(count++);
        }
        S[j].swap(s);
        Y[j].swap(y);
        rho[j] = 1.0 / sy;
    }
    // d = -H grad, by the two-loop recursion (Nocedal & Wright, Alg. 7.4).
    // Each update of q is fused with the dot product the next step needs
    // (same products and the same summation order as dotn, so the same bits
    // as separate passes), which halves the passes over the history.
    void direction(const std::vector<double> &grad, double gamma0, std::vector<double> &d) {
        const int64_t nn = n;
        double *__restrict__ qp = q.data();
        double *__restrict__ dp = d.data();
        const double *__restrict__ gp = grad.data();
        if (count == 0) {
            for (int64_t i = 0; i < nn; ++i) dp[i] = -gamma0 * gp[i];
            return;
        }
        // first loop, newest pair to oldest: a_t = rho_t s_t.q, q -= a_t y_t
        for (int64_t i = 0; i < nn; ++i) qp[i] = gp[i];
        double at = rho[slot(count - 1)] * dotn(S[slot(count - 1)].data(), qp, nn);
        for (int t = count - 1; t >= 0; --t) {
            const int j = slot(t);
            alpha[t] = at;
            const double *__restrict__ yj = Y[j].data();
            if (t > 0) {
                at = rho[slot(t - 1)] * axpy_dot(qp, -at, yj, S[slot(t - 1)].data(), nn);
            } else {
                // the last update, fused with gamma's scaling
                const int k = slot(count - 1);
                const double gamma = dot(S[k], Y[k]) / dot(Y[k], Y[k]);
                for (int64_t i = 0; i < nn; ++i) qp[i] = (qp[i] - at * yj[i]) * gamma;
            }
        }
        // second loop, oldest pair to newest: q += (a_t - rho_t y_t.q) s_t
        double c = alpha[0] - rho[slot(0)] * dotn(Y[slot(0)].data(), qp, nn);
        for (int t = 0; t < count; ++t) {
            const double *__restrict__ sj = S[slot(t)].data();
            if (t + 1 < count) {
                const int jn = slot(t + 1);
                c = alpha[t + 1] - rho[jn] * axpy_dot(qp, c, sj, Y[jn].data(), nn);
            } else {
                for (int64_t i = 0; i < nn; ++i) dp[i] = -(qp[i] + sj[i] * c);
            }
        }
    }
};

// s = wt - w, y = gt - g, and the dot products s.y, s.s, y.y (each in
// dotn's order) in one pass
void pair_dots(const double *__restrict__ wt, const double *__restrict__ w, const double *__restrict__ gt,
               const double *__restrict__ g, double *__restrict__ s, double *__restrict__ y, int64_t n,
               double *out) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0}, b[8] = {0, 0, 0, 0, 0, 0, 0, 0}, c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = 0;
    for (; i + 8 <= n; i += 8)
        for (int k = 0; k < 8; ++k) {
            const double sv = wt[i + k] - w[i + k], yv = gt[i + k] - g[i + k];
            s[i + k] = sv;
            y[i + k] = yv;
            a[k] += sv * yv;
            b[k] += sv * sv;
            c[k] += yv * yv;
        }
    for (int k = 0; i < n; ++i, ++k) {
        const double sv = wt[i] - w[i], yv = gt[i] - g[i];
        s[i] = sv;
        y[i] = yv;
        a[k] += sv * yv;
        b[k] += sv * sv;
        c[k] += yv * yv;
    }
    out[0] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    out[1] = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
    out[2] = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
}

void project_mean(std::vector<double> &g) {
    const double s = sumn(g.data(), (int64_t)g.size()) / (double)g.size();
    for (double &v : g) v -= s;
}

apd_status fit_impl(apd_ctx *c, const apd_problem *p, const double *x, double *w_inout,
                    const apd_fit_opts *o, apd_fit_report *rep) {
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t n = p->n;
    apd_status st = ensure_scratch(c, n, num_pixels(p));
    if (st != APD_OK) return st;
    if (!(o->eps > 0.0) || o->max_iter < 0 || o->max_evals < 1 || o->history < 0)
        return fail(c, APD_ERR_INVALID_ARG, "bad fit options");
    const double gamma0 = o->gamma0 > 0.0 ? o->gamma0 : default_gamma0(p->dim, n);
    std::vector<double> w(n, 0.0), wt(n), gr(n), gt(n), d(n);
    if (o->warm) {
        HIP_TRY(c, hipMemcpyAsync(w.data(), w_inout, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }

    // After the first evaluation (which validates the inputs and sizes the
    // scratch) the evaluation -- upload of w, the pass, the downloads -- is
    // captured once as a HIP graph on a stream of the library's and
    // replayed, one launch per evaluation instead of about ten.  Not with
    // per-pass profiling, whose events are recorded eagerly.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct GraphGuard {
        hipGraph_t *g;
        hipGraphExec_t *e;
        hipStream_t *s;
        ~GraphGuard() {
            // a replay may still be finishing after it published its result
            if (*e && *s) (void)hipStreamSynchronize(*s);
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } guard{&graph, &exec, &c->fit_stream};
    auto capture = [&]() -> apd_status {
        if (!c->fit_stream) HIP_TRY(c, hipStreamCreate(&c->fit_stream));
        hipStream_t user = c->stream;
        c->stream = c->fit_stream;
        HIP_TRY(c, hipStreamBeginCapture(c->fit_stream, hipStreamCaptureModeThreadLocal));
        // no copies in the graph: the prep kernel reads the weights from
        // the pinned staging buffer, and the finalize writes the gradient
        // and the scalars straight into pinned host buffers (measured: the
        // gradient's copy was 2 % of a fit)
        apd::FinalOut fo{c->h_grad, nullptr, nullptr};
        fo.host_sc = c->h_sc;
        const apd_status s2 = enqueue_pass(c, p, x, c->wbuf, nullptr, true, true, fo, o->prec, c->h_w);
        const hipError_t ce = hipStreamEndCapture(c->fit_stream, &graph);
        c->stream = user;
        if (s2 != APD_OK) return s2;
        if (ce != hipSuccess)
            return fail(c, APD_ERR_DEVICE, "capture of the evaluation failed: %s", hipGetErrorString(ce));
        HIP_TRY(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        return APD_OK;
    };
    // evaluate at host weights `ww`: upload, pass, download grad f = -grad g~
    auto eval = [&](const std::vector<double> &ww, std::vector<double> &gf, double &f, double &crit,
                    bool validate) -> apd_status {
        memcpy(c->h_w, ww.data(), n * sizeof(double));  // pinned staging
        double g;
        if (exec) {
            // the finalize publishes the pass by writing seq last (after the
            // gradient and the scalars); waiting for it on the pinned copy
            // skips the stream's completion signal, and the stream is
            // checked now and then so that a failed pass ends the wait
            const unsigned want = next_published(c);
            const hipError_t le = hipGraphLaunch(exec, c->fit_stream);
            if (le != hipSuccess) {
                --c->published;
                return fail(c, APD_ERR_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(le));
            }
            const apd_status ws = wait_published(c, c->fit_stream, want);
            if (ws != APD_OK) return ws;
            if (c->h_sc->bad) return decode_bad(c, c->h_sc->bad, true);
            g = c->h_sc->g;
            crit = c->h_sc->maxrel;
        } else {
            hipError_t e = hipMemcpyAsync(c->wbuf, c->h_w, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) return fail(c, APD_ERR_DEVICE, "upload of w: %s", hipGetErrorString(e));
            apd_status s2 = evaluate(c, p, x, c->wbuf, o->prec, true, &g, &crit, nullptr, validate);
            if (s2 != APD_OK) return s2;
            if (!c->profiling) {
                s2 = capture();
                if (s2 != APD_OK) return s2;
            }
        }
        for (int64_t i = 0; i < n; ++i) gf[i] = -c->h_grad[i];
        f = -g;
        return APD_OK;
    };

    Lbfgs lb(n, std::max(o->history, 1));
    std::vector<double> sv(n), yv(n);
    int iters = 0, evals = 0;
    double f = 0.0, crit = 0.0, ft = 0.0, critt = 0.0;
    apd_status result = APD_ERR_NOT_CONVERGED;
    st = eval(w, gr, f, crit, true);
    if (st != APD_OK) return st;
    evals = 1;
    if (crit < o->eps) {
        result = APD_OK;
    } else {
        project_mean(gr);
        while (iters < o->max_iter && evals < o->max_evals) {
            lb.direction(gr, gamma0, d);
            const double gd = Lbfgs::dot(gr, d);
            if (!(gd < 0.0)) {
                if (!lb.empty()) { lb.clear(); continue; }
                result = APD_ERR_LINESEARCH;
                break;
            }
            double a = 1.0;
            bool accepted = false, stop = false;
            for (int t = 0; t < 30; ++t) {
                for (int64_t i = 0; i < n; ++i) wt[i] = w[i] + a * d[i];
                st = eval(wt, gt, ft, critt, false);
                if (st != APD_OK) return st;
                ++evals;
                if (critt < o->eps) {
                    w = wt; f = ft; crit = critt; ++iters;
                    result = APD_OK;
                    stop = true;
                    break;
                }
                if (ft <= f + 1e-4 * a * gd) { accepted = true; break; }
                if (evals >= o->max_evals) { stop = true; break; }
                a *= 0.5;
            }
            if (stop) break;
            if (!accepted) {
                if (!lb.empty()) { lb.clear(); continue; }
                result = APD_ERR_LINESEARCH;
                break;
            }
            project_mean(gt);
            double dots[3];  // s.y, s.s, y.y
            pair_dots(wt.data(), w.data(), gt.data(), gr.data(), sv.data(), yv.data(), n, dots);
            const double sy = dots[0];
            const double ns = sqrt(dots[1]), ny = sqrt(dots[2]);
            if (sy > 1e-10 * ns * ny) lb.push(sv, yv, sy);
            w.swap(wt);  // wt and gt are rewritten whole before their next use
            gr.swap(gt);
            f = ft; crit = critt; ++iters;
        }
    }
    // the last published pass may still be finishing on the fit's stream
    if (c->fit_stream) HIP_TRY(c, hipStreamSynchronize(c->fit_stream));
    HIP_TRY(c, hipMemcpyAsync(w_inout, w.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (rep) {
        rep->converged = result == APD_OK;
        rep->iters = iters;
        rep->evals = evals;
        rep->rechecked = (int32_t)c->stats.rechecked;
        rep->max_rel_err = crit;
        rep->g = -f;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        for (int d = 0; d < 3; ++d) rep->grid[d] = d < p->dim ? p->grid[d] : 1;
        rep->refinements = 0;
    }
    if (result == APD_ERR_NOT_CONVERGED) {
        int32_t M = 0;
        double vmin = 0.0;
        // suggest eq. (2.10) from the smallest target volume
        std::vector<double> v(n);
        if (hipMemcpyAsync(v.data(), p->v, n * sizeof(double), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
            hipStreamSynchronize(c->stream) == hipSuccess) {
            vmin = *std::min_element(v.begin(), v.end());
            apd_choose_resolution(p->dim, o->eps, vmin, box_measure(p), &M);
        }
        return fail(c, APD_ERR_NOT_CONVERGED,
                    "not converged after %d iterations / %d passes (max rel. error %.4g); "
                    "eq. (2.10) suggests M = %d pixels per axis", iters, evals, crit, M);
    }
    if (result == APD_ERR_LINESEARCH)
        return fail(c, APD_ERR_LINESEARCH, "line search failed after a restart (max rel. error %.4g)", crit);
    return APD_OK;
}

// ---------------------------------------------------------------- batched

constexpr int kBatchHist = 10;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// A timed run of the batched solve for the kernel choice: the kernel to
// use, and the replay time of its graph (HIP events on the batch stream).
struct BatchTrial {
    int kernel;
    float replay_ms;
};

// kb_assign's V -> apd_kernel
int batch_public_kernel(int v) {
    return v == 0 ? APD_KERNEL_FP32_MATRIX : v == 1 ? APD_KERNEL_FP32_VECTOR
         : v == 3 ? APD_KERNEL_BF16_MATRIX : v == 5 ? APD_KERNEL_BF16_LISTS : APD_KERNEL_FP32_LISTS;
}

apd_status fit_batched_impl(apd_ctx *c, const apd_problem *probs, int32_t B,
                            double *const *w_inout, const apd_fit_opts *o, apd_fit_report *reps,
                            BatchTrial *trial = nullptr) {
    const auto t_start = std::chrono::steady_clock::now();
    const int dim = probs[0].dim;
    for (int b = 0; b < B; ++b) {
        apd_status st = check_problem(c, &probs[b], true);
        if (st != APD_OK) return fail(c, st, "instance %d: %s", b, c->err.c_str());
        if (probs[b].dim != dim) return fail(c, APD_ERR_INVALID_ARG, "all instances need the same dim");
        if (probs[b].mass)
            return fail(c, APD_ERR_INVALID_ARG, "instance %d: the batched solver takes no pixel weights", b);
        if (probs[b].power != 0 && probs[b].power != 2)
            return fail(c, APD_ERR_INVALID_ARG, "instance %d: the batched solver takes the squared norm only", b);
        if (!w_inout[b]) return fail(c, APD_ERR_INVALID_ARG, "w_inout[%d] is NULL", b);
    }
    if (!(o->eps > 0.0) || o->max_iter < 0 || o->max_evals < 1)
        return fail(c, APD_ERR_INVALID_ARG, "bad fit options");
    if (o->prec != APD_FP32 && o->prec != APD_BF16)
        return fail(c, APD_ERR_INVALID_ARG, "the batched solver runs the APD_FP32 or APD_BF16 tier");
    const int K = apd::moments_per_cell(dim);
    // kernel of the batched pass: a trial's, else the context's choice
    // (apd_set_batch_kernel, apd_autotune_batched: every kernel yields the
    // same certified labels), else by tier: bf16 matrix cores for APD_BF16
    // (with candidate lists unless culling is off); for APD_FP32 the
    // context's variant (vector with candidate lists by default, 8 pixels
    // per lane unless the context asks for 4)
    const int bvariant = trial ? trial->kernel : c->batch_kernel >= 0 ? c->batch_kernel
                         : o->prec == APD_BF16 ? (c->culling ? 5 : 3)
                         : (c->variant == 0 ? 0 : (c->culling ? (c->vec_p == 4 ? 4 : 2) : 1));
    const bool bf = bvariant == 3 || bvariant == 5;
    const int btp = bvariant == 4 ? apd::kP : bf ? (dim == 2 ? 4 : 2) : 8;
    // work list: largest instances first
    std::vector<int> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return probs[a].n * num_pixels(&probs[a]) > probs[b].n * num_pixels(&probs[b]);
    });
    // scratch layout
    size_t nd = 0, nm = 0;
    int64_t qcap = 0;
    std::vector<apd::BInst> hinst(B);
    std::vector<int64_t> tile0(B + 1, 0);
    std::vector<size_t> off_d(B), off_m(B);
    for (int q = 0; q < B; ++q) {
        const apd_problem &p = probs[order[q]];
        off_d[q] = nd;
        nd += (size_t)p.n * (7 + 2 * kBatchHist) + kBatchHist;
        off_m[q] = nm;
        nm += (size_t)p.n * K;
        qcap += num_pixels(&p);
        // tile extents of the kernel: fp32 matrix cores 16 x 32 (2D) /
        // 16 x 4 x 8 (3D); vector 64 x 32 / 32 x 8 x 8 (8 pixels per lane:
        // the batched tiles build their candidate lists from every seed of
        // the instance, so fewer, larger tiles pay less for them --
        // measured); bf16 32 x 32 / 8 x 8 x 8
        const bool vec = bvariant == 1 || bvariant == 2 || bvariant == 4 || bf;
        const int e0 = vec ? apd::tile_ext(dim, btp, 0) : apd::kWaves * apd::kP;
        const int e1 = vec ? apd::tile_ext(dim, btp, 1) : (dim == 2 ? 32 : 4);
        const int e2 = 8;
        int t0 = (p.grid[0] + e0 - 1) / e0;
        int t1 = (p.grid[1] + e1 - 1) / e1;
        int t2 = dim == 2 ? 1 : (p.grid[2] + e2 - 1) / e2;
        hinst[q].tiles1 = t1;
        hinst[q].tiles2 = t2;
        hinst[q].tiles0 = t0;
        tile0[q + 1] = tile0[q] + (int64_t)t0 * t1 * t2;
    }
    // candidate lists of the tiles, kept for the re-check (lists only)
    const int64_t ntiles = tile0[B];
    const bool lists = bvariant == 2 || bvariant == 4 || bvariant == 5;
    // super-tiles about six cell diameters across ((J/N)^(1/D) pixels),
    // whole tiles, at most 8 per axis; none where that is a single tile
    std::vector<int64_t> super0(B + 1, 0);
    std::vector<std::array<int, 6>> sfn(B);
    for (int q = 0; q < B; ++q) {
        const apd_problem &p = probs[order[q]];
        int64_t cnt = 0;
        std::array<int, 6> a{1, 1, 1, 0, 0, 0};
        if (lists) {
            const double diam = pow((double)num_pixels(&p) / (double)p.n, 1.0 / dim);
            const int ext[3] = {apd::tile_ext(dim, btp, 0), apd::tile_ext(dim, btp, 1), apd::tile_ext(dim, btp, 2)};
            const int tl[3] = {hinst[q].tiles0, hinst[q].tiles1, hinst[q].tiles2};
            cnt = 1;
            for (int d = 0; d < 3; ++d) {
                const int f = d < dim ? (int)lround(6.0 * diam / ext[d]) : 1;
                a[d] = std::max(1, std::min(8, f));
                a[3 + d] = (tl[d] + a[d] - 1) / a[d];
                cnt *= a[3 + d];
            }
            if (a[0] * a[1] * a[2] == 1) cnt = 0;
        }
        sfn[q] = a;
        super0[q + 1] = super0[q] + cnt;
    }
    const int64_t nsuper = super0[B];
    size_t bytes = 0;
    const size_t o_dbl = bytes; bytes = align_up(bytes + nd * sizeof(double), 256);
    const size_t o_mom = bytes; bytes = align_up(bytes + nm * sizeof(uint64_t), 256);
    const size_t o_inst = bytes; bytes = align_up(bytes + B * sizeof(apd::BInst), 256);
    const size_t o_st = bytes; bytes = align_up(bytes + B * sizeof(apd::BState), 256);
    const size_t o_tile = bytes; bytes = align_up(bytes + (B + 1) * sizeof(int64_t), 256);
    const size_t o_ctl = bytes; bytes = align_up(bytes + sizeof(apd::BCtl), 256);
    const size_t o_dst = bytes; bytes = align_up(bytes + B * sizeof(double *), 256);
    const size_t o_q = bytes; bytes = align_up(bytes + (size_t)qcap * sizeof(uint64_t), 256);
    const size_t o_seg = bytes; bytes = align_up(bytes + (size_t)ntiles * sizeof(apd::QSeg), 256);
    const size_t o_tl = bytes;
    if (lists) bytes = align_up(bytes + (size_t)ntiles * apd::kBatchListCap * sizeof(int), 256);
    const size_t o_tc = bytes;
    if (lists) bytes = align_up(bytes + (size_t)ntiles * sizeof(int), 256);
    const size_t o_sl = bytes;
    bytes = align_up(bytes + (size_t)nsuper * apd::kBatchSuperCap * sizeof(int), 256);
    const size_t o_sc = bytes;
    bytes = align_up(bytes + (size_t)nsuper * sizeof(int), 256);
    const size_t o_s0 = bytes;
    bytes = align_up(bytes + (size_t)(B + 1) * sizeof(int64_t), 256);
    if (bytes > c->batch_bytes) {
        (void)hipFree(c->batch_buf);
        c->batch_buf = nullptr;
        c->batch_bytes = 0;
        if (hipMalloc(&c->batch_buf, bytes) != hipSuccess)
            return fail(c, APD_ERR_OOM, "cannot allocate %zu bytes of batch scratch", bytes);
        c->batch_bytes = bytes;
    }
    // a stream of its own for the captured graph (the caller's may be the
    // null stream, which cannot be captured); created per call
    if (c->batch_stream) {
        (void)hipStreamDestroy(c->batch_stream);
        c->batch_stream = nullptr;
    }
    HIP_TRY(c, hipStreamCreate(&c->batch_stream));
    hipStream_t s = c->batch_stream;
    char *base = (char *)c->batch_buf;
    double *dbl = (double *)(base + o_dbl);
    uint64_t *mom = (uint64_t *)(base + o_mom);
    apd::BInst *d_inst = (apd::BInst *)(base + o_inst);
    apd::BState *d_st = (apd::BState *)(base + o_st);
    int64_t *d_tile0 = (int64_t *)(base + o_tile);
    apd::BCtl *d_ctl = (apd::BCtl *)(base + o_ctl);
    double **d_dst = (double **)(base + o_dst);
    uint64_t *d_queue = (uint64_t *)(base + o_q);
    apd::QSeg *d_segs = (apd::QSeg *)(base + o_seg);
    int *d_tl = lists ? (int *)(base + o_tl) : nullptr;
    int *d_tc = lists ? (int *)(base + o_tc) : nullptr;
    int *d_sl = (int *)(base + o_sl);
    int *d_sc = (int *)(base + o_sc);
    int64_t *d_super0 = (int64_t *)(base + o_s0);

    std::vector<apd::BState> hst(B);
    std::vector<double *> hdst(B);
    for (int q = 0; q < B; ++q) {
        const apd_problem &p = probs[order[q]];
        apd::BInst &I = hinst[q];
        I.g = make_geo(&p);
        I.x = p.x;
        I.A = p.A;
        I.v = p.v;
        double *v0 = dbl + off_d[q];
        const size_t n = (size_t)p.n;
        I.w = v0;
        I.g_acc = v0 + n;
        I.d = v0 + 2 * n;
        I.wt = v0 + 3 * n;
        I.gt = v0 + 4 * n;
        I.S = v0 + 5 * n;
        I.Y = v0 + (5 + kBatchHist) * n;
        I.rho = v0 + (5 + 2 * kBatchHist) * n;
        I.eig = I.rho + kBatchHist;
        I.mom = mom + off_m[q];
        I.tile_lists = lists ? d_tl + tile0[q] * apd::kBatchListCap : nullptr;
        I.tile_count = lists ? d_tc + tile0[q] : nullptr;
        const bool has_super = super0[q + 1] > super0[q];
        I.super_lists = has_super ? d_sl + super0[q] * apd::kBatchSuperCap : nullptr;
        I.super_count = has_super ? d_sc + super0[q] : nullptr;
        for (int d = 0; d < 3; ++d) {
            I.sf[d] = sfn[q][d];
            I.nst[d] = std::max(1, sfn[q][3 + d]);
        }
        I.tp = btp;
        apd::BState z{};
        z.active = 1;
        z.gamma0 = o->gamma0 > 0.0 ? o->gamma0 : default_gamma0(p.dim, p.n);
        hst[q] = z;
        hdst[q] = w_inout[order[q]];
    }
    apd::BCtl hctl{};
    hctl.active = B;
    hctl.max_iter = o->max_iter;
    hctl.max_evals = o->max_evals;
    hctl.eps = o->eps;
    if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));  // inputs written by the caller
    HIP_TRY(c, hipMemcpyAsync(d_inst, hinst.data(), B * sizeof(apd::BInst), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d_st, hst.data(), B * sizeof(apd::BState), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d_tile0, tile0.data(), (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d_super0, super0.data(), (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d_ctl, &hctl, sizeof hctl, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(d_dst, hdst.data(), B * sizeof(double *), hipMemcpyHostToDevice, s));
    // the starting point: the caller's weights (warm) or W_0 = 0 (Algorithm 2)
    HIP_TRY(c, apd::launch_batch_init(d_inst, d_dst, B, o->warm != 0, s));
    HIP_TRY(c, apd::launch_batch_setup(dim, d_inst, d_st, B, s));
    HIP_TRY(c, hipMemcpyAsync(hst.data(), d_st, B * sizeof(apd::BState), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    for (int q = 0; q < B; ++q) {
        apd_status st = decode_bad(c, hst[q].bad, true);
        if (st == APD_OK) {
            const double om = box_measure(&probs[order[q]]);
            if (fabs(hst[q].vsum - om) > 1e-12 * om)
                st = fail(c, APD_ERR_VOLUMES, "target volumes sum to %.17g, the box measure is %.17g", hst[q].vsum, om);
        }
        if (st != APD_OK) return fail(c, st, "instance %d: %s", order[q], c->err.c_str());
    }
    // capture one evaluation of every active instance as a graph
    int dev_cu = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev_cu = prop.multiProcessorCount;
    }
    const int grid_assign = dev_cu * 4;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    // the re-check: one block per queue segment (a tile's queued pixels);
    // blocks past the segments leave at once
    const int recheck_blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(512, ntiles / 8));
    hipError_t le = apd::launch_batch_step(dim, d_inst, d_st, d_tile0, B, d_ctl, d_queue, d_segs,
                                           grid_assign, bvariant, recheck_blocks, d_super0, nsuper, s);
    hipError_t ce = hipStreamEndCapture(s, &graph);
    if (le != hipSuccess || ce != hipSuccess)
        return fail(c, APD_ERR_DEVICE, "graph capture failed: %s / %s", hipGetErrorString(le), hipGetErrorString(ce));
    HIP_TRY(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    hipEvent_t tev[2] = {nullptr, nullptr};
    if (trial) {
        for (auto &e : tev)
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                (void)hipGraphDestroy(graph);
                return fail(c, APD_ERR_DEVICE, "hipEventCreate failed");
            }
        (void)hipEventRecord(tev[0], s);
    }
    int replays = 0, active = B;
    const int max_replays = o->max_evals + 2;
    apd_status st = APD_OK;
    while (active > 0 && replays < max_replays) {
        for (int r = 0; r < c->batch_poll && replays < max_replays; ++r, ++replays) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { st = fail(c, APD_ERR_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e)); break; }
        }
        if (st != APD_OK) break;
        hipError_t e = hipMemcpyAsync(&hctl, d_ctl, sizeof hctl, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { st = fail(c, APD_ERR_DEVICE, "poll: %s", hipGetErrorString(e)); break; }
        active = hctl.active;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (trial) {
        // the last poll synchronised the stream after the last replay
        if (st == APD_OK && hipEventRecord(tev[1], s) == hipSuccess && hipEventSynchronize(tev[1]) == hipSuccess)
            (void)hipEventElapsedTime(&trial->replay_ms, tev[0], tev[1]);
        for (auto &e : tev) (void)hipEventDestroy(e);
    }
    if (st != APD_OK) return st;
    HIP_TRY(c, apd::launch_batch_scatter(d_inst, d_dst, B, s));
    HIP_TRY(c, hipMemcpyAsync(hst.data(), d_st, B * sizeof(apd::BState), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    int failed = 0;
    for (int q = 0; q < B; ++q) {
        const apd::BState &z = hst[q];
        const int status = z.active ? APD_ERR_NOT_CONVERGED : z.status;
        if (status != APD_OK) ++failed;
        if (reps) {
            apd_fit_report &r = reps[order[q]];
            r.converged = status == APD_OK;
            r.iters = z.iters;
            r.evals = z.evals;
            r.rechecked = 0;
            r.max_rel_err = z.crit;
            r.g = -z.f;
            r.seconds = secs;
        }
    }
    c->stats = apd_pass_stats{0, 0, 0, 0.0, 0.0, 0, batch_public_kernel(bvariant), bvariant == 0 ? 0 : btp};
    if (failed && !trial) return fail(c, APD_ERR_NOT_CONVERGED, "%d of %d instances did not converge", failed, B);
    return APD_OK;
}

}  // namespace

struct apd_ws_model {
    int device = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;  // params, grad, Adam moments
    int64_t step = 0;
    int64_t cap_S = 0;
    float *act = nullptr;   // H1, H2, H3, dA, dB [cap_S][128], y, dy [cap_S]
    double *loss_d = nullptr;
    double *h_loss = nullptr;
    unsigned short *Wb = nullptr;  // BF16 weight copies for inference
    bool bf_stale = true;          // the copies predate the parameters
};

namespace {

constexpr int kWsHid = 128;
// floats of split weight-gradient partials after the activations
constexpr size_t kWsPart = (size_t)apd::ws::kSplitMax * (kWsHid * kWsHid + kWsHid);

apd_status ws_scratch(apd_ctx *c, apd_ws_model *m, int64_t S) {
    if (S <= m->cap_S) return APD_OK;
    (void)hipFree(m->act);
    m->act = nullptr;
    m->cap_S = 0;
    if (hipMalloc(&m->act, ((size_t)S * (5 * kWsHid + 2) + kWsPart) * sizeof(float)) != hipSuccess)
        return fail(c, APD_ERR_OOM, "cannot allocate network activations for %lld samples", (long long)S);
    m->cap_S = S;
    return APD_OK;
}

struct WsBufs {
    float *H1, *H2, *H3, *dA, *dB, *y, *dy, *part;
};

WsBufs ws_bufs(apd_ws_model *m) {
    const size_t S = (size_t)m->cap_S;
    float *a = m->act;
    return WsBufs{a, a + S * kWsHid, a + 2 * S * kWsHid, a + 3 * S * kWsHid, a + 4 * S * kWsHid,
                  a + 5 * S * kWsHid, a + 5 * S * kWsHid + S, a + 5 * S * kWsHid + 2 * S};
}

// Warm-start features: one pass at W = 0 gives the deficits (gradient in
// c->gbuf), then the per-seed features and their neighbour means.
apd_status ws_features_impl(apd_ctx *c, const apd_problem *p, float *F) {
    int64_t J = 1;
    for (int d = 0; d < p->dim; ++d) J *= p->grid[d];
    apd_status st = ensure_scratch(c, p->n, J);
    if (st != APD_OK) return st;
    HIP_TRY(c, hipMemsetAsync(c->wbuf, 0, (size_t)p->n * sizeof(double), c->stream));
    double g0 = 0.0, mr0 = 0.0;
    st = evaluate(c, p, p->x, c->wbuf, APD_FP32, false, &g0, &mr0, nullptr, true);
    if (st != APD_OK) return st;
    HIP_TRY(c, apd::ws::features(c->stream, (int)p->n, p->x, p->A, p->v, p->lo, p->hi, c->gbuf, c->ws_nb,
                                 c->cbuf, F));
    return APD_OK;
}

// BF16 inference (refreshing the BF16 weight copies when stale).
apd_status ws_infer_impl(apd_ctx *c, apd_ws_model *m, const float *F, int64_t S, float *y) {
    if (m->bf_stale) {
        HIP_TRY(c, apd::ws::to_bf16_weights(c->stream, m->P, m->Wb));
        m->bf_stale = false;
    }
    HIP_TRY(c, apd::ws::infer_bf16(c->stream, m->P, m->Wb, F, (int)S, y));
    return APD_OK;
}

}  // namespace

// ------------------------------------------------ allocation-free evaluation
//
// apd_dual_objective_grad_noalloc runs the evaluation of
// apd_dual_objective_grad with all of its scratch (scalars, block partials,
// moments, eigenvalue ranges, re-check queue, candidate lists) in the static
// device array `scratch`, for callers that cannot allocate device memory.
// Every device that runs it holds one copy until the process ends; its
// address on a device is looked up once, with that device current, and kept
// in scratch_addr (host code never passes the array's own name to a kernel:
// on the host that name is only a stand-in for the symbol).
namespace {
constexpr size_t kStaticScratch = (size_t)96 << 20;  // bytes per device
constexpr int kStaticListCap = 256;                  // candidates kept per tile
constexpr int kStaticSuperCap = 512;                 // candidates kept per super-tile
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratch];

namespace {

std::mutex scratch_mu;
unsigned char *scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on c's device (which is current), looked up
// on the first call there.
apd_status static_scratch(apd_ctx *c, unsigned char **out) {
    if (c->device < 0 || c->device >= kMaxDevices)
        return fail(c, APD_ERR_DEVICE, "device %d is beyond the static scratch table", c->device);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[c->device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(c, APD_ERR_DEVICE, "static scratch: hipGetSymbolAddress failed (%s)", hipGetErrorString(e));
        scratch_addr[c->device] = static_cast<unsigned char *>(ptr);
    }
    *out = scratch_addr[c->device];
    return APD_OK;
}

// Carves 256-byte aligned regions out of a base address.
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = reinterpret_cast<T *>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

extern "C" {

apd_status apd_create(apd_ctx **out, int device, void *hip_stream) {
    if (!out) return APD_ERR_INVALID_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return APD_ERR_DEVICE;
    apd_ctx *c = new apd_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc(&c->sc, sizeof(apd::Scalars)) != hipSuccess ||
        hipMalloc(&c->parts, sizeof(apd::BlockParts)) != hipSuccess ||
        hipHostMalloc(&c->h_sc, sizeof(apd::Scalars), hipHostMallocDefault) != hipSuccess) {
        apd_destroy(c);
        return APD_ERR_OOM;
    }
    // the ticket of the block partials starts at zero (each launch leaves it so)
    if (hipMemset(c->parts, 0, sizeof(apd::BlockParts)) != hipSuccess) {
        apd_destroy(c);
        return APD_ERR_DEVICE;
    }
    *out = c;
    return APD_OK;
}

void apd_destroy(apd_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->mom);
    (void)hipFree(c->queue);
    (void)hipFree(c->sc);
    (void)hipFree(c->parts);
    (void)hipFree(c->wbuf);
    (void)hipFree(c->gbuf);
    (void)hipFree(c->cbuf);
    (void)hipFree(c->eig);
    (void)hipFree(c->ord);
    (void)hipFree(c->ws_nb);
    (void)hipFree(c->tile_lists);
    (void)hipFree(c->tile_count);
    (void)hipFree(c->tile_U);
    (void)hipFree(c->cost_part);
    (void)hipFree(c->segs);
    (void)hipFree(c->super_lists);
    (void)hipFree(c->super_count);
    (void)hipFree(c->batch_buf);
    if (c->batch_stream) (void)hipStreamDestroy(c->batch_stream);
    if (c->fit_stream) (void)hipStreamDestroy(c->fit_stream);
    for (int k = 0; k < 3; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    (void)hipHostFree(c->h_sc);
    (void)hipHostFree(c->h_grad);
    (void)hipHostFree(c->h_w);
    delete c;
}

const char *apd_last_error(const apd_ctx *c) { return c ? c->err.c_str() : "no context"; }

apd_status apd_set_stream(apd_ctx *c, void *hip_stream) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->stream = (hipStream_t)hip_stream;
    return APD_OK;
}

apd_status apd_assign(apd_ctx *c, const apd_problem *p, const double *w, int32_t *labels,
                      float *rel_gap, apd_precision prec) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, false);
    if (st != APD_OK) return st;
    if (!w || !labels) return fail(c, APD_ERR_INVALID_ARG, "w and labels must be device pointers");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    apd::FinalOut fo{nullptr, nullptr, nullptr};
    st = enqueue_pass(c, p, p->x, w, labels, false, false, fo, prec, nullptr, rel_gap);
    if (st != APD_OK) return st;
    st = sync_scalars(c);
    if (st != APD_OK) return st;
    return decode_bad(c, c->h_sc->bad, false);
}

apd_status apd_dual_objective_grad(apd_ctx *c, const apd_problem *p, const double *w, double *g,
                                   double *grad, int64_t *counts, double *centroids,
                                   double *maxrel, apd_precision prec) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w || !g || !grad) return fail(c, APD_ERR_INVALID_ARG, "w, g and grad are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    apd::FinalOut fo{grad, counts, centroids};
    return evaluate(c, p, p->x, w, prec, false, g, maxrel, &fo, true);
}

apd_status apd_dual_objective_grad_noalloc(apd_ctx *c, const apd_problem *p, const double *w, double *g,
                                           double *grad, int64_t *counts, double *centroids,
                                           double *maxrel, apd_precision prec) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w || !g || !grad) return fail(c, APD_ERR_INVALID_ARG, "w, g and grad are required");
    if (prec != APD_FP64 && prec != APD_FP32 && prec != APD_BF16)
        return fail(c, APD_ERR_INVALID_ARG, "precision %d is not available", (int)prec);
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    unsigned char *base = nullptr;
    st = static_scratch(c, &base);
    if (st != APD_OK) return st;
    // the layout of this problem's buffers in the static array
    apd::Geo geo = make_geo(p);
    geo.vec_p = c->vec_p;
    const int64_t n = p->n, J = num_pixels(p);
    const bool cull = c->culling && ((prec == APD_FP32 && c->variant >= 1) || prec == APD_BF16);
    Carve k{base};
    PassBufs b;
    b.sc = k.take<apd::Scalars>(1);
    b.parts = k.take<apd::BlockParts>(1);
    b.mom = k.take<uint64_t>((size_t)n * 10);
    b.eig = k.take<double>((size_t)n * 2);
    b.ord = k.take<int>((size_t)n);
    b.queue = k.take<unsigned>((size_t)J);
    if (geo.power != 2) {
        b.cap_parts = apd::fp64_blocks(geo);
        b.cost_part = k.take<double>((size_t)b.cap_parts);
    }
    if (cull) {
        const ListGeometry L = list_geometry(p, geo, prec);
        b.tile_lists = k.take<int>((size_t)L.tiles * kStaticListCap);
        b.tile_count = k.take<int>((size_t)L.tiles);
        b.tile_U = k.take<double>((size_t)L.tiles);
        b.segs = k.take<apd::QSeg>((size_t)L.tiles);
        b.cap_tiles = L.tiles;
        b.list_cap = kStaticListCap;
        b.super_lists = k.take<int>((size_t)L.nsuper * kStaticSuperCap);
        b.super_count = k.take<int>((size_t)L.nsuper);
        b.cap_super = L.nsuper;
        b.super_cap = kStaticSuperCap;
    }
    if (k.off > kStaticScratch)
        return fail(c, APD_ERR_OOM,
                    "this problem needs %zu bytes of scratch; the static array holds %zu (n = %lld, J = %lld)",
                    k.off, kStaticScratch, (long long)n, (long long)J);
    // the block partials' ticket must start at zero (each launch leaves it
    // so; the array starts zeroed, but an aborted call may not have)
    HIP_TRY(c, apd::launch_zero(b.parts, sizeof(apd::BlockParts), c->stream));
    apd::FinalOut fo{grad, counts, centroids};
    c->need_qtotal = true;
    st = enqueue_pass(c, p, p->x, w, nullptr, true, true, fo, prec, nullptr, nullptr, &b);
    c->need_qtotal = false;
    if (st != APD_OK) return st;
    // the scalars into the context's pinned copy (allocated with the context)
    HIP_TRY(c, hipMemcpyAsync(c->h_sc, b.sc, sizeof(apd::Scalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->stats.rechecked = c->h_sc->qcount;
    c->stats.tiles_credited = c->h_sc->credited;
    st = decode_bad(c, c->h_sc->bad, true);
    if (st != APD_OK) return st;
    st = check_volumes(c, p);
    if (st != APD_OK) return st;
    *g = c->h_sc->g;
    if (maxrel) *maxrel = c->h_sc->maxrel;
    return APD_OK;
}

apd_status apd_fit_weights(apd_ctx *c, const apd_problem *p, double *w_inout,
                           const apd_fit_opts *o, apd_fit_report *rep) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w_inout || !o) return fail(c, APD_ERR_INVALID_ARG, "w_inout and opts are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    const auto t0 = std::chrono::steady_clock::now();
    apd_fit_opts of = *o;
    int32_t coarse_evals = 0, coarse_iters = 0;
    if (o->coarse_eps > 0.0 && !p->mass) {
        // coarse-to-fine start: the same seeds on the grid halved along every
        // axis, fitted to the looser tolerance; its weights (reached, or the
        // best iterate) start the fit on the problem's grid
        apd_problem qc = *p;
        for (int d = 0; d < p->dim; ++d) qc.grid[d] = (p->grid[d] + 1) / 2;
        st = check_problem(c, &qc, true);
        if (st != APD_OK) return st;
        apd_fit_opts oc = *o;
        oc.eps = o->coarse_eps;
        oc.max_evals = std::max(1, o->max_evals / 4);
        oc.refine = 0;
        oc.coarse_eps = 0.0;
        apd_fit_report rc{};
        st = fit_impl(c, &qc, qc.x, w_inout, &oc, &rc);
        if (st != APD_OK && st != APD_ERR_NOT_CONVERGED && st != APD_ERR_LINESEARCH) return st;
        c->err.clear();
        coarse_evals = rc.evals;
        coarse_iters = rc.iters;
        of.warm = 1;
    }
    apd_fit_report r0{};
    st = fit_impl(c, p, p->x, w_inout, &of, &r0);
    r0.evals += coarse_evals;
    r0.iters += coarse_iters;
    // the last step of Algorithm 2: refine the grid and restart from the
    // weights reached while the tolerance is out of reach
    apd_problem q = *p;
    int refined = 0;
    while ((st == APD_ERR_NOT_CONVERGED || st == APD_ERR_LINESEARCH) && refined < o->refine && !p->mass) {
        std::vector<double> v((size_t)p->n);
        HIP_TRY(c, hipMemcpyAsync(v.data(), p->v, v.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const double vmin = *std::min_element(v.begin(), v.end());
        const double target = o->eps * vmin / pow(2.0, (double)p->dim);
        double pix = 1.0;
        for (int d = 0; d < p->dim; ++d) pix *= (q.hi[d] - q.lo[d]) / (double)q.grid[d];
        double f = pow(pix / target, 1.0 / (double)p->dim);
        if (!(f > 1.5)) f = 1.5;
        for (int d = 0; d < p->dim; ++d) {
            const double m = ceil((double)q.grid[d] * f);
            if (m > 2147483647.0) return fail(c, APD_ERR_INVALID_ARG, "refined grid too large");
            q.grid[d] = (int32_t)m;
        }
        st = check_problem(c, &q, true);
        if (st != APD_OK) return st;
        apd_fit_opts o2 = of;
        o2.warm = 1;
        apd_fit_report r2{};
        c->err.clear();
        st = fit_impl(c, &q, q.x, w_inout, &o2, &r2);
        r2.iters += r0.iters;
        r2.evals += r0.evals;
        r0 = r2;
        ++refined;
    }
    if (rep) {
        *rep = r0;
        for (int d = 0; d < 3; ++d) rep->grid[d] = d < p->dim ? q.grid[d] : 1;
        rep->refinements = refined;
        rep->coarse_evals = coarse_evals;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

apd_status apd_lloyd_step(apd_ctx *c, const apd_problem *p, double *x_inout, double *w_inout,
                          const apd_fit_opts *o, apd_fit_report *rep) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_problem q = p ? *p : apd_problem{};
    q.x = x_inout;
    apd_status st = check_problem(c, &q, true);
    if (st != APD_OK) return st;
    if (!w_inout || !o) return fail(c, APD_ERR_INVALID_ARG, "w_inout and opts are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    apd_fit_opts ow = *o;
    ow.warm = 1;  // W_0^{k+1} = W^k
    const apd_status fs = fit_impl(c, &q, x_inout, w_inout, &ow, rep);
    if (fs != APD_OK && fs != APD_ERR_NOT_CONVERGED) return fs;
    const std::string fit_msg = c->err;
    // centroids of the cells at the fitted weights
    double g = 0.0;
    apd::FinalOut fo{nullptr, nullptr, c->cbuf};
    st = evaluate(c, &q, x_inout, w_inout, o->prec, false, &g, nullptr, &fo, false);
    if (st != APD_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(x_inout, c->cbuf, (size_t)q.n * q.dim * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->err = fit_msg;
    return fs;
}

apd_status apd_fit_weights_batched(apd_ctx *c, const apd_problem *probs, int32_t B,
                                   double *const *w_inout, const apd_fit_opts *o,
                                   apd_fit_report *reps) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    if (!probs || B < 1 || !w_inout || !o) return fail(c, APD_ERR_INVALID_ARG, "bad batch arguments");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    return fit_batched_impl(c, probs, B, w_inout, o, reps);
}

apd_status apd_ws_create(apd_ctx *c, apd_ws_model **out, const float *params, int64_t n_params) {
    if (!c || !out) return APD_ERR_INVALID_ARG;
    c->err.clear();
    *out = nullptr;
    if (!params || n_params != apd::ws::kParamCount)
        return fail(c, APD_ERR_INVALID_ARG, "the network has %lld parameters (got %lld)",
                    (long long)apd::ws::kParamCount, (long long)n_params);
    apd_ws_model *m = new apd_ws_model();
    m->device = c->device;
    const size_t bytes = (size_t)n_params * sizeof(float);
    if (hipMalloc(&m->P, bytes) != hipSuccess || hipMalloc(&m->G, bytes) != hipSuccess ||
        hipMalloc(&m->M, bytes) != hipSuccess || hipMalloc(&m->V, bytes) != hipSuccess ||
        hipMalloc(&m->loss_d, sizeof(double)) != hipSuccess ||
        hipMalloc(&m->Wb, (size_t)apd::ws::kBf16Count * sizeof(unsigned short)) != hipSuccess ||
        hipHostMalloc(&m->h_loss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        apd_ws_destroy(m);
        return fail(c, APD_ERR_OOM, "cannot allocate the network");
    }
    HIP_TRY(c, hipMemcpyAsync(m->P, params, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(m->M, 0, bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(m->V, 0, bytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(m->G, 0, bytes, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *out = m;
    return APD_OK;
}

void apd_ws_destroy(apd_ws_model *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(m->P);
    (void)hipFree(m->G);
    (void)hipFree(m->M);
    (void)hipFree(m->V);
    (void)hipFree(m->act);
    (void)hipFree(m->loss_d);
    (void)hipFree(m->Wb);
    (void)hipHostFree(m->h_loss);
    delete m;
}

apd_status apd_ws_get_params(apd_ctx *c, const apd_ws_model *m, float *params, int64_t n_params) {
    if (!c || !m || !params || n_params != apd::ws::kParamCount) return APD_ERR_INVALID_ARG;
    HIP_TRY(c, hipMemcpyAsync(params, m->P, (size_t)n_params * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_ws_features(apd_ctx *c, const apd_problem *p, float *F) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (p->dim != 2) return fail(c, APD_ERR_INVALID_ARG, "the warm start is defined in 2D");
    if (!F) return fail(c, APD_ERR_INVALID_ARG, "F is NULL");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    st = ws_features_impl(c, p, F);
    if (st != APD_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_ws_targets(apd_ctx *c, int64_t n, const double *w, float *t) {
    if (!c || n < 1 || n > 0x7fffffff || !w || !t) return APD_ERR_INVALID_ARG;
    c->err.clear();
    HIP_TRY(c, apd::ws::targets(c->stream, (int)n, w, t));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_ws_forward(apd_ctx *c, apd_ws_model *m, const float *F, int64_t S, float *y) {
    if (!c || !m || !F || !y || S < 1 || S > 0x7fffffff) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = ws_scratch(c, m, S);
    if (st != APD_OK) return st;
    WsBufs b = ws_bufs(m);
    HIP_TRY(c, apd::ws::forward(c->stream, m->P, F, (int)S, b.H1, b.H2, b.H3, y));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_ws_infer(apd_ctx *c, apd_ws_model *m, const float *F, int64_t S, float *y) {
    if (!c || !m || !F || !y || S < 1 || S > 0x7fffffff) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = ws_infer_impl(c, m, F, S, y);
    if (st != APD_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_ws_loss_grad(apd_ctx *c, apd_ws_model *m, const float *F, const float *t, int64_t S,
                            double *loss, float *grad) {
    if (!c || !m || !F || !t || S < 1 || S > 0x7fffffff) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = ws_scratch(c, m, S);
    if (st != APD_OK) return st;
    WsBufs b = ws_bufs(m);
    HIP_TRY(c, apd::ws::backward(c->stream, m->P, F, t, (int)S, b.H1, b.H2, b.H3, b.y, b.dy, b.dA, b.dB,
                                 m->G, m->loss_d, b.part));
    if (grad)
        HIP_TRY(c, hipMemcpyAsync(grad, m->G, (size_t)apd::ws::kParamCount * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(m->h_loss, m->loss_d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = *m->h_loss;
    return APD_OK;
}

apd_status apd_ws_train_step(apd_ctx *c, apd_ws_model *m, const float *F, const float *t, int64_t S,
                             float lr, double *loss) {
    if (!c || !m || !F || !t || S < 1 || S > 0x7fffffff || !(lr > 0.0f)) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = ws_scratch(c, m, S);
    if (st != APD_OK) return st;
    WsBufs b = ws_bufs(m);
    HIP_TRY(c, apd::ws::backward(c->stream, m->P, F, t, (int)S, b.H1, b.H2, b.H3, b.y, b.dy, b.dA, b.dB,
                                 m->G, m->loss_d, b.part));
    m->step += 1;
    HIP_TRY(c, apd::ws::adam(c->stream, m->P, m->G, m->M, m->V, lr, m->step));
    m->bf_stale = true;
    if (loss) {
        HIP_TRY(c, hipMemcpyAsync(m->h_loss, m->loss_d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        *loss = *m->h_loss;
    }
    return APD_OK;
}

apd_status apd_ws_train_epoch(apd_ctx *c, apd_ws_model *m, const float *F, const float *t, int64_t S,
                              float lr, double *loss) {
    if (!c || !m || !F || !t || S < 1 || !(lr > 0.0f)) return APD_ERR_INVALID_ARG;
    c->err.clear();
    constexpr int64_t kBatch = 4096;  // samples per Adam step
    constexpr int64_t kFeat = 20;     // features per sample
    double tot = 0.0;
    for (int64_t k = 0; k < S; k += kBatch) {
        const int64_t sb = std::min<int64_t>(kBatch, S - k);
        double l = 0.0;
        const apd_status st = apd_ws_train_step(c, m, F + k * kFeat, t + k, sb, lr, loss ? &l : nullptr);
        if (st != APD_OK) return st;
        tot += l * (double)sb;
    }
    if (loss) *loss = tot / (double)S;
    return APD_OK;
}

apd_status apd_ws_predict(apd_ctx *c, apd_ws_model *m, const apd_problem *p, double *w_out) {
    if (!c || !m) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (p->dim != 2) return fail(c, APD_ERR_INVALID_ARG, "the warm start is defined in 2D");
    if (!w_out) return fail(c, APD_ERR_INVALID_ARG, "w_out is NULL");
    const int64_t n = p->n;
    st = ws_scratch(c, m, n + 16 * ((n + 127) / 128 + 1));
    if (st != APD_OK) return st;
    WsBufs b = ws_bufs(m);
    float *F = b.dA;  // features in the gradient scratch ([n][20] fits in [n][128])
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    st = ws_features_impl(c, p, F);
    if (st != APD_OK) return st;
    st = ws_infer_impl(c, m, F, n, b.y);
    if (st != APD_OK) return st;
    HIP_TRY(c, apd::ws::center(c->stream, (int)n, b.y, w_out));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return APD_OK;
}

apd_status apd_fit_weights_ws(apd_ctx *c, apd_ws_model *m, const apd_problem *p, double *w_out,
                              const apd_fit_opts *o, apd_fit_report *rep, int32_t *used_warm) {
    if (!c || !o) return APD_ERR_INVALID_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    apd_status st = apd_ws_predict(c, m, p, w_out);
    if (st != APD_OK) return st;
    apd_fit_opts ow = *o;
    ow.warm = 1;
    st = apd_fit_weights(c, p, w_out, &ow, rep);
    if (rep) rep->evals += 1;  // the pass at W = 0 that made the features
    if (used_warm) *used_warm = 1;
    if (st == APD_ERR_NOT_CONVERGED || st == APD_ERR_LINESEARCH) {
        // the cold start stays the fallback and certifies the result
        ow.warm = 0;
        apd_fit_report r2{};
        st = apd_fit_weights(c, p, w_out, &ow, &r2);
        if (rep) {
            r2.iters += rep->iters;
            r2.evals += rep->evals;
            *rep = r2;
        }
        if (used_warm) *used_warm = 0;
    }
    if (rep) rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

apd_status apd_choose_resolution(int32_t dim, double eps, double vmin, double omega, int32_t *M) {
    if (!M || (dim != 2 && dim != 3) || !(eps > 0.0) || !(vmin > 0.0) || !(omega > 0.0))
        return APD_ERR_INVALID_ARG;
    // smallest M with omega / M^dim < eps vmin / 2^dim; ties (within a
    // relative 1e-12) are equality and rejected
    const double rhs = eps * vmin / (double)(1 << dim) * (1.0 - 1e-12);
    double m = floor(pow(omega / rhs, 1.0 / dim)) - 2.0;
    if (m < 1.0) m = 1.0;
    while (!(omega / pow(m, (double)dim) < rhs)) m += 1.0;
    if (m > 2147483647.0) return APD_ERR_INVALID_ARG;
    *M = (int32_t)m;
    return APD_OK;
}

apd_status apd_set_profiling(apd_ctx *c, int32_t on) {
    if (!c) return APD_ERR_INVALID_ARG;
    if (on && !c->ev[0]) {
        for (int k = 0; k < 3; ++k)
            if (hipEventCreate(&c->ev[k]) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipEventCreate failed");
    }
    c->profiling = on != 0;
    return APD_OK;
}

apd_status apd_set_variant(apd_ctx *c, int32_t variant) {
    if (!c || variant < 0 || variant > 3) return APD_ERR_INVALID_ARG;
    c->variant = variant;
    return APD_OK;
}

apd_status apd_autotune(apd_ctx *c, const apd_problem *p, const double *w, apd_precision prec,
                        int32_t reps, apd_tune_result *res) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w || !res || reps < 1) return fail(c, APD_ERR_INVALID_ARG, "w, res and reps >= 1 are required");
    if (prec != APD_FP32) return fail(c, APD_ERR_INVALID_ARG, "only the APD_FP32 tier has kernel variants");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    // candidates: (variant, culling, pixels per lane)
    constexpr int kCand = 6;
    const int cand[kCand][3] = {{1, 1, 4}, {1, 1, 8}, {1, 0, 4}, {1, 0, 8}, {0, 0, 0}, {3, 0, 0}};
    const int save_v = c->variant, save_pp = c->vec_p;
    const bool save_c = c->culling, save_p = c->profiling;
    st = apd_set_profiling(c, 1);
    if (st != APD_OK) return st;
    int best = -1;
    for (int k = 0; k < kCand; ++k) {
        c->variant = cand[k][0];
        c->culling = cand[k][1] != 0;
        c->vec_p = cand[k][2];
        double g = 0.0, tot = 0.0;
        apd::FinalOut fo{nullptr, nullptr, nullptr};
        st = evaluate(c, p, p->x, w, prec, false, &g, nullptr, &fo, k == 0);  // warm-up
        for (int r = 0; st == APD_OK && r < reps; ++r) {
            st = evaluate(c, p, p->x, w, prec, false, &g, nullptr, &fo, false);
            tot += c->stats.pass_ms;
        }
        if (st != APD_OK) {
            c->variant = save_v;
            c->culling = save_c;
            c->vec_p = save_pp;
            c->profiling = save_p;
            return st;
        }
        res->pass_ms[k] = tot / reps;
        if (best < 0 || res->pass_ms[k] < res->pass_ms[best]) best = k;
    }
    res->variant = cand[best][0];
    res->culling = cand[best][1];
    res->pixels_per_lane = cand[best][2];
    res->reserved = 0;
    c->variant = res->variant;
    c->culling = res->culling != 0;
    c->vec_p = res->pixels_per_lane;
    c->profiling = save_p;
    return APD_OK;
}

apd_status apd_autotune_batched(apd_ctx *c, const apd_problem *probs, int32_t B, int32_t evals,
                                apd_tune_batched_result *res) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    (void)hipGetLastError();
    if (!probs || B < 1 || !res || evals < 1) return fail(c, APD_ERR_INVALID_ARG, "probs, B >= 1, res and evals >= 1 are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    int64_t total = 0;
    for (int b = 0; b < B; ++b) {
        apd_status st = check_problem(c, &probs[b], true);
        if (st != APD_OK) return fail(c, st, "instance %d: %s", b, c->err.c_str());
        total += probs[b].n;
    }
    // trial weights: one buffer of this call
    double *wbuf = nullptr;
    if (hipMalloc(&wbuf, (size_t)total * sizeof(double)) != hipSuccess)
        return fail(c, APD_ERR_OOM, "cannot allocate %lld trial weights", (long long)total);
    std::vector<double *> wp(B);
    for (int b = 0, off = 0; b < B; off += (int)probs[b].n, ++b) wp[b] = wbuf + off;
    // candidates (kb_assign's V) in the order of fit_ms
    constexpr int kCand = 6;
    const int cand[kCand] = {4, 2, 1, 0, 5, 3};
    apd_fit_opts o{};
    o.eps = 1e-300;  // no instance stops before its evaluation budget
    o.max_iter = 1 << 30;
    o.history = 10;
    o.warm = 0;
    o.prec = APD_FP32;
    apd_status st = APD_OK;
    int best = -1;
    for (int k = 0; k < kCand && st == APD_OK; ++k) {
        BatchTrial t{cand[k], 0.0f};
        o.max_evals = 1;  // untimed: first launches of the candidate's kernels
        st = fit_batched_impl(c, probs, B, wp.data(), &o, nullptr, &t);
        if (st != APD_OK) break;
        o.max_evals = evals;
        t.replay_ms = 0.0f;
        st = fit_batched_impl(c, probs, B, wp.data(), &o, nullptr, &t);
        res->fit_ms[k] = t.replay_ms;
        if (st == APD_OK && (best < 0 || res->fit_ms[k] < res->fit_ms[best])) best = k;
    }
    (void)hipFree(wbuf);
    if (st != APD_OK) return st;
    c->batch_kernel = cand[best];
    res->kernel = c->stats.kernel = batch_public_kernel(cand[best]);
    const int dim = probs[0].dim;
    res->pixels_per_lane = cand[best] == 0 ? 0 : cand[best] == 4 ? apd::kP : (cand[best] == 3 || cand[best] == 5) ? (dim == 2 ? 4 : 2) : 8;
    c->stats.pixels_per_lane = res->pixels_per_lane;
    return APD_OK;
}

apd_status apd_set_batch_kernel(apd_ctx *c, int32_t kernel, int32_t pixels_per_lane) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    switch (kernel) {
    case -1: c->batch_kernel = -1; return APD_OK;
    case APD_KERNEL_FP32_MATRIX: c->batch_kernel = 0; return APD_OK;
    case APD_KERNEL_FP32_VECTOR: c->batch_kernel = 1; return APD_OK;
    case APD_KERNEL_FP32_LISTS:
        if (pixels_per_lane != 4 && pixels_per_lane != 8)
            return fail(c, APD_ERR_INVALID_ARG, "the listed vector kernel takes 4 or 8 pixels per lane");
        c->batch_kernel = pixels_per_lane == 4 ? 4 : 2;
        return APD_OK;
    case APD_KERNEL_BF16_MATRIX: c->batch_kernel = 3; return APD_OK;
    case APD_KERNEL_BF16_LISTS: c->batch_kernel = 5; return APD_OK;
    default: return fail(c, APD_ERR_INVALID_ARG, "kernel %d has no batched form", (int)kernel);
    }
}

apd_status apd_set_pixels_per_lane(apd_ctx *c, int32_t p) {
    if (!c) return APD_ERR_INVALID_ARG;
    if (p != 0 && p != 4 && p != 8) return fail(c, APD_ERR_INVALID_ARG, "pixels per lane must be 0, 4 or 8");
    c->vec_p = p;
    return APD_OK;
}

apd_status apd_set_adaptive(apd_ctx *c, int32_t on) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->adaptive = on != 0;
    return APD_OK;
}

apd_status apd_set_culling(apd_ctx *c, int32_t on) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->culling = on != 0;
    return APD_OK;
}

apd_status apd_last_pass_stats(const apd_ctx *c, apd_pass_stats *out) {
    if (!c || !out) return APD_ERR_INVALID_ARG;
    *out = c->stats;
    return APD_OK;
}

}  // extern "C"
