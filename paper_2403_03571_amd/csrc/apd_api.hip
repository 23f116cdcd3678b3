// apd_api.hip -- the C ABI of libapd (include/apd.h): validation, scratch,
// the evaluation pass, the L-BFGS weight solver (Algorithm 2 of
// arXiv 2403.03571) and the generalised Lloyd step (Algorithm 3).
#include "../../include/apd.h"
#include "apd_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
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
    double *wbuf = nullptr;           // [cap_n] trial weights of the solver
    double *gbuf = nullptr;           // [cap_n] gradient of the solver
    double *cbuf = nullptr;           // [cap_n][3] centroids of the Lloyd step
    // pinned host staging
    apd::Scalars *h_sc = nullptr;
    double *h_grad = nullptr;         // [cap_n]
    apd_pass_stats stats{0, 0, 0, 0.0, 0.0};
    // HIP-event timing of the passes
    bool profiling = false;
    int variant = 0;  // single-precision kernel: 0 = matrix cores, 1 = vector ALU
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

namespace {

apd_status fail(apd_ctx *c, apd_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
apd_status fail(apd_ctx *c, apd_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
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
    return g;
}

apd_status ensure_scratch(apd_ctx *c, int64_t n, int64_t J) {
    if (n > c->cap_n) {
        (void)hipFree(c->mom); c->mom = nullptr;
        (void)hipFree(c->wbuf); c->wbuf = nullptr;
        (void)hipFree(c->gbuf); c->gbuf = nullptr;
        (void)hipFree(c->cbuf); c->cbuf = nullptr;
        (void)hipHostFree(c->h_grad); c->h_grad = nullptr;
        c->cap_n = 0;
        const int64_t nn = std::max<int64_t>(n, 1024);
        if (hipMalloc(&c->mom, (size_t)nn * 10 * sizeof(uint64_t)) != hipSuccess ||
            hipMalloc(&c->wbuf, (size_t)nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->gbuf, (size_t)nn * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->cbuf, (size_t)nn * 3 * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&c->h_grad, (size_t)nn * sizeof(double), hipHostMallocDefault) != hipSuccess)
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

// Enqueue one evaluation pass: prep, assignment (+ re-check), optional finalize.
apd_status enqueue_pass(apd_ctx *c, const apd_problem *p, const double *x, const double *w,
                        int32_t *labels, bool moments, bool finalize, const apd::FinalOut &fo,
                        apd_precision prec) {
    const apd::Geo g = make_geo(p);
    const int64_t J = num_pixels(p);
    apd_status st = ensure_scratch(c, p->n, J);
    if (st != APD_OK) return st;
    apd::Seeds sd{x, p->A, w, p->v};
    uint64_t *mom = moments ? c->mom : nullptr;
    if (prec != APD_FP64 && prec != APD_FP32)
        return fail(c, APD_ERR_INVALID_ARG, "precision %d is not available", (int)prec);
    if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, apd::launch_prep(g, sd, c->sc, mom, c->stream));
    if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    apd::PassOut out{labels, mom, nullptr};
    if (prec == APD_FP64) {
        HIP_TRY(c, apd::launch_assign_fp64(g, sd, c->sc, out, c->stream));
        if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
    } else {
        out.queue = c->queue;
        if (c->variant == 1) HIP_TRY(c, apd::launch_assign_fp32(g, sd, c->sc, out, c->stream));
        else HIP_TRY(c, apd::launch_assign_mfma(g, sd, c->sc, out, c->stream));
        if (c->profiling) HIP_TRY(c, hipEventRecord(c->ev[2], c->stream));
        HIP_TRY(c, apd::launch_recheck(g, sd, c->sc, out, c->stream));
    }
    if (finalize) HIP_TRY(c, apd::launch_finalize(g, sd, c->mom, c->sc, fo, c->stream));
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

apd_status check_volumes(apd_ctx *c, const apd_problem *p) {
    const double om = box_measure(p);
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
    apd_status st = enqueue_pass(c, p, x, w, nullptr, true, true, fo, prec);
    if (st != APD_OK) return st;
    if (host_grad)
        HIP_TRY(c, hipMemcpyAsync(c->h_grad, fo.grad, (size_t)p->n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    st = sync_scalars(c);
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
struct Lbfgs {
    int64_t n;
    int m;
    std::vector<std::vector<double>> S, Y;
    std::vector<double> rho;

    static double dot(const std::vector<double> &a, const std::vector<double> &b) {
        double s = 0.0;
        for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
        return s;
    }
    void clear() { S.clear(); Y.clear(); rho.clear(); }
    void push(std::vector<double> s, std::vector<double> y, double sy) {
        if ((int)S.size() == m) {
            S.erase(S.begin());
            Y.erase(Y.begin());
            rho.erase(rho.begin());
        }
        S.push_back(std::move(s));
        Y.push_back(std::move(y));
        rho.push_back(1.0 / sy);
    }
    // d = -H grad
    void direction(const std::vector<double> &grad, double gamma0, std::vector<double> &d) const {
        const size_t k = S.size();
        if (k == 0) {
            for (int64_t i = 0; i < n; ++i) d[i] = -gamma0 * grad[i];
            return;
        }
        std::vector<double> q(grad), alpha(k);
        for (size_t t = k; t-- > 0;) {
            alpha[t] = rho[t] * dot(S[t], q);
            for (int64_t i = 0; i < n; ++i) q[i] -= alpha[t] * Y[t][i];
        }
        const double gamma = dot(S[k - 1], Y[k - 1]) / dot(Y[k - 1], Y[k - 1]);
        for (int64_t i = 0; i < n; ++i) q[i] *= gamma;
        for (size_t t = 0; t < k; ++t) {
            const double beta = rho[t] * dot(Y[t], q);
            for (int64_t i = 0; i < n; ++i) q[i] += S[t][i] * (alpha[t] - beta);
        }
        for (int64_t i = 0; i < n; ++i) d[i] = -q[i];
    }
};

void project_mean(std::vector<double> &g) {
    double s = 0.0;
    for (double v : g) s += v;
    s /= (double)g.size();
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

    // evaluate at host weights `ww`: upload, pass, download grad f = -grad g~
    auto eval = [&](const std::vector<double> &ww, std::vector<double> &gf, double &f, double &crit,
                    bool validate) -> apd_status {
        hipError_t e = hipMemcpyAsync(c->wbuf, ww.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return fail(c, APD_ERR_DEVICE, "upload of w: %s", hipGetErrorString(e));
        double g;
        apd_status s2 = evaluate(c, p, x, c->wbuf, o->prec, true, &g, &crit, nullptr, validate);
        if (s2 != APD_OK) return s2;
        for (int64_t i = 0; i < n; ++i) gf[i] = -c->h_grad[i];
        f = -g;
        return APD_OK;
    };

    Lbfgs lb{n, std::max(o->history, 1), {}, {}, {}};
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
                if (!lb.S.empty()) { lb.clear(); continue; }
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
                if (!lb.S.empty()) { lb.clear(); continue; }
                result = APD_ERR_LINESEARCH;
                break;
            }
            project_mean(gt);
            std::vector<double> s(n), y(n);
            for (int64_t i = 0; i < n; ++i) { s[i] = wt[i] - w[i]; y[i] = gt[i] - gr[i]; }
            const double sy = Lbfgs::dot(s, y);
            const double ns = sqrt(Lbfgs::dot(s, s)), ny = sqrt(Lbfgs::dot(y, y));
            if (sy > 1e-10 * ns * ny) lb.push(std::move(s), std::move(y), sy);
            w = wt; gr = gt; f = ft; crit = critt; ++iters;
        }
    }
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
        hipHostMalloc(&c->h_sc, sizeof(apd::Scalars), hipHostMallocDefault) != hipSuccess) {
        apd_destroy(c);
        return APD_ERR_OOM;
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
    (void)hipFree(c->wbuf);
    (void)hipFree(c->gbuf);
    (void)hipFree(c->cbuf);
    for (int k = 0; k < 3; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    (void)hipHostFree(c->h_sc);
    (void)hipHostFree(c->h_grad);
    delete c;
}

const char *apd_last_error(const apd_ctx *c) { return c ? c->err.c_str() : "no context"; }

apd_status apd_set_stream(apd_ctx *c, void *hip_stream) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->stream = (hipStream_t)hip_stream;
    return APD_OK;
}

apd_status apd_assign(apd_ctx *c, const apd_problem *p, const double *w, int32_t *labels,
                      apd_precision prec) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = check_problem(c, p, false);
    if (st != APD_OK) return st;
    if (!w || !labels) return fail(c, APD_ERR_INVALID_ARG, "w and labels must be device pointers");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    apd::FinalOut fo{nullptr, nullptr, nullptr};
    st = enqueue_pass(c, p, p->x, w, labels, false, false, fo, prec);
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
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w || !g || !grad) return fail(c, APD_ERR_INVALID_ARG, "w, g and grad are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    apd::FinalOut fo{grad, counts, centroids};
    return evaluate(c, p, p->x, w, prec, false, g, maxrel, &fo, true);
}

apd_status apd_fit_weights(apd_ctx *c, const apd_problem *p, double *w_inout,
                           const apd_fit_opts *o, apd_fit_report *rep) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
    apd_status st = check_problem(c, p, true);
    if (st != APD_OK) return st;
    if (!w_inout || !o) return fail(c, APD_ERR_INVALID_ARG, "w_inout and opts are required");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, APD_ERR_DEVICE, "hipSetDevice failed");
    return fit_impl(c, p, p->x, w_inout, o, rep);
}

apd_status apd_lloyd_step(apd_ctx *c, const apd_problem *p, double *x_inout, double *w_inout,
                          const apd_fit_opts *o, apd_fit_report *rep) {
    if (!c) return APD_ERR_INVALID_ARG;
    c->err.clear();
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
    if (!c || variant < 0 || variant > 1) return APD_ERR_INVALID_ARG;
    c->variant = variant;
    return APD_OK;
}

apd_status apd_last_pass_stats(const apd_ctx *c, apd_pass_stats *out) {
    if (!c || !out) return APD_ERR_INVALID_ARG;
    *out = c->stats;
    return APD_OK;
}

}  // extern "C"
