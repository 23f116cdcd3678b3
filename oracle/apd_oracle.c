/*
 * apd_oracle.c -- plain CPU FP64 reference of the APD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against; it is never part of the product path.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header or table with the HIP library.
 *
 * What it follows (Buze, Feydy, Roper, Sedighiani, Bourne, "Anisotropic
 * power diagrams for polycrystal modelling", arXiv 2403.03571):
 *   - the APD cell, Section 2.1 eq. (2.1), evaluated at pixel centres;
 *   - the regular pixel grid of Section 2.3 eq. (2.6);
 *   - Algorithm 1 (pixel method): cost C_ij = |y_j - x_i|^2_{A_i} - w_i,
 *     H_j = argmin_i C_ij;
 *   - the discretised dual objective, eq. (2.7), and its gradient
 *     v_i - m_i |P|, eq. (2.8);
 *   - the stopping rule of Algorithm 2, |v_i - m_i |P|| < eps v_i;
 *   - Algorithm 2 (L-BFGS maximisation of the objective from W_0 = 0);
 *   - Algorithm 3 (generalised Lloyd: discrete centroids, warm refit);
 *   - the resolution rules (2.9) and (2.10) of Section 2.3.1;
 *   - the general tessellation of Section 2.3 (the objective with a measure
 *     |P_j| per cell of the discretisation), restricted to the regular grid:
 *     pixel j has measure (q_j / 255) |P| with an integer weight q_j in
 *     [0, 255] (0: outside the domain, 255: a full pixel);
 *   - the last step of Algorithm 2: when the tolerance cannot be reached,
 *     refine the discretisation and restart;
 *   - costs beyond the squared anisotropic norm (Section 4): the norm to the
 *     power 1, 3 or 4 minus the weight, with the same objective (2.7) summed
 *     pixel by pixel and the same gradient (2.8).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - pixel centres are y_k = lo + (k + 1/2) s with s = (hi - lo)/M, the
 *     pixel index j is row-major with the last axis fastest;
 *   - argmin ties go to the lowest seed index;
 *   - the symmetric matrices are read through their upper triangle only;
 *   - the L-BFGS details (memory 10, first step, Armijo backtracking,
 *     gauge projection, restart rule) are this project's specification --
 *     the paper only names "classic L-BFGS";
 *   - an empty cell keeps its seed in the Lloyd update.
 *
 * Everything is computed in IEEE double with no contraction of a*b+c into
 * fused multiply-adds (build with -ffp-contract=off), in the fixed
 * expression order written below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dim;        /* 2 or 3 */
    int64_t n;          /* number of seeds */
    int32_t grid[3];    /* pixels per axis */
    double lo[3], hi[3];
    const double *x;    /* [n][dim] */
    const double *A;    /* [n][dim][dim], symmetric, upper triangle read */
    const double *v;    /* [n] target volumes (may be NULL for assignment) */
    const uint8_t *mass; /* [J] pixel weights q_j (measure q_j/255 |P|), or NULL: all full */
    int32_t power;      /* cost |y - x_i|_{A_i}^power - w_i; 0 or 2: the APD cost */
} orc_problem;

/* ---------------------------------------------------------------- grid -- */

static int64_t orc_num_pixels(const orc_problem *p) {
    int64_t J = 1;
    for (int d = 0; d < p->dim; ++d) J *= p->grid[d];
    return J;
}

/* |P| = prod_d s_d, Section 2.3 */
double orc_pixel_volume(const orc_problem *p) {
    double vol = 1.0;
    for (int d = 0; d < p->dim; ++d) vol *= (p->hi[d] - p->lo[d]) / (double)p->grid[d];
    return vol;
}

/* The measure unit of the integer pixel weights: |P| without masses (every
 * weight 1), |P| / 255 with them. */
static double orc_mass_unit(const orc_problem *p) {
    return p->mass ? orc_pixel_volume(p) / 255.0 : orc_pixel_volume(p);
}

static int64_t orc_weight(const orc_problem *p, int64_t j) {
    return p->mass ? (int64_t)p->mass[j] : 1;
}

/* Total measure of the discretised domain, sum_j |P_j|. */
double orc_domain_measure(const orc_problem *p) {
    const int64_t J = orc_num_pixels(p);
    int64_t q = 0;
    for (int64_t j = 0; j < J; ++j) q += orc_weight(p, j);
    return (double)q * orc_mass_unit(p);
}

/* Centre of pixel j (row-major, last axis fastest), eq. (2.6) */
static void orc_pixel_centre(const orc_problem *p, int64_t j, double *y, int64_t *k) {
    int64_t r = j;
    for (int d = p->dim - 1; d >= 0; --d) {
        k[d] = r % p->grid[d];
        r /= p->grid[d];
    }
    for (int d = 0; d < p->dim; ++d) {
        double s = (p->hi[d] - p->lo[d]) / (double)p->grid[d];
        y[d] = p->lo[d] + ((double)k[d] + 0.5) * s;
    }
}

/* ---------------------------------------------------------------- cost -- */

/* |y - x_i|^2_{A_i} (Section 2.1): d = y - x_i, row r of A d summed left to
 * right, then the rows weighted by d_r and summed left to right. */
static double orc_sqnorm(const orc_problem *p, int64_t i, const double *y) {
    const int D = p->dim;
    const double *xi = p->x + i * D;
    const double *Ai = p->A + i * D * D;
    double d[3];
    for (int r = 0; r < D; ++r) d[r] = y[r] - xi[r];
    double q = 0.0;
    for (int r = 0; r < D; ++r) {
        double row = 0.0;
        for (int c = 0; c < D; ++c) {
            int lo = r < c ? r : c, hi = r < c ? c : r;
            double a = Ai[lo * D + hi];
            double t = a * d[c];
            row = (c == 0) ? t : row + t;
        }
        double t = d[r] * row;
        q = (r == 0) ? t : q + t;
    }
    return q;
}

/* Algorithm 1: C_ij = |y_j - x_i|^2_{A_i} - w_i.  Other powers of the
 * anisotropic norm (the general costs the paper's discussion (Section 4)
 * names as an extension): C_ij = |y_j - x_i|_{A_i}^p - w_i, p = 1, 3, 4,
 * from the squared norm q (clamped at 0: its rounding may leave it slightly
 * negative) as sqrt(q), q sqrt(q), q q. */
static double orc_cost(const orc_problem *p, int64_t i, const double *y, const double *w) {
    const double q = orc_sqnorm(p, i, y);
    if (p->power == 0 || p->power == 2) return q - w[i];
    const double qc = q > 0.0 ? q : 0.0;
    double c;
    if (p->power == 1) c = sqrt(qc);
    else if (p->power == 3) c = qc * sqrt(qc);
    else c = qc * qc;
    return c - w[i];
}

/* ---------------------------------------------------------- assignment -- */

/* Algorithm 1 over every pixel: H_j = lowest i attaining min_i C_ij.
 * Also returns the minimum C_(1) and the runner-up C_(2) (the smallest
 * value among the other seeds; +inf when n = 1).  Any output may be NULL. */
void orc_assign(const orc_problem *p, const double *w, int32_t *labels,
                double *best, double *second) {
    const int64_t J = orc_num_pixels(p);
    const int64_t n = p->n;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < J; ++j) {
        double y[3];
        int64_t k[3];
        orc_pixel_centre(p, j, y, k);
        double b = INFINITY, s = INFINITY;
        int64_t bi = -1;
        for (int64_t i = 0; i < n; ++i) {
            double c = orc_cost(p, i, y, w);
            if (bi < 0 || c < b) {
                s = b;
                b = c;
                bi = i;
            } else if (c < s) {
                s = c;
            }
        }
        if (labels) labels[j] = (int32_t)bi;
        if (best) best[j] = b;
        if (second) second[j] = s;
    }
}

/* Algorithm 1 at a list of pixels only (for spot checks of large grids). */
void orc_assign_pixels(const orc_problem *p, const double *w, const int64_t *idx, int64_t count,
                       int32_t *labels, double *best, double *second) {
    const int64_t n = p->n;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        double y[3];
        int64_t k[3];
        orc_pixel_centre(p, idx[t], y, k);
        double b = INFINITY, s = INFINITY;
        int64_t bi = -1;
        for (int64_t i = 0; i < n; ++i) {
            double c = orc_cost(p, i, y, w);
            if (bi < 0 || c < b) {
                s = b;
                b = c;
                bi = i;
            } else if (c < s) {
                s = c;
            }
        }
        labels[t] = (int32_t)bi;
        if (best) best[t] = b;
        if (second) second[t] = s;
    }
}

/* ------------------------------------------------- objective, gradient -- */

/* Neumaier-compensated accumulation */
typedef struct { double s, c; } orc_ksum;
static void orc_ksum_add(orc_ksum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* One evaluation of the discretised problem at weights w:
 *   counts m_i = #{j : H_j = i}                              (Algorithm 2)
 *   g~(w)  = sum_i v_i w_i + |P| sum_j C_{H_j j}             (eq. (2.7))
 *   grad_i = v_i - m_i |P|                                    (eq. (2.8))
 *   maxrel = max_i |grad_i| / v_i                      (stopping rule, Alg. 2)
 *   centroid_i = (1/m_i) sum_{H_j = i} y_j, or x_i if m_i = 0 (Algorithm 3)
 * With pixel weights (the general-tessellation form of Section 2.3) every
 * pixel counts with its measure |P_j| = (q_j/255)|P|: m_i = sum q_j over the
 * cell (in units of |P|/255), the objective sums |P_j| C_{H_j j}, and the
 * centroid is the q-weighted mean.
 * The sum over j uses Neumaier compensation per thread, then the thread
 * partials are added in thread order.  Outputs other than g may be NULL. */
double orc_evaluate(const orc_problem *p, const double *w, double *grad,
                    int64_t *counts, double *centroids, double *maxrel) {
    const int64_t J = orc_num_pixels(p);
    const int64_t n = p->n;
    const int D = p->dim;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    int64_t *cnt = (int64_t *)calloc((size_t)nthreads * (size_t)n, sizeof(int64_t));
    double *ysum = (double *)calloc((size_t)nthreads * (size_t)n * D, sizeof(double));
    orc_ksum *part = (orc_ksum *)calloc((size_t)nthreads, sizeof(orc_ksum));
#pragma omp parallel num_threads(nthreads)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t *mc = cnt + (size_t)t * n;
        double *my = ysum + (size_t)t * n * D;
        orc_ksum acc = {0.0, 0.0};
#pragma omp for schedule(static)
        for (int64_t j = 0; j < J; ++j) {
            double y[3];
            int64_t k[3];
            orc_pixel_centre(p, j, y, k);
            double b = INFINITY;
            int64_t bi = -1;
            for (int64_t i = 0; i < n; ++i) {
                double c = orc_cost(p, i, y, w);
                if (bi < 0 || c < b) { b = c; bi = i; }
            }
            const int64_t q = orc_weight(p, j);
            mc[bi] += q;
            for (int d = 0; d < D; ++d) my[bi * D + d] += (double)q * y[d];
            orc_ksum_add(&acc, (double)q * b);
        }
        part[t] = acc;
    }
    orc_ksum tot = {0.0, 0.0};
    for (int t = 0; t < nthreads; ++t) {
        orc_ksum_add(&tot, part[t].s);
        orc_ksum_add(&tot, part[t].c);
    }
    const double P = orc_mass_unit(p);
    orc_ksum lin = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) orc_ksum_add(&lin, p->v[i] * w[i]);
    double g = (lin.s + lin.c) + P * (tot.s + tot.c);

    double mr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t m = 0;
        for (int t = 0; t < nthreads; ++t) m += cnt[(size_t)t * n + i];
        double gi = p->v[i] - (double)m * P;
        if (grad) grad[i] = gi;
        if (counts) counts[i] = m;
        double r = fabs(gi) / p->v[i];
        if (r > mr) mr = r;
        if (centroids) {
            for (int d = 0; d < D; ++d) {
                if (m == 0) {
                    centroids[i * D + d] = p->x[i * D + d];
                } else {
                    double s = 0.0;
                    for (int t = 0; t < nthreads; ++t) s += ysum[((size_t)t * n + i) * D + d];
                    centroids[i * D + d] = s / (double)m;
                }
            }
        }
    }
    if (maxrel) *maxrel = mr;
    free(cnt);
    free(ysum);
    free(part);
    return g;
}

/* -------------------------------------------------------------- L-BFGS -- */

/* The solver minimises f = -g~.  A callback returns f(w), writes grad f and
 * the stopping quantity crit (for the APD problem: max_i |grad_i|/v_i). */
typedef double (*orc_fg_fn)(void *ctx, const double *w, double *grad_f, double *crit);

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 4, ORC_LINESEARCH = 5 };

typedef struct {
    double eps;        /* stop when crit < eps */
    int32_t max_iter;  /* accepted steps */
    int32_t max_evals; /* callback calls */
    int32_t history;   /* stored (s, y) pairs */
    double gamma0;     /* scale of the first / restart step */
} orc_lbfgs_opts;

typedef struct {
    int32_t converged, iters, evals;
    double f, crit;
} orc_lbfgs_report;

static double orc_dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* remove the mean: the objective is invariant under w -> w + c when the
 * target volumes sum to the domain measure, so the gradient is kept in the
 * subspace sum = 0 */
static void orc_project(int64_t n, double *g) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m += g[i];
    m /= (double)n;
    for (int64_t i = 0; i < n; ++i) g[i] -= m;
}

/* Two-loop recursion (Nocedal & Wright, Alg. 7.4): r = H q with the pairs
 * stored oldest first in S, Y (row k = pair k), rho_k = 1/(s_k.y_k), and the
 * initial matrix gamma I. */
void orc_two_loop(int64_t n, int32_t npairs, const double *S, const double *Y,
                  const double *rho, double gamma, const double *q_in, double *r) {
    double *q = (double *)malloc((size_t)n * sizeof(double));
    double *alpha = (double *)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(double));
    memcpy(q, q_in, (size_t)n * sizeof(double));
    for (int32_t k = npairs - 1; k >= 0; --k) {
        const double *s = S + (size_t)k * n, *y = Y + (size_t)k * n;
        alpha[k] = rho[k] * orc_dot(n, s, q);
        for (int64_t i = 0; i < n; ++i) q[i] -= alpha[k] * y[i];
    }
    for (int64_t i = 0; i < n; ++i) r[i] = gamma * q[i];
    for (int32_t k = 0; k < npairs; ++k) {
        const double *s = S + (size_t)k * n, *y = Y + (size_t)k * n;
        double beta = rho[k] * orc_dot(n, y, r);
        for (int64_t i = 0; i < n; ++i) r[i] += s[i] * (alpha[k] - beta);
    }
    free(q);
    free(alpha);
}

int orc_lbfgs(int64_t n, double *w, orc_fg_fn fg, void *ctx, const orc_lbfgs_opts *o,
              orc_lbfgs_report *rep) {
    const int m = o->history > 0 ? o->history : 1;
    double *g = (double *)malloc((size_t)n * sizeof(double));   /* projected grad f at w */
    double *gt = (double *)malloc((size_t)n * sizeof(double));  /* grad f at the trial point */
    double *wt = (double *)malloc((size_t)n * sizeof(double));  /* trial point */
    double *d = (double *)malloc((size_t)n * sizeof(double));   /* search direction */
    double *s = (double *)malloc((size_t)n * sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    double *S = (double *)malloc((size_t)m * n * sizeof(double));
    double *Y = (double *)malloc((size_t)m * n * sizeof(double));
    double *rho = (double *)malloc((size_t)m * sizeof(double));
    int32_t npairs = 0, iters = 0, evals = 0, status = ORC_NOT_CONVERGED;
    double crit = 0.0, critt = 0.0;

    /* evaluate at the starting point and test the stopping rule there */
    double f = fg(ctx, w, g, &crit);
    evals = 1;
    if (crit < o->eps) { status = ORC_OK; goto done; }
    orc_project(n, g);

    while (iters < o->max_iter && evals < o->max_evals) {
        /* direction: d = -H g by the two-loop recursion with H0 = gamma I,
         * gamma = s.y / y.y of the newest pair; with no pairs, d = -gamma0 g */
        if (npairs > 0) {
            const double *sl = S + (size_t)(npairs - 1) * n, *yl = Y + (size_t)(npairs - 1) * n;
            double gamma = orc_dot(n, sl, yl) / orc_dot(n, yl, yl);
            orc_two_loop(n, npairs, S, Y, rho, gamma, g, d);
            for (int64_t i = 0; i < n; ++i) d[i] = -d[i];
        } else {
            for (int64_t i = 0; i < n; ++i) d[i] = -o->gamma0 * g[i];
        }
        double gd = orc_dot(n, g, d);
        if (!(gd < 0.0)) {
            /* not a descent direction: restart from the scaled steepest
             * step once; a steepest step that is not descent means g = 0 */
            if (npairs > 0) { npairs = 0; continue; }
            status = ORC_LINESEARCH;
            break;
        }
        /* Armijo backtracking from a unit step, halving up to 30 times; the
         * stopping rule is tested after every evaluation */
        double a = 1.0, ft = 0.0;
        int accepted = 0, stop = 0;
        for (int t = 0; t < 30; ++t) {
            for (int64_t i = 0; i < n; ++i) wt[i] = w[i] + a * d[i];
            ft = fg(ctx, wt, gt, &critt);
            ++evals;
            if (critt < o->eps) {
                memcpy(w, wt, (size_t)n * sizeof(double));
                f = ft;
                crit = critt;
                ++iters;
                status = ORC_OK;
                stop = 1;
                break;
            }
            if (ft <= f + 1e-4 * a * gd) { accepted = 1; break; }
            if (evals >= o->max_evals) { stop = 1; break; }
            a *= 0.5;
        }
        if (stop) break;
        if (!accepted) {
            /* failed search: clear the history and retry once with the
             * scaled steepest step */
            if (npairs > 0) { npairs = 0; continue; }
            status = ORC_LINESEARCH;
            break;
        }
        orc_project(n, gt);
        for (int64_t i = 0; i < n; ++i) s[i] = wt[i] - w[i];
        for (int64_t i = 0; i < n; ++i) y[i] = gt[i] - g[i];
        /* keep the curvature pair only when s.y > 1e-10 |s| |y| */
        double sy = orc_dot(n, s, y);
        double ns = sqrt(orc_dot(n, s, s)), ny = sqrt(orc_dot(n, y, y));
        if (sy > 1e-10 * ns * ny) {
            if (npairs == m) {
                memmove(S, S + n, (size_t)(m - 1) * n * sizeof(double));
                memmove(Y, Y + n, (size_t)(m - 1) * n * sizeof(double));
                memmove(rho, rho + 1, (size_t)(m - 1) * sizeof(double));
                --npairs;
            }
            memcpy(S + (size_t)npairs * n, s, (size_t)n * sizeof(double));
            memcpy(Y + (size_t)npairs * n, y, (size_t)n * sizeof(double));
            rho[npairs] = 1.0 / sy;
            ++npairs;
        }
        memcpy(w, wt, (size_t)n * sizeof(double));
        memcpy(g, gt, (size_t)n * sizeof(double));
        f = ft;
        crit = critt;
        ++iters;
    }
done:
    if (rep) {
        rep->converged = (status == ORC_OK);
        rep->iters = iters;
        rep->evals = evals;
        rep->f = f;
        rep->crit = crit;
    }
    free(g); free(gt); free(wt); free(d); free(s); free(y); free(S); free(Y); free(rho);
    return status;
}

/* -------------------------------------------------- Algorithms 2 and 3 -- */

typedef struct {
    const orc_problem *p;
    double *grad;
} orc_apd_ctx;

/* f = -g~, grad f = m |P| - v, crit = max_i |v_i - m_i |P|| / v_i */
static double orc_apd_fg(void *vctx, const double *w, double *grad_f, double *crit) {
    orc_apd_ctx *c = (orc_apd_ctx *)vctx;
    double g = orc_evaluate(c->p, w, c->grad, NULL, NULL, crit);
    for (int64_t i = 0; i < c->p->n; ++i) grad_f[i] = -c->grad[i];
    return -g;
}

/* default first-step scale: 0.3 in 2D, 0.2 N^(1/3) in 3D (a stable step for
 * the graph-Laplacian-like Hessian of near-regular cells) */
double orc_default_gamma0(int32_t dim, int64_t n) {
    return dim == 2 ? 0.3 : 0.2 * cbrt((double)n);
}

/* Algorithm 2: maximise g~ by L-BFGS from w (W_0 = 0 unless warm). */
int orc_fit_weights(const orc_problem *p, double *w, int32_t warm, const orc_lbfgs_opts *o,
                    orc_lbfgs_report *rep) {
    if (!warm) memset(w, 0, (size_t)p->n * sizeof(double));
    orc_apd_ctx c = {p, (double *)malloc((size_t)p->n * sizeof(double))};
    int st = orc_lbfgs(p->n, w, orc_apd_fg, &c, o, rep);
    free(c.grad);
    return st;
}

/* Algorithm 2 with its last step: if the fit does not converge, refine the
 * grid and restart from the weights reached, at most max_refine times.  The
 * refinement scales every axis by f = max(3/2, ((|P| 2^D) / (eps min v))^(1/D)),
 * the factor that also meets the pixel-size rule (2.10), and rounds up.
 * The grid of the last fit is returned in grid_out.  Pixel weights are tied
 * to their grid, so problems with them are not refined. */
int orc_fit_weights_refine(const orc_problem *p0, double *w, int32_t warm, const orc_lbfgs_opts *o,
                           int32_t max_refine, orc_lbfgs_report *rep, int32_t *grid_out) {
    orc_problem p = *p0;
    int st = orc_fit_weights(&p, w, warm, o, rep);
    for (int r = 0; r < max_refine && st != ORC_OK && !p.mass; ++r) {
        double vmin = INFINITY;
        for (int64_t i = 0; i < p.n; ++i) vmin = fmin(vmin, p.v[i]);
        const double target = o->eps * vmin / pow(2.0, (double)p.dim);
        double f = pow(orc_pixel_volume(&p) / target, 1.0 / (double)p.dim);
        if (!(f > 1.5)) f = 1.5;
        for (int d = 0; d < p.dim; ++d) p.grid[d] = (int32_t)ceil((double)p.grid[d] * f);
        orc_lbfgs_report r2;
        st = orc_fit_weights(&p, w, 1, o, &r2);
        r2.iters += rep->iters;
        r2.evals += rep->evals;
        *rep = r2;
    }
    for (int d = 0; d < 3; ++d) grid_out[d] = p.grid[d];
    return st;
}

/* One pass of the loop of Algorithm 3: fit from the current w (warm start
 * W_0^{k+1} = W^k), then move every seed to the discrete centroid of its
 * cell (an empty cell keeps its seed).  x is updated in place. */
int orc_lloyd_step(orc_problem *p, double *x, double *w, const orc_lbfgs_opts *o,
                   orc_lbfgs_report *rep) {
    p->x = x;
    int st = orc_fit_weights(p, w, 1, o, rep);
    double *cen = (double *)malloc((size_t)p->n * p->dim * sizeof(double));
    orc_evaluate(p, w, NULL, NULL, cen, NULL);
    memcpy(x, cen, (size_t)p->n * p->dim * sizeof(double));
    free(cen);
    return st;
}

/* ---------------------------------------------------------- resolution -- */

/* eq. (2.9): single-phase lower bound M > (N / eps)^(1/D) */
double orc_resolution_lower_bound(int32_t dim, int64_t n, double eps) {
    return pow((double)n / eps, 1.0 / (double)dim);
}

/* eq. (2.10): the smallest integer M with |Omega| / M^D < (eps / 2^D) min_i v_i.
 * The inequality is strict in the reals; decimal inputs such as eps = 0.01
 * and v = 1/N make exact ties common (N = 10^4 in 2D: M = 2000 gives
 * equality), so a tie within a relative 1e-12 of rounding counts as a tie
 * and is rejected. */
int64_t orc_choose_resolution(int32_t dim, double eps, double vmin, double omega) {
    double rhs = eps / pow(2.0, (double)dim) * vmin;
    int64_t M = 1;
    while (!(omega / pow((double)M, (double)dim) < rhs * (1.0 - 1e-12))) ++M;
    return M;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
