// apd_kernels.hip -- gfx950 kernels of the APD hot path.
//
// One evaluation of the discretised dual problem (Section 2.3 of
// arXiv 2403.03571) is a chain of four kernels on one stream:
//
//   k_prep        one block: gauge max of w, Gershgorin bound of the
//                 anisotropy matrices, input validation, zeroed moments.
//   k_assign_*    the O(N J) part (Algorithm 1): every pixel of a tile
//                 scans every seed, keeps the argmin, and the tile reduces
//                 the exact integer moments of each cell it touched.
//                 _fp64 evaluates C_ij = |y_j - x_i|^2_{A_i} - w_i exactly as
//                 the definition is written; _fp32 evaluates it in local
//                 coordinates in single precision and queues every pixel
//                 whose top-two gap is within its rounding bound.
//   k_recheck     one wave per queued pixel re-runs the scan in double, in
//                 the definition's own expression order, so every label
//                 equals that of an exact double-precision argmin.
//   k_finalize    one block: objective (2.7), gradient (2.8), maximum
//                 relative volume error, centroids, from the moments.
//
// The whole file is built with -ffp-contract=off: the double-precision
// costs are evaluated without fused multiply-adds, and the single-precision
// path fuses only where it says so (fmaf).
#include "apd_device.h"

#include <math.h>

namespace apd {
namespace {

using namespace dev;

// ------------------------------------------------------------- k_prep

// Eigenvalue range of a symmetric 2x2 or 3x3 matrix (upper triangle u),
// closed form (the 3x3 case by the trigonometric solution of the
// characteristic cubic), widened by a relative 1e-6 for the rounding of the
// formulas.
template <int D>
__device__ inline void eig_range(const double (&u)[3][3], double *lmin, double *lmax) {
    if (D == 2) {
        const double m = 0.5 * (u[0][0] + u[1][1]);
        const double h = 0.5 * (u[0][0] - u[1][1]);
        const double r = sqrt(h * h + u[0][1] * u[0][1]);
        *lmin = m - r;
        *lmax = m + r;
    } else {
        const double p1 = u[0][1] * u[0][1] + u[0][2] * u[0][2] + u[1][2] * u[1][2];
        const double q = (u[0][0] + u[1][1] + u[2][2]) / 3.0;
        const double d0 = u[0][0] - q, d1 = u[1][1] - q, d2 = u[2][2] - q;
        const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
        const double pp = sqrt(p2 / 6.0);
        if (pp <= 1e-300) {
            *lmin = *lmax = q;
        } else {
            const double b00 = d0 / pp, b11 = d1 / pp, b22 = d2 / pp;
            const double b01 = u[0][1] / pp, b02 = u[0][2] / pp, b12 = u[1][2] / pp;
            const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
                               b02 * (b01 * b12 - b11 * b02);
            const double rr = fmin(1.0, fmax(-1.0, 0.5 * det));
            const double phi = acos(rr) / 3.0;
            *lmax = q + 2.0 * pp * cos(phi);
            *lmin = q + 2.0 * pp * cos(phi + 2.0943951023931957);  // + 2 pi / 3
        }
    }
    const double span = fabs(*lmax) + fabs(*lmin);
    *lmin -= 1e-6 * span;
    *lmax += 1e-6 * span;
}

template <int D>
__global__ __launch_bounds__(1024) void k_prep(Geo g, Seeds sd, Scalars *sc, uint64_t *mom,
                                               double *eig) {
    constexpr int K = moments_per_cell(D);
    __shared__ double s_w[1024];
    __shared__ double s_v[1024];
    __shared__ float s_l[1024];
    __shared__ int s_b[1024];
    const int tid = threadIdx.x;
    if (mom)
        for (size_t t = tid; t < (size_t)g.n * K; t += 1024) mom[t] = 0ull;
    double wm = -INFINITY, vs = 0.0;
    float lam = 0.0f;
    int bad = 0;
    for (int i = tid; i < g.n; i += 1024) {
        const double wi = sd.w[i];
        if (!isfinite(wi)) bad |= kBadW;
        wm = fmax(wm, wi);
        for (int d = 0; d < D; ++d)
            if (!isfinite(sd.x[(size_t)i * D + d])) bad |= kBadX;
        const double *a = sd.A + (size_t)i * D * D;
        double u[3][3];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                u[r][c] = (r <= c) ? a[r * D + c] : a[c * D + r];
                if (!isfinite(u[r][c])) bad |= kBadA;
            }
        // Sylvester: leading principal minors positive
        bool spd = u[0][0] > 0.0;
        const double m2 = u[0][0] * u[1][1] - u[0][1] * u[0][1];
        spd = spd && m2 > 0.0;
        if (D == 3) {
            const double det = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[1][2]) -
                               u[0][1] * (u[0][1] * u[2][2] - u[1][2] * u[0][2]) +
                               u[0][2] * (u[0][1] * u[1][2] - u[1][1] * u[0][2]);
            spd = spd && det > 0.0;
        }
        if (!spd) bad |= kBadSPD;
        if (eig) {
            double lo, hi;
            eig_range<D>(u, &lo, &hi);
            eig[2 * (size_t)i] = lo;
            eig[2 * (size_t)i + 1] = hi;
        }
        // Gershgorin: lambda_max <= max_r sum_c |a_rc|
        for (int r = 0; r < D; ++r) {
            double rs = 0.0;
            for (int c = 0; c < D; ++c) rs += fabs(u[r][c]);
            lam = fmaxf(lam, (float)rs);
        }
        if (sd.v) {
            const double vi = sd.v[i];
            if (!(vi > 0.0) || !isfinite(vi)) bad |= kBadV;
            vs += vi;
        }
    }
    s_w[tid] = wm;
    s_v[tid] = vs;
    s_l[tid] = lam;
    s_b[tid] = bad;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (tid < o) {
            s_w[tid] = fmax(s_w[tid], s_w[tid + o]);
            s_v[tid] = s_v[tid] + s_v[tid + o];
            s_l[tid] = fmaxf(s_l[tid], s_l[tid + o]);
            s_b[tid] = s_b[tid] | s_b[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        sc->wmax = s_w[0];
        sc->vsum = s_v[0];
        sc->lam = s_l[0] * 1.0001f;
        sc->bad = s_b[0];
        sc->qcount = 0u;
        sc->g = 0.0;
        sc->maxrel = 0.0;
    }
}

// ------------------------------------------------------ k_assign_fp64

template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_fp64(Geo g, Seeds sd, const Scalars *sc,
                                                         PassOut out) {
    const Tile<D> t = tile_of<D>(g);
    const bool lane_ok = lane_in_grid<D>(g, t);
    bool act[kP];
    double y[kP][D];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        act[p] = lane_ok && (t.k0w + p) < g.grid[0];
        y[p][0] = centre(g, 0, t.k0w + p);
        for (int d = 1; d < D; ++d) y[p][d] = centre(g, d, t.k[d]);
    }
    double best[kP];
    int lab[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        best[p] = INFINITY;
        lab[p] = 0;
    }
    for (int i = 0; i < g.n; ++i) {
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const double c = exact_cost<D>(sd.x, sd.A, sd.w, i, y[p]);
            if (c < best[p]) {
                best[p] = c;
                lab[p] = i;
            }
        }
    }
    bool flag[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) flag[p] = false;
    PassOut o = out;
    o.queue = nullptr;
    tile_epilogue<D>(g, t, act, lab, flag, o, nullptr);
}

// ------------------------------------------------------ k_assign_fp32

// Single precision on the vector ALU, with a certified margin.  For the tile
// anchor a (tile centre) and u = y - a, e_i = x_i - a:
//   C_ij = (u - e)^T A (u - e) - w_i' = u^T A u - 2 u^T A e + e^T A e - w_i'
// with w' = w - max w <= 0 (the argmin does not change under a common shift).
// The coefficients of the quadratic in u are formed per tile in LDS; each
// lane evaluates it for its kPv pixels along axis 0 as
//   C = (a00 u0 + beta) u0 + alpha,
// beta and alpha being the parts that depend only on the lane's other axes
// (3 FMA per seed and lane, 2 per pair).  The running argmin keeps the cost's
// float bits with the low 4 mantissa bits replaced by the seed's index within
// a group of 16 (signed-integer order is the cost order), so one and_or,
// one min and one med3 keep the best and the runner-up; the group that last
// improved the best is recorded once per 16 seeds.
//
// Rounding bound: with T the sum of the absolute values of all terms of the
// expansion, |C_fp32 - C| <= rho T, rho = 2^-18 (several times the ~20
// roundings the inputs and the evaluation go through).  For any seed with
// true cost C <= B, T <= 2B + 4 r sqrt(B) + 5 r^2 with r = sqrt(lambda) |u|max
// (lambda bounding every eigenvalue of every A_i).  A pixel is settled when
// C_(2) - C_(1) > 2 rho T(B1) + 2^-18 max|C| (the dropped key bits), B1 an
// upper bound of the true C_(1); every other pixel goes to the double
// re-check.
constexpr int kPv = 8;  // pixels per lane of the vector kernel

template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_fp32(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    constexpr int NS = D == 2 ? 2 : 3;
    constexpr int P = kPv;
    constexpr int E0 = kWaves * P;
    __shared__ float4 sC[NS][kChunk];
    const Tile<D> t = tile_of<D, P>(g);
    const bool lane_ok = lane_in_grid<D>(g, t);

    float s[3];
    double anc[3];
    for (int d = 0; d < D; ++d) {
        s[d] = (float)g.s[d];
        anc[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
    }
    bool act[P];
    float u0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        act[p] = lane_ok && (t.k0w + p) < g.grid[0];
        u0[p] = ((float)(t.k0w + p - t.anc[0]) + 0.5f) * s[0];
    }
    const float u1 = ((float)(t.k[1] - t.anc[1]) + 0.5f) * s[1];
    const float u2 = D == 3 ? ((float)(t.k[2] - t.anc[2]) + 0.5f) * s[2] : 0.0f;

    const double wmax = sc->wmax;
    int best[P], second[P], blk[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        best[p] = 0x7fffffff;
        second[p] = 0x7fffffff;
        blk[p] = 0;
    }

    for (int base = 0; base < g.n; base += kChunk) {
        const int cnt = min(kChunk, g.n - base);
        const int padded = (cnt + 15) & ~15;
        __syncthreads();
        for (int q = threadIdx.x; q < padded; q += kThreads) {
            if (q >= cnt) {  // padding seeds: a constant cost beyond any real one
                sC[0][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (D == 2) {
                    sC[1][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
                } else {
                    sC[1][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    sC[2][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
                }
                continue;
            }
            const int i = base + q;
            const double *xi = sd.x + (size_t)i * D;
            const double *a = sd.A + (size_t)i * D * D;
            float e[3];
            for (int d = 0; d < D; ++d) e[d] = (float)(xi[d] - anc[d]);
            const float wp = (float)(sd.w[i] - wmax);
            if (D == 2) {
                const float a00 = (float)a[0], a01 = (float)a[1], a11 = (float)a[3];
                const float ae0 = fmaf(a00, e[0], a01 * e[1]);
                const float ae1 = fmaf(a01, e[0], a11 * e[1]);
                const float cc = fmaf(e[0], ae0, e[1] * ae1) - wp;
                sC[0][q] = make_float4(a00, 2.0f * a01, a11, -2.0f * ae0);
                sC[1][q] = make_float4(-2.0f * ae1, cc, 0.0f, 0.0f);
            } else {
                const float a00 = (float)a[0], a01 = (float)a[1], a02 = (float)a[2];
                const float a11 = (float)a[4], a12 = (float)a[5], a22 = (float)a[8];
                const float ae0 = fmaf(a00, e[0], fmaf(a01, e[1], a02 * e[2]));
                const float ae1 = fmaf(a01, e[0], fmaf(a11, e[1], a12 * e[2]));
                const float ae2 = fmaf(a02, e[0], fmaf(a12, e[1], a22 * e[2]));
                const float cc = fmaf(e[0], ae0, fmaf(e[1], ae1, e[2] * ae2)) - wp;
                sC[0][q] = make_float4(a00, 2.0f * a01, 2.0f * a02, -2.0f * ae0);
                sC[1][q] = make_float4(a11, 2.0f * a12, a22, -2.0f * ae1);
                sC[2][q] = make_float4(-2.0f * ae2, cc, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        for (int q0 = 0; q0 < padded; q0 += 16) {
            int old[P];
#pragma unroll
            for (int p = 0; p < P; ++p) old[p] = best[p];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int q = q0 + r;
                const float4 c0 = sC[0][q];
                const float4 c1 = sC[1][q];
                float a00, beta, alpha;
                if (D == 2) {
                    a00 = c0.x;
                    beta = fmaf(c0.y, u1, c0.w);
                    alpha = fmaf(fmaf(c0.z, u1, c1.x), u1, c1.y);
                } else {
                    const float4 c2 = sC[2][q];
                    a00 = c0.x;
                    beta = fmaf(c0.y, u1, fmaf(c0.z, u2, c0.w));
                    alpha = fmaf(fmaf(c1.x, u1, fmaf(c1.y, u2, c1.w)), u1,
                                 fmaf(fmaf(c1.z, u2, c2.x), u2, c2.y));
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                    const int key = (__float_as_int(c) & ~15) | r;
                    second[p] = med3i(best[p], key, second[p]);
                    best[p] = min(best[p], key);
                }
            }
            const int sblk = base + q0;
#pragma unroll
            for (int p = 0; p < P; ++p) blk[p] = (best[p] != old[p]) ? sblk : blk[p];
        }
    }

    // certification
    float umax2 = 0.0f;
    {
        const float h0 = (0.5f * E0 - 0.5f) * s[0];
        const float h1 = (0.5f * Lanes<D>::L1 - 0.5f) * s[1];
        umax2 = h0 * h0 + h1 * h1;
        if (D == 3) {
            const float h2 = (0.5f * Lanes<D>::L2 - 0.5f) * s[2];
            umax2 += h2 * h2;
        }
    }
    const float r2 = sc->lam * umax2 * 1.01f;
    const float r = sqrtf(r2);
    constexpr float rho = 0x1p-18f;
    bool flag[P];
    int lab[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        lab[p] = min(blk[p] + (best[p] & 15), g.n - 1);
        const float fb = __int_as_float(best[p]), fs = __int_as_float(second[p]);
        const float bb = fmaxf(fb, 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float T = 2.0f * B1 + 4.0f * r * sqrtf(B1) + 5.0f * r2;
        const float thr = 2.0f * rho * T + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fs));
        flag[p] = !((fs - fb) > thr);
    }
    tile_epilogue<D, P>(g, t, act, lab, flag, out, &sc->qcount);
}

// ------------------------------------------------------ k_assign_cull

// The vector single-precision kernel over the seeds that can win somewhere
// in the tile.  For the box B spanned by the tile's pixel centres,
//   min_{y in B} C_i(y) >= lmin_i dist(x_i, B)^2 - w_i'        = LB_i
//   max_{y in B} C_i(y) <= lmax_i maxdist(x_i, B)^2 - w_i'     = UB_i
// (lmin, lmax the eigenvalue range of A_i), so a seed with LB_i above
// U = min_k UB_k is beaten everywhere in the tile by the seed attaining U
// and cannot be the argmin (nor a near-tie) at any of its pixels.  The
// bounds are evaluated in double and widened by a relative 1e-9, far above
// the rounding of the double costs, so the candidate list contains every
// seed the exact double argmin could pick.  The argmin and its certificate
// are then those of k_assign_fp32 restricted to the candidates; the labels
// are unchanged.  Tiles with more than kCullCap candidates scan every seed.
constexpr int kCullCap = 2048;

template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_cull(Geo g, Seeds sd, Scalars *sc,
                                                         const double *eig, PassOut out) {
    constexpr int NS = D == 2 ? 2 : 3;
    constexpr int P = kPv;
    constexpr int E0 = kWaves * P;
    __shared__ float4 sC[NS][kChunk];
    __shared__ int s_list[kCullCap];
    __shared__ double s_red[kWaves];
    __shared__ int s_cnt;
    const Tile<D> t = tile_of<D, P>(g);
    const bool lane_ok = lane_in_grid<D>(g, t);
    const double wmax = sc->wmax;

    // ---- the candidate list
    double blo[3], bhi[3];
    {
        const int ext[3] = {E0, Lanes<D>::L1, Lanes<D>::L2};
        for (int d = 0; d < D; ++d) {
            const int k0 = t.anc[d] - ext[d] / 2;
            const int k1 = min(k0 + ext[d], g.grid[d]) - 1;
            blo[d] = centre(g, d, k0);
            bhi[d] = centre(g, d, max(k1, k0));
        }
    }
    auto bounds = [&](int i, double *lb, double *ub) {
        double dist2 = 0.0, far2 = 0.0;
        for (int d = 0; d < D; ++d) {
            const double xd = sd.x[(size_t)i * D + d];
            const double dd = fmax(0.0, fmax(blo[d] - xd, xd - bhi[d]));
            const double fd = fmax(xd - blo[d], bhi[d] - xd);
            dist2 += dd * dd;
            far2 += fd * fd;
        }
        const double wp = sd.w[i] - wmax;
        const double l = eig[2 * (size_t)i] * dist2, h = eig[2 * (size_t)i + 1] * far2;
        const double slack = 1e-9 * (fabs(l) + fabs(h) + fabs(wp));
        *lb = l - wp - slack;
        *ub = h - wp + slack;
    };
    double umin = INFINITY;
    for (int i = threadIdx.x; i < g.n; i += kThreads) {
        double lb, ub;
        bounds(i, &lb, &ub);
        umin = fmin(umin, ub);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) umin = fmin(umin, __shfl_xor(umin, o));
    if (threadIdx.x == 0) s_cnt = 0;
    if (t.lane == 0) s_red[threadIdx.x >> 6] = umin;
    __syncthreads();
    const double U = fmin(fmin(s_red[0], s_red[1]), fmin(s_red[2], s_red[3]));
    for (int i0 = 0; i0 < g.n; i0 += kThreads) {
        const int i = i0 + threadIdx.x;
        bool cand = false;
        if (i < g.n) {
            double lb, ub;
            bounds(i, &lb, &ub);
            cand = lb <= U;
        }
        const unsigned long long m = __ballot(cand);
        int base = 0;
        if (t.lane == 0 && m) base = atomicAdd(&s_cnt, (int)__popcll(m));
        base = __shfl(base, 0);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (cand && base + below < kCullCap) s_list[base + below] = i;
    }
    __syncthreads();
    const int ncand = s_cnt;
    const bool full = ncand > kCullCap;
    const int nscan = full ? g.n : ncand;

    // ---- the argmin over the candidates (as k_assign_fp32)
    float s[3];
    double anc[3];
    for (int d = 0; d < D; ++d) {
        s[d] = (float)g.s[d];
        anc[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
    }
    bool act[P];
    float u0[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        act[p] = lane_ok && (t.k0w + p) < g.grid[0];
        u0[p] = ((float)(t.k0w + p - t.anc[0]) + 0.5f) * s[0];
    }
    const float u1 = ((float)(t.k[1] - t.anc[1]) + 0.5f) * s[1];
    const float u2 = D == 3 ? ((float)(t.k[2] - t.anc[2]) + 0.5f) * s[2] : 0.0f;
    int best[P], second[P], blk[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        best[p] = 0x7fffffff;
        second[p] = 0x7fffffff;
        blk[p] = 0;
    }
    for (int base = 0; base < nscan; base += kChunk) {
        const int cnt = min(kChunk, nscan - base);
        const int padded = (cnt + 15) & ~15;
        __syncthreads();
        for (int q = threadIdx.x; q < padded; q += kThreads) {
            if (q >= cnt) {
                sC[0][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (D == 2) {
                    sC[1][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
                } else {
                    sC[1][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    sC[2][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
                }
                continue;
            }
            const int i = full ? base + q : s_list[base + q];
            const double *xi = sd.x + (size_t)i * D;
            const double *a = sd.A + (size_t)i * D * D;
            float e[3];
            for (int d = 0; d < D; ++d) e[d] = (float)(xi[d] - anc[d]);
            const float wp = (float)(sd.w[i] - wmax);
            if (D == 2) {
                const float a00 = (float)a[0], a01 = (float)a[1], a11 = (float)a[3];
                const float ae0 = fmaf(a00, e[0], a01 * e[1]);
                const float ae1 = fmaf(a01, e[0], a11 * e[1]);
                const float cc = fmaf(e[0], ae0, e[1] * ae1) - wp;
                sC[0][q] = make_float4(a00, 2.0f * a01, a11, -2.0f * ae0);
                sC[1][q] = make_float4(-2.0f * ae1, cc, 0.0f, 0.0f);
            } else {
                const float a00 = (float)a[0], a01 = (float)a[1], a02 = (float)a[2];
                const float a11 = (float)a[4], a12 = (float)a[5], a22 = (float)a[8];
                const float ae0 = fmaf(a00, e[0], fmaf(a01, e[1], a02 * e[2]));
                const float ae1 = fmaf(a01, e[0], fmaf(a11, e[1], a12 * e[2]));
                const float ae2 = fmaf(a02, e[0], fmaf(a12, e[1], a22 * e[2]));
                const float cc = fmaf(e[0], ae0, fmaf(e[1], ae1, e[2] * ae2)) - wp;
                sC[0][q] = make_float4(a00, 2.0f * a01, 2.0f * a02, -2.0f * ae0);
                sC[1][q] = make_float4(a11, 2.0f * a12, a22, -2.0f * ae1);
                sC[2][q] = make_float4(-2.0f * ae2, cc, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        for (int q0 = 0; q0 < padded; q0 += 16) {
            int old[P];
#pragma unroll
            for (int p = 0; p < P; ++p) old[p] = best[p];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int q = q0 + r;
                const float4 c0 = sC[0][q];
                const float4 c1 = sC[1][q];
                float a00, beta, alpha;
                if (D == 2) {
                    a00 = c0.x;
                    beta = fmaf(c0.y, u1, c0.w);
                    alpha = fmaf(fmaf(c0.z, u1, c1.x), u1, c1.y);
                } else {
                    const float4 c2 = sC[2][q];
                    a00 = c0.x;
                    beta = fmaf(c0.y, u1, fmaf(c0.z, u2, c0.w));
                    alpha = fmaf(fmaf(c1.x, u1, fmaf(c1.y, u2, c1.w)), u1,
                                 fmaf(fmaf(c1.z, u2, c2.x), u2, c2.y));
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                    const int key = (__float_as_int(c) & ~15) | r;
                    second[p] = med3i(best[p], key, second[p]);
                    best[p] = min(best[p], key);
                }
            }
            const int sblk = base + q0;
#pragma unroll
            for (int p = 0; p < P; ++p) blk[p] = (best[p] != old[p]) ? sblk : blk[p];
        }
    }
    float umax2;
    {
        const float h0 = (0.5f * E0 - 0.5f) * s[0];
        const float h1 = (0.5f * Lanes<D>::L1 - 0.5f) * s[1];
        umax2 = h0 * h0 + h1 * h1;
        if (D == 3) {
            const float h2 = (0.5f * Lanes<D>::L2 - 0.5f) * s[2];
            umax2 += h2 * h2;
        }
    }
    const float r2 = sc->lam * umax2 * 1.01f;
    const float r = sqrtf(r2);
    constexpr float rho = 0x1p-18f;
    bool flag[P];
    int lab[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int pos = min(blk[p] + (best[p] & 15), nscan - 1);
        lab[p] = full ? pos : s_list[pos];
        const float fb = __int_as_float(best[p]), fs = __int_as_float(second[p]);
        const float bb = fmaxf(fb, 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float T = 2.0f * B1 + 4.0f * r * sqrtf(B1) + 5.0f * r2;
        const float thr = 2.0f * rho * T + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fs));
        flag[p] = !((fs - fb) > thr);
    }
    tile_epilogue<D, P>(g, t, act, lab, flag, out, &sc->qcount);
}

// ------------------------------------------------------ k_assign_mfma

// One block per tile; the tile body (dev::mfma_tile) is shared with the
// batched persistent kernel.
template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_mfma(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    __shared__ __attribute__((aligned(16))) float sC[kMfmaLds];
    if (D == 2)
        dev::mfma_tile<2>(g, sd, sc->wmax, sc->lam, blockIdx.y, blockIdx.x, 0, sC, out, &sc->qcount);
    else
        dev::mfma_tile<3>(g, sd, sc->wmax, sc->lam, blockIdx.z, blockIdx.y, blockIdx.x, sC, out,
                          &sc->qcount);
}

// ------------------------------------------------------ k_assign_bf16

template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_bf16(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    __shared__ __attribute__((aligned(16))) float sC[kMfmaLds];
    if (D == 2)
        dev::mfma_tile_bf16<2>(g, sd, sc->wmax, sc->lam, blockIdx.y, blockIdx.x, 0, sC, out,
                               &sc->qcount);
    else
        dev::mfma_tile_bf16<3>(g, sd, sc->wmax, sc->lam, blockIdx.z, blockIdx.y, blockIdx.x, sC,
                               out, &sc->qcount);
}

// ---------------------------------------------------------- k_recheck

// One wave per queued pixel (dev::recheck_pixel).
template <int D>
__global__ __launch_bounds__(kThreads) void k_recheck(Geo g, Seeds sd, const Scalars *sc,
                                                     PassOut out) {
    const unsigned nq = sc->qcount;
    const int lane = __lane_id();
    const unsigned wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const unsigned nw = gridDim.x * kWaves;
    for (unsigned q = wave; q < nq; q += nw) {
        const uint32_t j = out.queue[q];
        int k[3];
        const int bi = dev::recheck_pixel<D>(g, sd, j, k);
        if (lane == 0) {
            if (out.labels) out.labels[j] = bi;
            if (out.mom) dev::pixel_moments_add<D>(out.mom, bi, k);
        }
    }
}

// -------------------------------------------------------- k_finalize

// One block: every cell's term of eq. (2.7) (dev::cell_final), summed over
// cells in a fixed order (deterministic), and the maximum relative error.
template <int D>
__global__ __launch_bounds__(1024) void k_finalize(Geo g, Seeds sd, const uint64_t *mom,
                                                  Scalars *sc, FinalOut out) {
    constexpr int K = moments_per_cell(D);
    __shared__ double s_g[1024];
    __shared__ double s_m[1024];
    const int tid = threadIdx.x;
    double gs = 0.0, mr = 0.0;
    for (int i = tid; i < g.n; i += 1024) {
        double gi, rel, ybar[3];
        gs += dev::cell_final<D>(g, sd, mom + (size_t)i * K, i, &gi, &rel, ybar);
        mr = fmax(mr, rel);
        if (out.grad) out.grad[i] = gi;
        if (out.counts) out.counts[i] = (int64_t)mom[(size_t)i * K];
        if (out.centroids)
            for (int d = 0; d < D; ++d) out.centroids[(size_t)i * D + d] = ybar[d];
    }
    s_g[tid] = gs;
    s_m[tid] = mr;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (tid < o) {
            s_g[tid] = s_g[tid] + s_g[tid + o];
            s_m[tid] = fmax(s_m[tid], s_m[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        sc->g = s_g[0];
        sc->maxrel = s_m[0];
    }
}


template <int D, int P = kP>
dim3 tile_grid(const Geo &g) {
    constexpr int E0 = kWaves * P;
    if (D == 2)
        return dim3((g.grid[1] + Lanes<2>::L1 - 1) / Lanes<2>::L1, (g.grid[0] + E0 - 1) / E0, 1);
    return dim3((g.grid[2] + Lanes<3>::L2 - 1) / Lanes<3>::L2, (g.grid[1] + Lanes<3>::L1 - 1) / Lanes<3>::L1,
                (g.grid[0] + E0 - 1) / E0);
}

}  // namespace

hipError_t launch_prep(const Geo &g, const Seeds &sd, Scalars *sc, uint64_t *mom, double *eig,
                       hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_prep<2><<<1, 1024, 0, st>>>(g, sd, sc, mom, eig);
    else k_prep<3><<<1, 1024, 0, st>>>(g, sd, sc, mom, eig);
    return hipGetLastError();
}

hipError_t launch_assign_fp64(const Geo &g, const Seeds &sd, const Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_assign_fp64<2><<<tile_grid<2>(g), kThreads, 0, st>>>(g, sd, sc, out);
    else k_assign_fp64<3><<<tile_grid<3>(g), kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_assign_fp32(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_assign_fp32<2><<<tile_grid<2, kPv>(g), kThreads, 0, st>>>(g, sd, sc, out);
    else k_assign_fp32<3><<<tile_grid<3, kPv>(g), kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_assign_cull(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                              const PassOut &out, hipStream_t st) {
    (void)hipGetLastError();
    if (g.dim == 2) k_assign_cull<2><<<tile_grid<2, kPv>(g), kThreads, 0, st>>>(g, sd, sc, eig, out);
    else k_assign_cull<3><<<tile_grid<3, kPv>(g), kThreads, 0, st>>>(g, sd, sc, eig, out);
    return hipGetLastError();
}

hipError_t launch_assign_mfma(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) {
        dim3 grid((g.grid[1] + 31) / 32, (g.grid[0] + kExt0 - 1) / kExt0, 1);
        k_assign_mfma<2><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    } else {
        dim3 grid((g.grid[2] + 7) / 8, (g.grid[1] + 3) / 4, (g.grid[0] + kExt0 - 1) / kExt0);
        k_assign_mfma<3><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    }
    return hipGetLastError();
}

hipError_t launch_assign_bf16(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();
    if (g.dim == 2) {
        dim3 grid((g.grid[1] + 31) / 32, (g.grid[0] + kExt0 - 1) / kExt0, 1);
        k_assign_bf16<2><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    } else {
        dim3 grid((g.grid[2] + 7) / 8, (g.grid[1] + 3) / 4, (g.grid[0] + kExt0 - 1) / kExt0);
        k_assign_bf16<3><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    }
    return hipGetLastError();
}

hipError_t launch_recheck(const Geo &g, const Seeds &sd, const Scalars *sc, const PassOut &out,
                          hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_recheck<2><<<512, kThreads, 0, st>>>(g, sd, sc, out);
    else k_recheck<3><<<512, kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const Geo &g, const Seeds &sd, const uint64_t *mom, Scalars *sc,
                           const FinalOut &out, hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_finalize<2><<<1, 1024, 0, st>>>(g, sd, mom, sc, out);
    else k_finalize<3><<<1, 1024, 0, st>>>(g, sd, mom, sc, out);
    return hipGetLastError();
}

}  // namespace apd
