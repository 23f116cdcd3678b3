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
#include "apd_internal.h"

#include <math.h>

namespace apd {
namespace {

// ------------------------------------------------------------ tile layout

// A block covers a tile of pixels.  Its 4 waves are stacked along axis 0;
// each lane owns kP pixels along axis 0 and a fixed position on the other
// axes (2D: 64 lanes along axis 1; 3D: 8 x 8 lanes on axes 1 and 2), so
// consecutive lanes touch consecutive pixel indices.
template <int D> struct Lanes;
template <> struct Lanes<2> { static constexpr int L1 = 64, L2 = 1; };
template <> struct Lanes<3> { static constexpr int L1 = 8, L2 = 8; };

constexpr int kExt0 = kWaves * kP;  // tile extent along axis 0

template <int D>
struct Tile {
    int k0w;         // axis-0 index of this wave's first pixel
    int k[3];        // this lane's pixel indices (k[0] of p = 0)
    int org[3];      // wave origin (k of lane 0, p = 0)
    int anc[3];      // tile anchor (centre) in index units
    int lane;
};

template <int D>
__device__ inline Tile<D> tile_of(const Geo &g) {
    Tile<D> t;
    const int lane = __lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    t.lane = lane;
    if (D == 2) {
        const int b1 = blockIdx.x, b0 = blockIdx.y;
        t.org[0] = b0 * kExt0 + wave * kP;
        t.org[1] = b1 * Lanes<2>::L1;
        t.org[2] = 0;
        t.k[0] = t.org[0];
        t.k[1] = t.org[1] + lane;
        t.k[2] = 0;
        t.anc[0] = b0 * kExt0 + kExt0 / 2;
        t.anc[1] = b1 * Lanes<2>::L1 + Lanes<2>::L1 / 2;
        t.anc[2] = 0;
    } else {
        const int b2 = blockIdx.x, b1 = blockIdx.y, b0 = blockIdx.z;
        t.org[0] = b0 * kExt0 + wave * kP;
        t.org[1] = b1 * Lanes<3>::L1;
        t.org[2] = b2 * Lanes<3>::L2;
        t.k[0] = t.org[0];
        t.k[1] = t.org[1] + (lane >> 3);
        t.k[2] = t.org[2] + (lane & 7);
        t.anc[0] = b0 * kExt0 + kExt0 / 2;
        t.anc[1] = b1 * Lanes<3>::L1 + Lanes<3>::L1 / 2;
        t.anc[2] = b2 * Lanes<3>::L2 + Lanes<3>::L2 / 2;
    }
    t.k0w = t.org[0];
    return t;
}

template <int D>
__device__ inline bool lane_in_grid(const Geo &g, const Tile<D> &t) {
    bool ok = t.k[1] < g.grid[1];
    if (D == 3) ok = ok && t.k[2] < g.grid[2];
    return ok;
}

template <int D>
__device__ inline uint32_t pixel_index(const Geo &g, int k0, const Tile<D> &t) {
    if (D == 2) return (uint32_t)k0 * (uint32_t)g.grid[1] + (uint32_t)t.k[1];
    return ((uint32_t)k0 * (uint32_t)g.grid[1] + (uint32_t)t.k[1]) * (uint32_t)g.grid[2] +
           (uint32_t)t.k[2];
}

// ------------------------------------------------- exact double-precision

// Pixel centre y_d = lo_d + (k_d + 1/2) s_d (eq. (2.6)).
__device__ inline double centre(const Geo &g, int d, int k) {
    return g.lo[d] + ((double)k + 0.5) * g.s[d];
}

// C_ij = (y - x_i)^T A_i (y - x_i) - w_i in the definition's order: d = y - x,
// each row of A d summed left to right, then sum_r d_r (A d)_r left to right.
template <int D>
__device__ inline double exact_cost(const double *__restrict__ x, const double *__restrict__ A,
                                    const double *__restrict__ w, int i, const double *y) {
    double d[D];
#pragma unroll
    for (int r = 0; r < D; ++r) d[r] = y[r] - x[(size_t)i * D + r];
    const double *a = A + (size_t)i * D * D;
    double q = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        double row = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double arc = (r <= c) ? a[r * D + c] : a[c * D + r];
            const double t = arc * d[c];
            row = (c == 0) ? t : row + t;
        }
        const double t = d[r] * row;
        q = (r == 0) ? t : q + t;
    }
    return q - w[i];
}

// --------------------------------------------------------- wave helpers

__device__ inline unsigned wave_sum(unsigned v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------ tile epilogue

// Labels, the re-check queue, and the exact per-cell moments of every
// settled pixel.  For a cell the moments are the pixel count and the sums
// of o_d = 2 k_d + 1 and o_d o_e over its pixels (unsigned 64-bit atomics,
// so the result does not depend on the order of the additions).  Within a
// wave the pixels of one cell are first summed in 32 bits relative to the
// wave origin, then shifted to global coordinates once.
template <int D>
__device__ inline void tile_epilogue(const Geo &g, const Tile<D> &t, const bool (&act)[kP],
                                     const int (&lab)[kP], const bool (&flag)[kP],
                                     const PassOut &out, Scalars *sc) {
    constexpr int K = moments_per_cell(D);
    const int lane = t.lane;
    // labels (queued pixels are overwritten by the re-check)
    if (out.labels) {
#pragma unroll
        for (int p = 0; p < kP; ++p)
            if (act[p]) out.labels[pixel_index<D>(g, t.k0w + p, t)] = lab[p];
    }
    // re-check queue, one atomic per wave and row
    if (out.queue) {
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const bool f = act[p] && flag[p];
            const unsigned long long m = __ballot(f);
            if (m) {
                const int leader = __ffsll(m) - 1;
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&sc->qcount, (unsigned)__popcll(m));
                base = __shfl(base, leader);
                const unsigned below = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                if (f) out.queue[base + below] = pixel_index<D>(g, t.k0w + p, t);
            }
        }
    }
    if (!out.mom) return;
    bool pend[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) pend[p] = act[p] && !flag[p];
    const unsigned o1 = 2u * (unsigned)(t.k[1] - t.org[1]) + 1u;
    const unsigned o2 = D == 3 ? 2u * (unsigned)(t.k[2] - t.org[2]) + 1u : 0u;
    for (;;) {
        int L = -1;
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            if (L < 0) {
                const unsigned long long m = __ballot(pend[p]);
                if (m) L = __shfl(lab[p], __ffsll(m) - 1);
            }
        }
        if (L < 0) break;
        unsigned acc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = 0u;
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            if (pend[p] && lab[p] == L) {
                pend[p] = false;
                const unsigned o0 = 2u * (unsigned)p + 1u;
                if (D == 2) {
                    acc[0] += 1u; acc[1] += o0; acc[2] += o1;
                    acc[3] += o0 * o0; acc[4] += o0 * o1; acc[5] += o1 * o1;
                } else {
                    acc[0] += 1u; acc[1] += o0; acc[2] += o1; acc[3] += o2;
                    acc[4] += o0 * o0; acc[5] += o0 * o1; acc[6] += o0 * o2;
                    acc[7] += o1 * o1; acc[8] += o1 * o2; acc[9] += o2 * o2;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = wave_sum(acc[c]);
        if (lane == 0) {
            // global o = G + local o with G_d = 2 org_d
            const uint64_t m = acc[0];
            uint64_t G[3] = {2ull * (uint64_t)t.org[0], 2ull * (uint64_t)t.org[1],
                             2ull * (uint64_t)t.org[2]};
            uint64_t S1[3], S2[6];
            for (int d = 0; d < D; ++d) S1[d] = m * G[d] + acc[1 + d];
            int c = 0;
            for (int d = 0; d < D; ++d)
                for (int e = d; e < D; ++e, ++c)
                    S2[c] = m * G[d] * G[e] + G[d] * (uint64_t)acc[1 + e] +
                            G[e] * (uint64_t)acc[1 + d] + (uint64_t)acc[1 + D + c];
            unsigned long long *dst = (unsigned long long *)out.mom + (size_t)L * K;
            atomicAdd(dst, (unsigned long long)m);
            for (int d = 0; d < D; ++d) atomicAdd(dst + 1 + d, (unsigned long long)S1[d]);
            for (int q = 0; q < c; ++q) atomicAdd(dst + 1 + D + q, (unsigned long long)S2[q]);
        }
    }
}

// Moments of one pixel in global coordinates (re-check path).
template <int D>
__device__ inline void pixel_moments_add(uint64_t *mom, int L, const int *k) {
    constexpr int K = moments_per_cell(D);
    unsigned long long *dst = (unsigned long long *)mom + (size_t)L * K;
    uint64_t o[3];
    for (int d = 0; d < D; ++d) o[d] = 2ull * (uint64_t)k[d] + 1ull;
    atomicAdd(dst, 1ull);
    for (int d = 0; d < D; ++d) atomicAdd(dst + 1 + d, (unsigned long long)o[d]);
    int c = 0;
    for (int d = 0; d < D; ++d)
        for (int e = d; e < D; ++e, ++c) atomicAdd(dst + 1 + D + c, (unsigned long long)(o[d] * o[e]));
}

// ------------------------------------------------------------- k_prep

template <int D>
__global__ __launch_bounds__(1024) void k_prep(Geo g, Seeds sd, Scalars *sc, uint64_t *mom) {
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

// Single precision with a certified margin.  For the tile anchor a (tile
// centre) and u = y - a, e_i = x_i - a:
//   C_ij = (u - e)^T A (u - e) - w_i' = u^T A u - 2 u^T A e + e^T A e - w_i'
// with w' = w - max w <= 0 (the argmin does not change under a common shift).
// The coefficients of the quadratic in u are formed per tile in LDS; each
// lane evaluates it for its kP pixels along axis 0 as
//   C = (a00 u0 + beta) u0 + alpha,
// beta and alpha being the parts that depend only on the lane's other axes.
//
// Rounding bound: with T the sum of the absolute values of all terms of the
// expansion, |C_fp32 - C| <= rho T, rho = 2^-18 (several times the ~20
// roundings the inputs and the evaluation go through).  For any seed with
// true cost C <= B, T <= 2B + 4 r sqrt(B) + 5 r^2 with r = sqrt(lambda) |u|max
// (lambda bounding every eigenvalue of every A_i).  A pixel is settled when
// C_(2) - C_(1) > 2 rho T(B1), B1 an upper bound of the true C_(1); every
// other pixel goes to the double re-check.
template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_fp32(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    constexpr int NS = D == 2 ? 2 : 3;
    __shared__ float4 sC[NS][kChunk];
    const Tile<D> t = tile_of<D>(g);
    const bool lane_ok = lane_in_grid<D>(g, t);

    float s[3];
    double anc[3];
    for (int d = 0; d < D; ++d) {
        s[d] = (float)g.s[d];
        anc[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
    }
    bool act[kP];
    float u0[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        act[p] = lane_ok && (t.k0w + p) < g.grid[0];
        u0[p] = ((float)(t.k0w + p - t.anc[0]) + 0.5f) * s[0];
    }
    const float u1 = ((float)(t.k[1] - t.anc[1]) + 0.5f) * s[1];
    const float u2 = D == 3 ? ((float)(t.k[2] - t.anc[2]) + 0.5f) * s[2] : 0.0f;

    const double wmax = sc->wmax;
    float best[kP], second[kP];
    int lab[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        best[p] = INFINITY;
        second[p] = INFINITY;
        lab[p] = 0;
    }

    for (int base = 0; base < g.n; base += kChunk) {
        const int cnt = min(kChunk, g.n - base);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += kThreads) {
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
        for (int q = 0; q < cnt; ++q) {
            const int i = base + q;
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
            for (int p = 0; p < kP; ++p) {
                const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                // second = median(best, c, second) is the new runner-up
                second[p] = __builtin_amdgcn_fmed3f(best[p], c, second[p]);
                const bool lt = c < best[p];
                lab[p] = lt ? i : lab[p];
                best[p] = lt ? c : best[p];
            }
        }
    }

    // certification
    float umax2 = 0.0f;
    {
        const float h0 = (0.5f * kExt0 - 0.5f) * s[0];
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
    bool flag[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const float bb = fmaxf(best[p], 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float T = 2.0f * B1 + 4.0f * r * sqrtf(B1) + 5.0f * r2;
        flag[p] = !((second[p] - best[p]) > 2.0f * rho * T);
    }
    tile_epilogue<D>(g, t, act, lab, flag, out, sc);
}

// ------------------------------------------------------ k_assign_mfma

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// Single precision on the matrix cores.  The cost of seed i at pixel j in
// tile-local coordinates is a dot product of K = 6 (2D) or 10 (3D) terms,
//   C_ij = sum_k c_k(i) phi_k(u_j),
// c = (a00, 2a01, a11, -2(Ae)_0, -2(Ae)_1, e^T A e - w') and
// phi = (u0^2, u0 u1, u1^2, u0, u1, 1) in 2D (the 3D analogue has K = 10),
// so a 32-seed x 32-pixel block of costs is K/2 v_mfma_f32_32x32x2f32 with
// the seeds on the rows (operand A) and the pixels on the columns (operand
// B).  Each lane's 16 accumulators then hold one pixel against 16 seeds, and
// the running argmin stays inside the lane: the cost's float bits, whose low
// 4 mantissa bits are replaced by the accumulator number, order like the
// costs as signed integers, so min and med3 track the best and the
// runner-up in 3 ALU operations per pair.  The 32-seed block that last
// improved the best is recorded per pixel; the two half-waves, which hold
// the same pixels against the other 16 seeds, are merged at the end.
//
// Accumulator layout of the 32x32x2 f32 MFMA (one block): register r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
//
// Rounding bound as for k_assign_fp32, plus the 4 dropped mantissa bits
// (2^-19 relative of each compared cost).
template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_mfma(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    constexpr int KK = D == 2 ? 3 : 5;    // MFMA steps, K = 2 KK
    constexpr int SPS = D == 2 ? 8 : 16;  // floats per seed in LDS (two parity halves)
    constexpr int G = kP;                 // 32-pixel groups per wave, stacked on axis 0
    constexpr int E1 = D == 2 ? 32 : 4;   // group extent on axis 1
    constexpr int E2 = D == 2 ? 1 : 8;    // group extent on axis 2
    constexpr float kPad = 1.7e38f;       // cost of padding seeds
    __shared__ __attribute__((aligned(16))) float sC[kChunk * SPS];

    const int lane = __lane_id();
    const int half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    Tile<D> t;
    t.lane = lane;
    if (D == 2) {
        t.org[0] = blockIdx.y * kExt0 + wave * G;
        t.org[1] = blockIdx.x * E1;
        t.org[2] = 0;
        t.k[1] = t.org[1] + col;
        t.k[2] = 0;
        t.anc[0] = blockIdx.y * kExt0 + kExt0 / 2;
        t.anc[1] = blockIdx.x * E1 + E1 / 2;
        t.anc[2] = 0;
    } else {
        t.org[0] = blockIdx.z * kExt0 + wave * G;
        t.org[1] = blockIdx.y * E1;
        t.org[2] = blockIdx.x * E2;
        t.k[1] = t.org[1] + col / E2;
        t.k[2] = t.org[2] + col % E2;
        t.anc[0] = blockIdx.z * kExt0 + kExt0 / 2;
        t.anc[1] = blockIdx.y * E1 + E1 / 2;
        t.anc[2] = blockIdx.x * E2 + E2 / 2;
    }
    t.k[0] = t.org[0];
    t.k0w = t.org[0];
    bool lane_ok = t.k[1] < g.grid[1];
    if (D == 3) lane_ok = lane_ok && t.k[2] < g.grid[2];

    float s[3];
    double anc[3];
    for (int d = 0; d < D; ++d) {
        s[d] = (float)g.s[d];
        anc[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
    }
    // operand B: features of this lane's pixel in every group, parity = half
    float bf[G][KK];
    bool act[kP];
    {
        const float u1 = ((float)(t.k[1] - t.anc[1]) + 0.5f) * s[1];
        const float u2 = D == 3 ? ((float)(t.k[2] - t.anc[2]) + 0.5f) * s[2] : 0.0f;
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
            act[gi] = lane_ok && half == 0 && (t.k0w + gi) < g.grid[0];
            const float u0 = ((float)(t.k0w + gi - t.anc[0]) + 0.5f) * s[0];
            if (D == 2) {
                const float ev[3] = {u0 * u0, u1 * u1, u1};
                const float od[3] = {u0 * u1, u0, 1.0f};
#pragma unroll
                for (int q = 0; q < KK; ++q) bf[gi][q] = half ? od[q] : ev[q];
            } else {
                const float ev[5] = {u0 * u0, u0 * u2, u1 * u2, u0, u2};
                const float od[5] = {u0 * u1, u1 * u1, u2 * u2, u1, 1.0f};
#pragma unroll
                for (int q = 0; q < KK; ++q) bf[gi][q] = half ? od[q] : ev[q];
            }
        }
    }

    const double wmax = sc->wmax;
    int best[G], second[G], blk[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        best[gi] = 0x7fffffff;
        second[gi] = 0x7fffffff;
        blk[gi] = 0;
    }

    for (int base = 0; base < g.n; base += kChunk) {
        const int cnt = min(kChunk, g.n - base);
        const int padded = (cnt + 31) & ~31;
        __syncthreads();
        for (int q = threadIdx.x; q < padded; q += kThreads) {
            float *dst = sC + q * SPS;
            if (q >= cnt) {
                for (int z = 0; z < SPS; ++z) dst[z] = 0.0f;
                dst[SPS / 2 + KK - 1] = kPad;  // the constant term (odd parity, last step)
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
                // even k: a00, a11, -2(Ae)_1 ; odd k: 2a01, -2(Ae)_0, cc
                dst[0] = a00; dst[1] = a11; dst[2] = -2.0f * ae1; dst[3] = 0.0f;
                dst[4] = 2.0f * a01; dst[5] = -2.0f * ae0; dst[6] = cc; dst[7] = 0.0f;
            } else {
                const float a00 = (float)a[0], a01 = (float)a[1], a02 = (float)a[2];
                const float a11 = (float)a[4], a12 = (float)a[5], a22 = (float)a[8];
                const float ae0 = fmaf(a00, e[0], fmaf(a01, e[1], a02 * e[2]));
                const float ae1 = fmaf(a01, e[0], fmaf(a11, e[1], a12 * e[2]));
                const float ae2 = fmaf(a02, e[0], fmaf(a12, e[1], a22 * e[2]));
                const float cc = fmaf(e[0], ae0, fmaf(e[1], ae1, e[2] * ae2)) - wp;
                // even k: a00, 2a02, 2a12, -2(Ae)_0, -2(Ae)_2
                // odd k:  2a01, a11, a22, -2(Ae)_1, cc
                dst[0] = a00; dst[1] = 2.0f * a02; dst[2] = 2.0f * a12; dst[3] = -2.0f * ae0;
                dst[4] = -2.0f * ae2; dst[5] = 0.0f; dst[6] = 0.0f; dst[7] = 0.0f;
                dst[8] = 2.0f * a01; dst[9] = a11; dst[10] = a22; dst[11] = -2.0f * ae1;
                dst[12] = cc; dst[13] = 0.0f; dst[14] = 0.0f; dst[15] = 0.0f;
            }
        }
        __syncthreads();
        for (int cb = 0; cb < padded; cb += 32) {
            const float *src = sC + (cb + col) * SPS + half * (SPS / 2);
            float av[KK];
            {
                const float4 v0 = *reinterpret_cast<const float4 *>(src);
                av[0] = v0.x; av[1] = v0.y; av[2] = v0.z;
                if (D == 3) {
                    const float4 v1 = *reinterpret_cast<const float4 *>(src + 4);
                    av[3] = v0.w; av[4] = v1.x;
                }
            }
            const int sblk = base + cb;
            // all groups' products first, so the matrix cores run ahead of
            // the ALU work of the argmin
            floatx16 acc[G];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
                acc[gi] = floatx16{};
#pragma unroll
                for (int q = 0; q < KK; ++q)
                    acc[gi] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q], bf[gi][q], acc[gi], 0, 0, 0);
            }
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
                const int old = best[gi];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int key = (__float_as_int(acc[gi][r]) & ~15) | r;
                    second[gi] = med3i(best[gi], key, second[gi]);
                    best[gi] = min(best[gi], key);
                }
                blk[gi] = (best[gi] != old) ? sblk : blk[gi];
            }
        }
    }

    // merge the half-waves, decode the seed, certify
    float umax2;
    {
        const float h0 = (0.5f * kExt0 - 0.5f) * s[0];
        const float h1 = (0.5f * E1 - 0.5f) * s[1];
        umax2 = h0 * h0 + h1 * h1;
        if (D == 3) {
            const float h2 = (0.5f * E2 - 0.5f) * s[2];
            umax2 += h2 * h2;
        }
    }
    const float r2 = sc->lam * umax2 * 1.01f;
    const float rr = sqrtf(r2);
    constexpr float rho = 0x1p-18f;
    int lab[kP];
    bool flag[kP];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        const int r = best[gi] & 15;
        const int seed = blk[gi] + 8 * (r >> 2) + 4 * half + (r & 3);
        const int ob = __shfl_xor(best[gi], 32);
        const int os = __shfl_xor(second[gi], 32);
        const int oseed = __shfl_xor(seed, 32);
        const bool other = ob < best[gi] || (ob == best[gi] && oseed < seed);
        const int nb = other ? ob : best[gi];
        const int ns = min(max(best[gi], ob), min(second[gi], os));
        lab[gi] = min(other ? oseed : seed, g.n - 1);
        const float fb = __int_as_float(nb), fs = __int_as_float(ns);
        const float bb = fmaxf(fb, 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float T = 2.0f * B1 + 4.0f * rr * sqrtf(B1) + 5.0f * r2;
        const float thr = 2.0f * rho * T + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fs));
        flag[gi] = !((fs - fb) > thr);
    }
    tile_epilogue<D>(g, t, act, lab, flag, out, sc);
}

// ---------------------------------------------------------- k_recheck

// One wave per queued pixel: lanes stride over the seeds with the exact
// double cost, then a (value, index) minimum across the wave gives the
// lowest index attaining the minimum, as a sequential scan would.
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
        uint32_t r = j;
        for (int d = D - 1; d >= 0; --d) {
            k[d] = (int)(r % (uint32_t)g.grid[d]);
            r /= (uint32_t)g.grid[d];
        }
        double y[D];
        for (int d = 0; d < D; ++d) y[d] = centre(g, d, k[d]);
        double b = INFINITY;
        int bi = 0x7fffffff;
        for (int i = lane; i < g.n; i += 64) {
            const double c = exact_cost<D>(sd.x, sd.A, sd.w, i, y);
            if (c < b) {
                b = c;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(b, o);
            const int oi = __shfl_xor(bi, o);
            if (ob < b || (ob == b && oi < bi)) {
                b = ob;
                bi = oi;
            }
        }
        if (bi >= g.n) bi = 0;  // no finite cost (non-finite input, reported by k_prep)
        if (lane == 0) {
            if (out.labels) out.labels[j] = bi;
            if (out.mom) pixel_moments_add<D>(out.mom, bi, k);
        }
    }
}

// -------------------------------------------------------- k_finalize

// Per cell from the exact moments (o = 2k + 1, y = lo + h o with h = s/2):
//   m_i, grad_i = v_i - m_i |P|                                  eq. (2.8)
//   centroid ybar = lo + h S_d / m                                 Alg. 3
//   sum_{cell} |y - x_i|^2_A = m |ybar - x_i|^2_A
//                              + sum_de A_de h_d h_e (S_de - S_d S_e / m)
//   g~ = sum_i [(v_i - m_i |P|) w_i + |P| sum_{cell} |y - x_i|^2_A]  eq. (2.7)
// summed over cells in a fixed order (deterministic).
template <int D>
__global__ __launch_bounds__(1024) void k_finalize(Geo g, Seeds sd, const uint64_t *mom,
                                                  Scalars *sc, FinalOut out) {
    constexpr int K = moments_per_cell(D);
    __shared__ double s_g[1024];
    __shared__ double s_m[1024];
    const int tid = threadIdx.x;
    double h[3];
    for (int d = 0; d < D; ++d) h[d] = 0.5 * g.s[d];
    double gs = 0.0, mr = 0.0;
    for (int i = tid; i < g.n; i += 1024) {
        const uint64_t *M = mom + (size_t)i * K;
        const uint64_t m = M[0];
        const double md = (double)m;
        const double vi = sd.v[i], wi = sd.w[i];
        const double gi = vi - md * g.pixvol;
        mr = fmax(mr, fabs(gi) / vi);
        const double *a = sd.A + (size_t)i * D * D;
        double integral = 0.0;
        double ybar[3];
        if (m > 0) {
            double S1[3], dev[3];
            for (int d = 0; d < D; ++d) {
                S1[d] = (double)M[1 + d];
                ybar[d] = g.lo[d] + h[d] * (S1[d] / md);
                dev[d] = ybar[d] - sd.x[(size_t)i * D + d];
            }
            double q1 = 0.0, q2 = 0.0;
            int c = 0;
            for (int d = 0; d < D; ++d)
                for (int e = d; e < D; ++e, ++c) {
                    const double ade = a[d * D + e] * (d == e ? 1.0 : 2.0);
                    const double cov = (double)M[1 + D + c] - S1[d] * (S1[e] / md);
                    q1 += ade * dev[d] * dev[e];
                    q2 += ade * h[d] * h[e] * cov;
                }
            integral = g.pixvol * (md * q1 + q2);
        } else {
            for (int d = 0; d < D; ++d) ybar[d] = sd.x[(size_t)i * D + d];
        }
        gs += gi * wi + integral;
        if (out.grad) out.grad[i] = gi;
        if (out.counts) out.counts[i] = (int64_t)m;
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

template <int D>
dim3 tile_grid(const Geo &g) {
    if (D == 2)
        return dim3((g.grid[1] + Lanes<2>::L1 - 1) / Lanes<2>::L1, (g.grid[0] + kExt0 - 1) / kExt0, 1);
    return dim3((g.grid[2] + Lanes<3>::L2 - 1) / Lanes<3>::L2, (g.grid[1] + Lanes<3>::L1 - 1) / Lanes<3>::L1,
                (g.grid[0] + kExt0 - 1) / kExt0);
}

}  // namespace

hipError_t launch_prep(const Geo &g, const Seeds &sd, Scalars *sc, uint64_t *mom, hipStream_t st) {
    if (g.dim == 2) k_prep<2><<<1, 1024, 0, st>>>(g, sd, sc, mom);
    else k_prep<3><<<1, 1024, 0, st>>>(g, sd, sc, mom);
    return hipGetLastError();
}

hipError_t launch_assign_fp64(const Geo &g, const Seeds &sd, const Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    if (g.dim == 2) k_assign_fp64<2><<<tile_grid<2>(g), kThreads, 0, st>>>(g, sd, sc, out);
    else k_assign_fp64<3><<<tile_grid<3>(g), kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_assign_fp32(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    if (g.dim == 2) k_assign_fp32<2><<<tile_grid<2>(g), kThreads, 0, st>>>(g, sd, sc, out);
    else k_assign_fp32<3><<<tile_grid<3>(g), kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_assign_mfma(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    if (g.dim == 2) {
        dim3 grid((g.grid[1] + 31) / 32, (g.grid[0] + kExt0 - 1) / kExt0, 1);
        k_assign_mfma<2><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    } else {
        dim3 grid((g.grid[2] + 7) / 8, (g.grid[1] + 3) / 4, (g.grid[0] + kExt0 - 1) / kExt0);
        k_assign_mfma<3><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    }
    return hipGetLastError();
}

hipError_t launch_recheck(const Geo &g, const Seeds &sd, const Scalars *sc, const PassOut &out,
                          hipStream_t st) {
    if (g.dim == 2) k_recheck<2><<<512, kThreads, 0, st>>>(g, sd, sc, out);
    else k_recheck<3><<<512, kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const Geo &g, const Seeds &sd, const uint64_t *mom, Scalars *sc,
                           const FinalOut &out, hipStream_t st) {
    if (g.dim == 2) k_finalize<2><<<1, 1024, 0, st>>>(g, sd, mom, sc, out);
    else k_finalize<3><<<1, 1024, 0, st>>>(g, sd, mom, sc, out);
    return hipGetLastError();
}

}  // namespace apd
