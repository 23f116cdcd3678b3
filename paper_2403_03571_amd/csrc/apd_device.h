// apd_device.h -- device building blocks shared by the single-instance and
// the batched kernels of libapd: tile layout, the exact double cost, the
// per-tile epilogue (labels, re-check queue, exact integer moments), the
// matrix-core assignment of one tile, the double re-check of one pixel and
// the finalize of one cell.  Included by the .hip sources only.
#pragma once

#include "apd_internal.h"

#include <math.h>

namespace apd {
namespace dev {

// ------------------------------------------------------------ tile layout

// A block covers a tile of pixels (tile_ext: 2D 8P x 32 as 2 x 2 waves of
// 4 x 16 lanes, 3D 4P x 8 x 8 as 4 waves stacked along axis 0); each lane
// owns P consecutive pixels along axis 0 and a fixed position on the other
// axes, so consecutive lanes touch consecutive pixel indices along the
// last axis.

constexpr int kExt0 = kWaves * kP;  // extent along axis 0 of the matrix-core tile

template <int D>
struct Tile {
    int k0w;         // axis-0 index of this lane's first pixel
    int k[3];        // this lane's pixel indices (k[0] of p = 0)
    int org[3];      // origin of this wave's box of pixels
    int anc[3];      // tile anchor (centre) in index units
    int lane;
};

// Axis-0 index of the first pixel and the other indices of lane L of a wave
// whose box starts at org.
template <int D, int P>
__device__ inline void lane_pixel(const int *org, int L, int &k0, int &k1, int &k2) {
    if (D == 2) {
        k0 = org[0] + (L >> 4) * P;
        k1 = org[1] + (L & 15);
        k2 = 0;
    } else {
        k0 = org[0];
        k1 = org[1] + (L >> 3);
        k2 = org[2] + (L & 7);
    }
}

// Tile (b0, b1, b2): b0 along axis 0, b1 along axis 1, b2 along axis 2.
template <int D, int P = kP>
__device__ inline Tile<D> tile_at(int b0, int b1, int b2) {
    constexpr int E0 = tile_ext(D, P, 0), E1 = tile_ext(D, P, 1), E2 = tile_ext(D, P, 2);
    Tile<D> t;
    const int lane = __lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    t.lane = lane;
    if (D == 2) {
        t.org[0] = b0 * E0 + (wave >> 1) * wave_ext(D, P, 0);
        t.org[1] = b1 * E1 + (wave & 1) * wave_ext(D, P, 1);
        t.org[2] = 0;
    } else {
        t.org[0] = b0 * E0 + wave * P;
        t.org[1] = b1 * E1;
        t.org[2] = b2 * E2;
    }
    lane_pixel<D, P>(t.org, lane, t.k0w, t.k[1], t.k[2]);
    t.k[0] = t.k0w;
    t.anc[0] = b0 * E0 + E0 / 2;
    t.anc[1] = b1 * E1 + E1 / 2;
    t.anc[2] = D == 3 ? b2 * E2 + E2 / 2 : 0;
    return t;
}

// The tile of this block (grid x along the last axis).
template <int D, int P = kP>
__device__ inline Tile<D> tile_of(const Geo &g) {
    if (D == 2) return tile_at<D, P>(blockIdx.y, blockIdx.x, 0);
    return tile_at<D, P>(blockIdx.z, blockIdx.y, blockIdx.x);
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
// For power p != 2 the cost is |y - x_i|_{A_i}^p - w_i, from the squared
// norm q clamped at 0 as sqrt(q) (p = 1), q sqrt(q) (p = 3) or q q (p = 4).
template <int D>
__device__ inline double exact_cost(const double *__restrict__ x, const double *__restrict__ A,
                                    const double *__restrict__ w, int i, const double *y, int power = 2) {
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
    if (power != 2) {
        const double qc = q > 0.0 ? q : 0.0;
        q = power == 1 ? sqrt(qc) : power == 3 ? qc * sqrt(qc) : qc * qc;
    }
    return q - w[i];
}

// The expanded cost of seed i about a tile anchor, for the single-precision
// tiers: with e = x_i - anchor and u = y - anchor,
//   C_i(u) = sum_{d<=e'} q_de' u_d u_e' + sum_d l_d u_d + c,
// q the upper triangle of A_i with the off-diagonal entries doubled (2D:
// a00, 2a01, a11; 3D: a00, 2a01, 2a02, a11, 2a12, a22), l = -2 A_i e and
// c = e^T A_i e - (w_i - w_max).  Computed in double, so that rounding each
// to FP32 once leaves it within 2^-24 of its own value, whatever the
// conditioning of A_i (in FP32 the cancellation in e^T A e could cost up to
// the condition number times that).
template <int D>
__device__ inline void seed_terms(const Seeds &sd, int i, const double *anc, double wmax, double *q,
                                  double *l, double *c, double *e, double *wp) {
    const double *xi = sd.x + (size_t)i * D;
    const double *a = sd.A + (size_t)i * D * D;
    for (int d = 0; d < D; ++d) e[d] = xi[d] - anc[d];
    *wp = sd.w[i] - wmax;
    double ee = 0.0;
    for (int r = 0; r < D; ++r) {
        double ae = 0.0;
        for (int k = 0; k < D; ++k) ae += a[(r <= k) ? r * D + k : k * D + r] * e[k];
        l[r] = -2.0 * ae;
        ee += e[r] * ae;
    }
    *c = ee - *wp;
    int t = 0;
    for (int r = 0; r < D; ++r)
        for (int k = r; k < D; ++k) q[t++] = (r == k ? 1.0 : 2.0) * a[r * D + k];
}

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

// --------------------------------------------------------- wave helpers

// The wave's total of v, wave-uniform, without LDS round trips: DPP adds
// within each row of 16 lanes (lane xor 1, xor 2, then the half-row and
// row mirrors), so that every lane of a row holds the row's sum, then the
// four row sums read from lanes 0, 16, 32, 48.  All lanes must be active.
__device__ inline unsigned wave_total(unsigned v) {
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    return (unsigned)__builtin_amdgcn_readlane((int)v, 0) + (unsigned)__builtin_amdgcn_readlane((int)v, 16) +
           (unsigned)__builtin_amdgcn_readlane((int)v, 32) + (unsigned)__builtin_amdgcn_readlane((int)v, 48);
}

// The wave's minimum, wave-uniform, the same way (float and double).
__device__ inline float wave_min(float v) {
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)));
    v = fminf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)));
    const int b = __float_as_int(v);
    return fminf(fminf(__int_as_float(__builtin_amdgcn_readlane(b, 0)), __int_as_float(__builtin_amdgcn_readlane(b, 16))),
                 fminf(__int_as_float(__builtin_amdgcn_readlane(b, 32)), __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}
template <int CTRL>
__device__ inline double dpp_double(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double lane_double(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double wave_min(double v) {
    v = fmin(v, dpp_double<0xB1>(v));
    v = fmin(v, dpp_double<0x4E>(v));
    v = fmin(v, dpp_double<0x141>(v));
    v = fmin(v, dpp_double<0x140>(v));
    return fmin(fmin(lane_double(v, 0), lane_double(v, 16)), fmin(lane_double(v, 32), lane_double(v, 48)));
}

// ------------------------------------------------------ tile epilogue

// Labels, the re-check queue, and the exact per-cell moments of every
// settled pixel.  For a cell the moments are the pixel count and the sums
// of o_d = 2 k_d + 1 and o_d o_e over its pixels (unsigned 64-bit atomics,
// so the result does not depend on the order of the additions).  Within a
// wave the pixels of one cell are first summed in 32 bits relative to the
// wave origin, then shifted to global coordinates once.
template <int D, int P = kP>
__device__ inline void tile_epilogue(const Geo &g, const Tile<D> &t, const bool (&act)[P],
                                     const int (&lab)[P], const bool (&flag)[P],
                                     const PassOut &out, unsigned *qcount) {
    constexpr int K = moments_per_cell(D);
    const int lane = t.lane;
    // labels (queued pixels are overwritten by the re-check)
    if (out.labels) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (act[p]) out.labels[pixel_index<D>(g, t.k0w + p, t)] = lab[p];
    }
    // re-check queue: one atomic per block (the counter is a single address
    // shared by every block of the pass).  Every thread of the block comes
    // here (the queue pointers are uniform), so the barriers are safe.
    if (out.queue || out.queue64) {
        __shared__ unsigned s_q[kWaves + 1];
        const int wave = threadIdx.x >> 6;
        unsigned long long mk[P];
        unsigned tot = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            mk[p] = __ballot(act[p] && flag[p]);
            tot += (unsigned)__popcll(mk[p]);
        }
        if (lane == 0) s_q[wave] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned all = 0;
            for (int w = 0; w < kWaves; ++w) all += s_q[w];
            unsigned first = 0u;
            if (all && out.segs) {
                // pixels and segments with one atomic on the (pixels,
                // segments) pair
                const unsigned long long old =
                    atomicAdd(reinterpret_cast<unsigned long long *>(qcount), (1ull << 32) | all);
                first = (unsigned)old;
                out.segs[(unsigned)(old >> 32)] = QSeg{first, all, out.tile_id, (int32_t)out.tag};
            } else if (all) {
                first = atomicAdd(qcount, all);
            }
            s_q[kWaves] = first;
        }
        __syncthreads();
        if (tot) {
            unsigned base = s_q[kWaves];
            for (int w = 0; w < wave; ++w) base += s_q[w];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const unsigned long long m = mk[p];
                if (act[p] && flag[p]) {
                    const unsigned below = __builtin_amdgcn_mbcnt_hi(
                        (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                    const uint32_t j = pixel_index<D>(g, t.k0w + p, t);
                    if (out.queue64) out.queue64[base + below] = ((uint64_t)out.tag << 32) | j;
                    else out.queue[base + below] = j;
                }
                base += (unsigned)__popcll(m);
            }
        }
    }
    if (!out.mom) return;
    bool pend[P];
    unsigned qw[P];  // pixel weights (1 without them)
#pragma unroll
    for (int p = 0; p < P; ++p) {
        pend[p] = act[p] && !flag[p];
        qw[p] = (pend[p] && g.mass) ? (unsigned)g.mass[pixel_index<D>(g, t.k0w + p, t)] : 1u;
    }
    // the lane's position on axes 1, 2 is fixed: its pixels' monomials are
    // those of o0 (count, sum, sum of squares) times lane constants
    const unsigned o1 = 2u * (unsigned)(t.k[1] - t.org[1]) + 1u;
    const unsigned o2 = D == 3 ? 2u * (unsigned)(t.k[2] - t.org[2]) + 1u : 0u;
    const uint64_t G[3] = {2ull * (uint64_t)t.org[0], 2ull * (uint64_t)t.org[1],
                           2ull * (uint64_t)t.org[2]};
    for (;;) {
        int L = -1;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (L < 0) {
                const unsigned long long m = __ballot(pend[p]);
                if (m) L = __builtin_amdgcn_readlane(lab[p], __ffsll(m) - 1);
            }
        }
        if (L < 0) break;
        unsigned s0 = 0u, s1 = 0u, s2 = 0u;  // sum q, q o0, q o0^2 over this lane's pixels of L
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (pend[p] && lab[p] == L) {
                pend[p] = false;
                const unsigned o0 = 2u * (unsigned)(t.k0w - t.org[0] + p) + 1u;
                const unsigned q = qw[p];
                s0 += q;
                s1 += q * o0;
                s2 += q * o0 * o0;
            }
        }
        unsigned acc[K];
        if constexpr (D == 2) {
            // 1, o0, o1, o0^2, o0 o1, o1^2
            acc[0] = s0; acc[1] = s1; acc[2] = s0 * o1; acc[3] = s2; acc[4] = s1 * o1; acc[5] = s0 * (o1 * o1);
        } else {
            // 1, o0, o1, o2, o0^2, o0 o1, o0 o2, o1^2, o1 o2, o2^2
            acc[0] = s0; acc[1] = s1; acc[2] = s0 * o1; acc[3] = s0 * o2; acc[4] = s2; acc[5] = s1 * o1;
            acc[6] = s1 * o2; acc[7] = s0 * (o1 * o1); acc[8] = s0 * (o1 * o2); acc[9] = s0 * (o2 * o2);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = wave_total(acc[c]);
        // global o = G + local o with G_d = 2 org_d; every lane forms the
        // cell's K sums, lane q adds the q-th: one instruction, K
        // consecutive 8-byte atomics in one or two 64-byte lines
        const uint64_t m = acc[0];
        uint64_t val[K];
        val[0] = m;
#pragma unroll
        for (int d = 0; d < D; ++d) val[1 + d] = m * G[d] + acc[1 + d];
        {
            int c = 0;
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int e = d; e < D; ++e, ++c)
                    val[1 + D + c] = m * G[d] * G[e] + G[d] * (uint64_t)acc[1 + e] +
                                     G[e] * (uint64_t)acc[1 + d] + (uint64_t)acc[1 + D + c];
        }
        uint64_t mine = 0;
#pragma unroll
        for (int q = 0; q < K; ++q) mine = lane == q ? val[q] : mine;
        if (lane < K)
            atomicAdd((unsigned long long *)out.mom + (size_t)L * K + lane, (unsigned long long)mine);
    }
}

// Moments of one pixel in global coordinates (re-check path).
template <int D>
__device__ inline void pixel_moments_add(uint64_t *mom, int L, const int *k, uint64_t q = 1) {
    constexpr int K = moments_per_cell(D);
    if (q == 0) return;
    unsigned long long *dst = (unsigned long long *)mom + (size_t)L * K;
    uint64_t o[3];
    for (int d = 0; d < D; ++d) o[d] = 2ull * (uint64_t)k[d] + 1ull;
    atomicAdd(dst, (unsigned long long)q);
    for (int d = 0; d < D; ++d) atomicAdd(dst + 1 + d, (unsigned long long)(q * o[d]));
    int c = 0;
    for (int d = 0; d < D; ++d)
        for (int e = d; e < D; ++e, ++c)
            atomicAdd(dst + 1 + D + c, (unsigned long long)(q * o[d] * o[e]));
}

// Moments of a whole box of pixels k_d in [a_d, b_d] in one go (closed
// forms of the sums of o = 2k + 1 and of its products): over an interval
// sum o = (b + 1)^2 - a^2 and sum o^2 = F(b + 1) - F(a), F(K) = K (4K^2 - 1) / 3
// (the sum of the first K odd squares), multiplied by the pixel counts of
// the other axes.  Exact in unsigned 64-bit arithmetic for the grids the
// moments allow.
template <int D>
__device__ inline void box_moments_add(uint64_t *mom, int L, const int *a, const int *b) {
    constexpr int K = moments_per_cell(D);
    uint64_t n[3] = {1, 1, 1}, s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
    auto F = [](uint64_t k) { return k * (4ull * k * k - 1ull) / 3ull; };
    for (int d = 0; d < D; ++d) {
        const uint64_t lo = (uint64_t)a[d], hi = (uint64_t)b[d] + 1ull;
        n[d] = hi - lo;
        s1[d] = hi * hi - lo * lo;
        s2[d] = F(hi) - F(lo);
    }
    uint64_t m = 1;
    for (int d = 0; d < D; ++d) m *= n[d];
    unsigned long long *dst = (unsigned long long *)mom + (size_t)L * K;
    atomicAdd(dst, (unsigned long long)m);
    for (int d = 0; d < D; ++d) atomicAdd(dst + 1 + d, (unsigned long long)(m / n[d] * s1[d]));
    int c = 0;
    for (int d = 0; d < D; ++d)
        for (int e = d; e < D; ++e, ++c) {
            uint64_t v;
            if (d == e) {
                v = m / n[d] * s2[d];
            } else {
                uint64_t rest = 1;
                for (int f = 0; f < D; ++f)
                    if (f != d && f != e) rest *= n[f];
                v = rest * s1[d] * s1[e];
            }
            atomicAdd(dst + 1 + D + c, (unsigned long long)v);
        }
}

// Weight of pixel j in the moments: its q_j with pixel weights, else 1.
__device__ inline unsigned pixel_weight(const Geo &g, uint32_t j) {
    return g.mass ? (unsigned)g.mass[j] : 1u;
}

// ------------------------------------------- slack of the double costs

// The labels must agree with the double-precision evaluation of the
// definition (d = y - x, each row of A d, d^T (A d), minus w), whose own
// rounding is not zero.  For seed i with cost C <= B its error is at most
// 2^-48 ((kappa + 1) B + |w_max| + lambda_G sum_d Y_d^2): the products and
// sums of the form carry at most 12 roundings of 2^-53 each over terms
// summing to |d|^T |A| |d| <= lambda_G |d|^2 <= kappa |d|_A^2 <= kappa C,
// the subtraction of w over |w| <= |w_max| + C, and the rounding of y and d
// (|y_d| <= Y_d = |lo_d| + M_d s_d) adds 2 lambda_G |dd| |d| <= 2^-50
// (lambda_G sum Y_d^2 + 2 kappa C).  The certificates add twice that, with
// 2^-44 in place of 2^-48, to the required gap: the absolute part here, the
// part proportional to B as kslack() (B + r^2) (the r^2 covers the double
// rounding of the expansion's own coefficients, seed_terms, whose terms
// sum to at most lambda_G |e|^2 <= kappa (sqrt(B) + r)^2).
__device__ inline float dslack_abs(const Geo &g, double wmax, Cert ct) {
    double y2 = 0.0;
    for (int d = 0; d < g.dim; ++d) {
        const double y = fabs(g.lo[d]) + (double)g.grid[d] * g.s[d];
        y2 += y * y;
    }
    return (float)(0x1p-44 * (fabs(wmax) + (double)ct.lam * y2));
}
__device__ inline float kslack(Cert ct) { return 0x1p-44f * (ct.kap + 1.0f); }

// Rounding bounds of the single-precision costs (derivations at vec_tile and
// bf16_tile) for any seed whose true cost, in the gauge w - w_max, is at
// most B, at a pixel at offset u from the tile anchor, r^2 = lambda_G |u|^2:
//   FP32 vector tile: gamma_9 S <= 2^-20 (B + 4 r sqrt(B) + 4 r^2)
//                     (gamma_9 = 0.5625 2^-20: a factor 1.78 to spare);
//   bf16 tile:        2^-15 (3 r^2 + 2 r sqrt(B)) + 2^-18 B
//                     (the proven 2^-15 (2.27 r^2 + 1.26 r sqrt(B)) +
//                     1.07 2^-19 B, with room).
__device__ inline float e32_bound(float B, float r, float r2) {
    return 0x1p-20f * (B + 4.0f * r * sqrtf(B) + 4.0f * r2);
}
__device__ inline float e16_bound(float B, float r, float r2) {
    return 0x1p-15f * (3.0f * r2 + 2.0f * r * sqrtf(B)) + 0x1p-18f * B;
}
// r^2 of a pixel at offset u (1.01 covers the FP32 rounding of this product)
__device__ inline float pixel_r2(Cert ct, float u0, float u1, float u2) {
    return ct.lam * fmaf(u0, u0, fmaf(u1, u1, u2 * u2)) * 1.01f;
}

// Certified lower bound of the relative top-two gap (C_(2) - C_(1)) / C_(2)
// (costs in the gauge w - w_max, so non-negative) of a settled pixel, from
// an upper bound c1u of the winner's true cost and a lower bound c2l of
// every other seed's: 1 - c1u / c2l, made smaller by 2^-20 for the FP32
// rounding of this expression; 0 when c2l <= 0, 1 when it is infinite.
// Costs of 1e37 and above are those of padding slots (1.7e38): pad_inf maps
// them to +infinity before any bound is formed, so nothing overflows.
__device__ inline float pad_inf(float c) { return c >= 1e37f ? INFINITY : c; }
__device__ inline float gap_lower(float c1u, float c2l) {
    if (c2l == INFINITY) return 1.0f;  // no other seed (only padding)
    if (!(c2l > 0.0f)) return 0.0f;
    const float g = (c2l - c1u) / c2l * (1.0f - 0x1p-20f);
    return g > 0.0f ? fminf(g, 1.0f) : 0.0f;
}
// The gap in double from the exact best and runner-up costs b <= s of the
// definition (weights not shifted): (s - b) / (s + w_max), rounded down to
// FP32; 1 for a single seed (s infinite).
__device__ inline float gap_exact(double b, double s, double wmax) {
    if (isinf(s) && s > 0.0) return 1.0f;
    const double den = s + wmax;
    if (!(den > 0.0)) return 0.0f;
    const double g = (s - b) / den;
    return g > 0.0 ? __double2float_rd(g) : 0.0f;
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
// Tile (b0, b1, b2) of the grid: b0 along axis 0, b1 along axis 1, b2 along
// axis 2 (3D).  sC is the block's LDS staging area (kMfmaLds floats).
template <int D>
__device__ inline void mfma_tile(const Geo &g, const Seeds &sd, double wmax, Cert ct, int b0,
                                 int b1, int b2, float *sC, const PassOut &out,
                                 unsigned *qcount) {
    constexpr int KK = D == 2 ? 3 : 5;    // MFMA steps, K = 2 KK
    constexpr int SPS = D == 2 ? 8 : 16;  // floats per seed in LDS (two parity halves)
    constexpr int G = kP;                 // 32-pixel groups per wave, stacked on axis 0
    constexpr int E1 = D == 2 ? 32 : 4;   // group extent on axis 1
    constexpr int E2 = D == 2 ? 1 : 8;    // group extent on axis 2
    constexpr float kPad = 1.7e38f;       // cost of padding seeds

    const int lane = __lane_id();
    const int half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    Tile<D> t;
    t.lane = lane;
    if (D == 2) {
        t.org[0] = b0 * kExt0 + wave * G;
        t.org[1] = b1 * E1;
        t.org[2] = 0;
        t.k[1] = t.org[1] + col;
        t.k[2] = 0;
        t.anc[0] = b0 * kExt0 + kExt0 / 2;
        t.anc[1] = b1 * E1 + E1 / 2;
        t.anc[2] = 0;
    } else {
        t.org[0] = b0 * kExt0 + wave * G;
        t.org[1] = b1 * E1;
        t.org[2] = b2 * E2;
        t.k[1] = t.org[1] + col / E2;
        t.k[2] = t.org[2] + col % E2;
        t.anc[0] = b0 * kExt0 + kExt0 / 2;
        t.anc[1] = b1 * E1 + E1 / 2;
        t.anc[2] = b2 * E2 + E2 / 2;
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
            double qd[6], ld[3], cd, ed[3], wpd;
            seed_terms<D>(sd, i, anc, wmax, qd, ld, &cd, ed, &wpd);
            if (D == 2) {
                // even k: a00, a11, -2(Ae)_1 ; odd k: 2a01, -2(Ae)_0, cc
                dst[0] = (float)qd[0]; dst[1] = (float)qd[2]; dst[2] = (float)ld[1]; dst[3] = 0.0f;
                dst[4] = (float)qd[1]; dst[5] = (float)ld[0]; dst[6] = (float)cd; dst[7] = 0.0f;
            } else {
                // even k: a00, 2a02, 2a12, -2(Ae)_0, -2(Ae)_2
                // odd k:  2a01, a11, a22, -2(Ae)_1, cc
                dst[0] = (float)qd[0]; dst[1] = (float)qd[2]; dst[2] = (float)qd[4]; dst[3] = (float)ld[0];
                dst[4] = (float)ld[2]; dst[5] = 0.0f; dst[6] = 0.0f; dst[7] = 0.0f;
                dst[8] = (float)qd[1]; dst[9] = (float)qd[3]; dst[10] = (float)qd[5]; dst[11] = (float)ld[1];
                dst[12] = (float)cd; dst[13] = 0.0f; dst[14] = 0.0f; dst[15] = 0.0f;
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
    const float r2 = ct.lam * umax2 * 1.01f;
    const float sab = dslack_abs(g, wmax, ct), skb = kslack(ct);
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
        const float thr = 2.0f * rho * T + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fs)) + sab + skb * (B1 + r2);
        flag[gi] = !((fs - fb) > thr);
        if (out.rel_gap && act[gi] && !flag[gi]) {
            const float c1u = (fb + 0x1p-19f * fabsf(fb) + rho * T + sab + skb * (B1 + r2)) * (1.0f + 0x1p-20f);
            const float f2 = pad_inf(fs);
            const float bs = fmaxf(f2, 0.0f);
            const float B2 = bs + 0x1p-10f * (bs + r2);
            const float eT2 = rho * (2.0f * B2 + 4.0f * rr * sqrtf(B2) + 5.0f * r2);
            const float c2l =
                f2 == INFINITY ? f2 : (f2 - 0x1p-19f * fabsf(f2) - eT2 - sab - skb * (B2 + r2)) * (1.0f - 0x1p-20f);
            out.rel_gap[pixel_index<D>(g, t.k0w + gi, t)] = fs > 0.0f ? gap_lower(c1u, c2l) : 0.0f;
        }
    }
    tile_epilogue<D>(g, t, act, lab, flag, out, qcount);
}

// ------------------------------------------------- vector fp32 tile

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
// Rounding bound.  Write the cost as the sum of its monomials m: q_de u_d u_e,
// l_d u_d and c, and let S = sum |m|.  Each monomial reaches the computed
// cost through at most 9 roundings of relative size 2^-24 (3D; 8 in 2D):
// its FP32 coefficient (1; formed in double, seed_terms), its factors
// u_d = fl(fl(s_d) (k_d - a_d + 1/2)) (2 each, at most 2 factors) and the
// fused multiply-adds on its way (2 inside beta or alpha, then the 2 of
// the Horner step), so |C_fp32 - C| <= gamma_9 S, gamma_9 = 9u/(1 - 9u)
// < 2^-20 (u = 2^-24).  For a seed of true cost C: the quadratic part is at
// most |u|^T |A| |u| <= lambda_G |u|^2 <= r^2 (lambda_G the Gershgorin bound
// max_r sum_c |a_rc|, r^2 = lambda_G |u|max^2), the linear part
// 2 sum_d |(Ae)_d u_d| <= 2 |u| |Ae| <= 2 r sqrt(e^T A e), the constant
// e^T A e + w_max - w >= 0, and sqrt(e^T A e) <= sqrt(C) + r, so
// S <= C + 4 r sqrt(C) + 4 r^2, and T = 2B + 4 r sqrt(B) + 5 r^2 >= 1.13 S
// for every C <= B.  Hence |C_fp32 - C| <= rho T with rho = 2^-18 (4.5
// times gamma_9 / 1.13), for any symmetric positive definite A_i.
// A pixel is settled when C_(2) - C_(1) > 2 rho T(B1) + 2^-18 max|C| (the
// key bits dropped by the short scan) + the slack of the double costs
// (dslack_abs, kslack), B1 an upper bound of the true C_(1): any seed j
// with C_j <= B1 then has C_j >= C_(2) - rho T > C_(1) + rho T, one with
// C_j > B1 exceeds the winner's cost outright.  Every other pixel goes to
// the double re-check.
constexpr int kPv = 8;  // pixels per lane of the vector kernel (4 on small grids)


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


// The box spanned by the pixel centres of the block of pixels starting at
// k0 with extents ext (clipped to the grid).
template <int D>
__device__ inline void cull_box(const Geo &g, const int *k0, const int *ext, double *blo, double *bhi) {
    for (int d = 0; d < D; ++d) {
        const int a = k0[d];
        const int b = min(a + ext[d], g.grid[d]) - 1;
        blo[d] = centre(g, d, a);
        bhi[d] = centre(g, d, max(b, a));
    }
}

template <class T> __device__ inline T tmin(T a, T b) { return a < b ? a : b; }
template <class T> __device__ inline T tmax(T a, T b) { return a > b ? a : b; }

// Range of the 2D quadratic form q(d) = a00 d0^2 + a01x2 d0 d1 + a11 d1^2
// (positive definite) over the box [p0, P0] x [p1, P1] of offsets d: the
// maximum is at a corner (q is convex); the minimum is 0 when the box holds
// d = 0, else it lies on an edge, where q is a 1D convex quadratic with its
// minimum at the stationary point clamped to the edge.
template <class T>
__device__ inline void quad_box_range2(T a00, T a01x2, T a11, T p0, T P0, T p1, T P1, T *qmin, T *qmax) {
    auto q = [&](T d0, T d1) { return a00 * d0 * d0 + a01x2 * d0 * d1 + a11 * d1 * d1; };
    auto clampv = [](T v, T lo, T hi) { return tmin(tmax(v, lo), hi); };
    *qmax = tmax(tmax(q(p0, p1), q(P0, p1)), tmax(q(p0, P1), q(P0, P1)));
    if (p0 <= T(0) && P0 >= T(0) && p1 <= T(0) && P1 >= T(0)) {
        *qmin = T(0);
        return;
    }
    T m = q(clampv(-a01x2 * p1 / (T(2) * a00), p0, P0), p1);
    m = tmin(m, q(clampv(-a01x2 * P1 / (T(2) * a00), p0, P0), P1));
    m = tmin(m, q(p0, clampv(-a01x2 * p0 / (T(2) * a11), p1, P1)));
    m = tmin(m, q(P0, clampv(-a01x2 * P0 / (T(2) * a11), p1, P1)));
    *qmin = m;
}

// Lower and upper bounds of seed i's cost C_i(y) - (w_i - wmax) over the box:
// in 2D with EXACT the exact range of the quadratic form (quad_box_range2),
// else the eigenvalue bounds lambda_min dist^2 and lambda_max maxdist^2.  The slack
// covers the rounding of either form: the absolute values of the form's
// terms sum to at most D lambda_max maxdist^2 (|2 a_rc d_r d_c| <=
// a_rr d_r^2 + a_cc d_c^2 for positive definite A).
template <int D, bool EXACT = true>
__device__ inline void cull_bounds(const Seeds &sd, const double *eig, double wmax, const double *blo,
                                   const double *bhi, int i, double *lb, double *ub) {
    double dist2 = 0.0, far2 = 0.0;
    for (int d = 0; d < D; ++d) {
        const double xd = sd.x[(size_t)i * D + d];
        const double dd = fmax(0.0, fmax(blo[d] - xd, xd - bhi[d]));
        const double fd = fmax(xd - blo[d], bhi[d] - xd);
        dist2 += dd * dd;
        far2 += fd * fd;
    }
    const double wp = sd.w[i] - wmax;
    double l = eig[2 * (size_t)i] * dist2, h = eig[2 * (size_t)i + 1] * far2;
    const double slack = 1e-9 * (fabs(l) + (double)D * fabs(h) + fabs(wp));
    if constexpr (D == 2 && EXACT) {
        const double *a = sd.A + (size_t)i * 4;
        const double x0 = sd.x[(size_t)i * 2], x1 = sd.x[(size_t)i * 2 + 1];
        quad_box_range2<double>(a[0], 2.0 * a[1], a[3], blo[0] - x0, bhi[0] - x0, blo[1] - x1, bhi[1] - x1,
                                &l, &h);
    }
    *lb = l - wp - slack;
    *ub = h - wp + slack;
}

// Block-wide: the seeds of src[0..nsrc) (of 0..nsrc-1 when src is null)
// whose lower bound does not exceed the smallest upper bound U, written to
// dst (at most cap of them, in any order); returns their number (which may
// exceed cap) and U in *Uout: every seed left out costs more than U
// everywhere in the box.  All threads of the block call it.
template <int D, bool EXACT = true>
__device__ inline int build_candidates(const Seeds &sd, const double *eig, double wmax,
                                       const double *blo, const double *bhi, const int *src,
                                       int nsrc, int *dst, int cap, int &s_cnt, double *s_red,
                                       double *Uout = nullptr) {
    const int lane = __lane_id();
    // a short source list keeps each thread's bounds in registers between
    // the two passes (one read of the seed data); a long one is read twice
    constexpr int kReg = 8;
    const bool in_regs = src && nsrc <= kReg * kThreads;
    double lbr[kReg];
    int ir[kReg];
    double umin = INFINITY;
    if (in_regs) {
#pragma unroll
        for (int r = 0; r < kReg; ++r) {
            const int q = threadIdx.x + r * kThreads;
            lbr[r] = INFINITY;
            ir[r] = 0;
            if (q < nsrc) {
                double ub;
                ir[r] = src[q];
                cull_bounds<D, EXACT>(sd, eig, wmax, blo, bhi, ir[r], &lbr[r], &ub);
                umin = fmin(umin, ub);
            }
        }
    } else {
        for (int q = threadIdx.x; q < nsrc; q += kThreads) {
            double lb, ub;
            cull_bounds<D, EXACT>(sd, eig, wmax, blo, bhi, src ? src[q] : q, &lb, &ub);
            umin = fmin(umin, ub);
        }
    }
    umin = wave_min(umin);
    __syncthreads();  // s_cnt and s_red may still be read by an earlier use
    if (threadIdx.x == 0) s_cnt = 0;
    if (lane == 0) s_red[threadIdx.x >> 6] = umin;
    __syncthreads();
    const double U = fmin(fmin(s_red[0], s_red[1]), fmin(s_red[2], s_red[3]));
    if (Uout) *Uout = U;
    auto emit = [&](bool cand, int i) {
        const unsigned long long m = __ballot(cand);
        int base = 0;
        if (lane == 0 && m) base = atomicAdd(&s_cnt, (int)__popcll(m));
        base = __builtin_amdgcn_readlane(base, 0);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (cand && base + below < cap) dst[base + below] = i;
    };
    if (in_regs) {
#pragma unroll
        for (int r = 0; r < kReg; ++r)
            if (r * kThreads < nsrc) emit(lbr[r] <= U, ir[r]);
    } else {
        for (int q0 = 0; q0 < nsrc; q0 += kThreads) {
            const int q = q0 + threadIdx.x;
            bool cand = false;
            int i = 0;
            if (q < nsrc) {
                i = src ? src[q] : q;
                double lb, ub;
                cull_bounds<D, EXACT>(sd, eig, wmax, blo, bhi, i, &lb, &ub);
                cand = lb <= U;
            }
            emit(cand, i);
        }
    }
    __syncthreads();
    return s_cnt;
}

// The candidate list of super-tile st (a box of sf[0] x sf[1] x sf[2]
// vector-kernel tiles of out.tp pixels per lane): the seeds that can attain
// the minimum somewhere in it, at most cap of them into list, their number
// into *count.  A seed that cannot win anywhere in the super-tile cannot win
// in any of its tiles, and a tile's smallest upper bound over the
// super-tile's list is at least its smallest over all seeds, so the tile
// lists built from these lists still hold every seed that can be the exact
// argmin (ties included).  All threads of the block call it.
template <int D>
__device__ inline void super_tile_list(const Geo &g, const Seeds &sd, double wmax, const double *eig,
                                       const PassOut &out, int st, int *list, int *count, int cap,
                                       int &s_cnt, double *s_red) {
    int c[3];
    c[2] = st % out.nst[2];
    c[1] = (st / out.nst[2]) % out.nst[1];
    c[0] = st / (out.nst[2] * out.nst[1]);
    const int ext[3] = {tile_ext(D, out.tp, 0) * out.sf[0], tile_ext(D, out.tp, 1) * out.sf[1],
                        tile_ext(D, out.tp, 2) * out.sf[2]};
    int k0[3];
    for (int d = 0; d < 3; ++d) k0[d] = c[d] * ext[d];
    double blo[3], bhi[3];
    cull_box<D>(g, k0, ext, blo, bhi);
    // the eigenvalue bounds here: a super-tile filters every seed, and its
    // list is only the source of the tiles' exact filters
    const int n = build_candidates<D, false>(sd, eig, wmax, blo, bhi, nullptr, g.n, list, cap, s_cnt, s_red);
    if (threadIdx.x == 0) *count = n;
}

// Two scans of the staged seeds, with the same costs and certificate:
//  * short scans (fewer than kGroupScan seeds) keep the index of the best
//    seed in the low 4 bits of its cost (integer min / med3 on the keys:
//    3 operations per pixel and seed besides the 2 fused multiply-adds);
//  * long scans take the minimum of each group of 16 seeds with 3-input
//    minima (about half an operation per pixel and seed), keep the top two
//    group minima and the group of the best, and at the end of each staged
//    chunk re-evaluate the 16 costs of the winning group -- bit-identical
//    values, same operations on the same operands -- to find the winning
//    seed and the second-smallest cost inside that group.  The top two of
//    all costs are then (best, min(second group minimum, second inside the
//    winning group)).
//
// With candidate lists, each wave then narrows the tile's list to the box of
// its own P x L1 (x L2) pixels (same bounds, the tile's candidates as the
// seed set) and scans only those; a wave whose list would not fit scans the
// tile's list.
constexpr int kGroupScan = 96;   // scans at least this long use group minima
constexpr int kWaveCap = 256;    // per-wave candidate positions

// Boundary-aware refinement, the owner test: does one candidate beat every
// other candidate at every point of the box [blo, bhi] of pixel centres?
// The owner is the candidate of least cost at the box centre c (lowest seed
// on ties); for any other candidate j the difference D = C_j - C_i is a
// quadratic, D(c + d) = D(c) + g.d + d^T M d with g = 2 A_j (c - x_j) -
// 2 A_i (c - x_i) and M = A_j - A_i (indefinite in general), so over
// |d_k| <= h_k
//   D >= D(c) - sum_k |g_k| h_k + min(0, lambda_min(M)) |h|^2,
// lambda_min from the closed-form eigenvalue range in 2D (widened by 1e-6 of
// its span), bounded below by minus the Gershgorin bound of M in 3D.  The
// owner is returned when every such bound exceeds a relative 1e-9 of the
// terms (far above the double rounding), so the owner is the strict argmin
// at every pixel of the box; else -1.  Lists longer than kOwnerMax are not
// tried (such tiles meet several cells).  All threads of the block call it.
constexpr int kOwnerMax = 8;  // longer lists: the tile meets several cells

template <int D>
__device__ inline int box_owner(const Seeds &sd, double wmax, const double *blo, const double *bhi,
                                const int *list, int ncand, double *s_red, int *s_redi) {
    if (ncand < 1 || ncand > kOwnerMax) return -1;
    if (ncand == 1) return list[0];
    double c[3], h[3];
    for (int d = 0; d < D; ++d) {
        c[d] = 0.5 * (blo[d] + bhi[d]);
        h[d] = 0.5 * (bhi[d] - blo[d]);
    }
    const int q = threadIdx.x;
    const int i = q < ncand ? list[q] : 0;
    // this candidate's cost and gradient at the centre (gauge w - w_max)
    double cc = INFINITY, gi[3] = {0.0, 0.0, 0.0};
    if (q < ncand) {
        const double *a = sd.A + (size_t)i * D * D;
        double dd[3];
        for (int d = 0; d < D; ++d) dd[d] = c[d] - sd.x[(size_t)i * D + d];
        double qf = 0.0;
        for (int r = 0; r < D; ++r) {
            double ad = 0.0;
            for (int k = 0; k < D; ++k) ad += a[(r <= k) ? r * D + k : k * D + r] * dd[k];
            gi[r] = 2.0 * ad;
            qf += dd[r] * ad;
        }
        cc = qf - (sd.w[i] - wmax);
    }
    // owner: least cost at the centre, lowest seed on ties
    double v = cc;
    int vi = q < ncand ? i : 0x7fffffff;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(v, o);
        const int oi = __shfl_xor(vi, o);
        if (ov < v || (ov == v && oi < vi)) {
            v = ov;
            vi = oi;
        }
    }
    __syncthreads();  // earlier readers of the slots are done
    if (__lane_id() == 0) {
        s_red[threadIdx.x >> 6] = v;
        s_redi[threadIdx.x >> 6] = vi;
    }
    __syncthreads();
    double ov = s_red[0];
    int oi = s_redi[0];
    for (int w = 1; w < kWaves; ++w)
        if (s_red[w] < ov || (s_red[w] == ov && s_redi[w] < oi)) {
            ov = s_red[w];
            oi = s_redi[w];
        }
    // the owner's gradient and matrix, and the bound for this candidate
    bool ok = true;
    if (q < ncand && i != oi) {
        const double *ao = sd.A + (size_t)oi * D * D;
        const double *a = sd.A + (size_t)i * D * D;
        double go[3], dd[3];
        for (int d = 0; d < D; ++d) dd[d] = c[d] - sd.x[(size_t)oi * D + d];
        for (int r = 0; r < D; ++r) {
            double ad = 0.0;
            for (int k = 0; k < D; ++k) ad += ao[(r <= k) ? r * D + k : k * D + r] * dd[k];
            go[r] = 2.0 * ad;
        }
        double m[3][3];
        for (int r = 0; r < D; ++r)
            for (int k = 0; k < D; ++k) {
                const int t = (r <= k) ? r * D + k : k * D + r;
                m[r][k] = a[t] - ao[t];
            }
        double lmin, lmax;
        if (D == 2) {
            eig_range<D>(m, &lmin, &lmax);
        } else {
            // Gershgorin: lambda_min(M) >= -max_r sum_c |m_rc|
            lmin = 0.0;
            for (int r = 0; r < D; ++r) {
                double rs = 0.0;
                for (int k = 0; k < D; ++k) rs += fabs(m[r][k]);
                lmin = fmin(lmin, -rs);
            }
        }
        double gh = 0.0, h2 = 0.0;
        for (int d = 0; d < D; ++d) {
            gh += fabs(gi[d] - go[d]) * h[d];
            h2 += h[d] * h[d];
        }
        const double quad = fmin(0.0, lmin) * h2;
        const double lb = (cc - ov) - gh + quad;
        const double slack = 1e-9 * (fabs(cc) + fabs(ov) + gh + fabs(quad) + fabs(sd.w[i] - wmax) +
                                     fabs(sd.w[oi] - wmax));
        ok = lb > slack;
    }
    return __syncthreads_and(ok) ? oi : -1;
}

// Boundary-aware refinement: a tile whose owner is L (box_owner: a single
// candidate, or one that beats every other candidate everywhere in the
// tile) lies inside L's cell, so its pixels are labelled L and its moments
// are added in closed form (box_moments_add) -- the pixel-level scan, the
// certificate and the re-check are skipped; the labels and moments are
// those of the full evaluation.  All threads of the block call it (with the
// same L).
template <int D, int P>
__device__ inline void credit_tile(const Geo &g, const Tile<D> &t, int b0, int b1, int b2, int L,
                                   const PassOut &out) {
    constexpr int E0 = tile_ext(D, P, 0), E1 = tile_ext(D, P, 1), E2 = tile_ext(D, P, 2);
    if (out.labels && lane_in_grid<D>(g, t)) {
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (t.k0w + p < g.grid[0]) out.labels[pixel_index<D>(g, t.k0w + p, t)] = L;
    }
    if (threadIdx.x == 0) {
        const int base[3] = {b0 * E0, b1 * E1, b2 * E2};
        const int ext[3] = {E0, E1, E2};
        int a[3], b[3];
        for (int d = 0; d < D; ++d) {
            a[d] = base[d];
            b[d] = min(base[d] + ext[d], g.grid[d]) - 1;
        }
        if (out.mom) box_moments_add<D>(out.mom, L, a, b);
        if (out.tile_lists) {
            const int tid = ((b0 * out.ntile[1]) + b1) * out.ntile[2] + b2;
            out.tile_lists[(size_t)tid * out.list_cap] = L;
            out.tile_count[tid] = 1;
        }
        if (out.credited) atomicAdd(out.credited, 1u);
    }
}

// Staging of the vector tile: float4 rows per seed, seeds per chunk (the
// 2D scan over every seed stages 1024 so that N = 1000 is one chunk).
template <int D, bool CULL>
struct VecCfg {
    static constexpr int kRows = D == 2 ? 2 : 3;
    static constexpr int kChunk = CULL ? 256 : (D == 2 ? 1024 : 512);
};

// LDS of the vector tile.
template <int D, bool CULL>
struct VecSmem {
    // seed coefficients of one chunk, + a dummy slot (index kChunk); with
    // candidate lists the free lanes of the last row hold the seed's
    // eigenvalue range (FP32, rounded outwards)
    float4 sC[VecCfg<D, CULL>::kRows][VecCfg<D, CULL>::kChunk + 1];
    float4 sB[CULL ? VecCfg<D, CULL>::kChunk : 1];  // (x - anchor, w - wmax) in FP32
    int list[CULL ? kCullCap : 1];        // candidate seeds of the tile
    int wl[kWaves][CULL ? kWaveCap : 1];  // staged positions of each wave's candidates
    double red[kWaves];
    int redi[kWaves];
    int cnt;
};

template <int D, bool CULL, int P = kPv>
__device__ inline void vec_tile(const Geo &g, const Seeds &sd, double wmax, Cert ct,
                                const double *eig, int b0, int b1, int b2, VecSmem<D, CULL> &sm,
                                const PassOut &out, unsigned *qcount) {
    constexpr int E0 = tile_ext(D, P, 0), E1 = tile_ext(D, P, 1), E2 = tile_ext(D, P, 2);
    constexpr int kVecChunk = VecCfg<D, CULL>::kChunk;
    constexpr int kDummy = kVecChunk;  // staged slot whose cost is never the minimum
    auto &sC = sm.sC;
    int *s_list = sm.list;
    double *s_red = sm.red;
    int &s_cnt = sm.cnt;
    const Tile<D> t = tile_at<D, P>(b0, b1, b2);
    const bool lane_ok = lane_in_grid<D>(g, t);
    int nscan = g.n;
    bool full = true;
    int ncand_kept = 0;
    double Utile = INFINITY;  // no seed left out of the tile's list costs less
    float Uwave = INFINITY;   // nor out of this wave's list
    if (CULL) {
        // ---- the candidate list, from the super-tile's list when it has one
        double blo[3], bhi[3];
        const int ext[3] = {E0, E1, E2};
        const int k0[3] = {t.anc[0] - E0 / 2, t.anc[1] - E1 / 2, D == 3 ? t.anc[2] - E2 / 2 : 0};
        cull_box<D>(g, k0, ext, blo, bhi);
        const int *src = nullptr;
        int nsrc = g.n;
        if (out.super_list) {
            const int st = ((b0 / out.sf[0]) * out.nst[1] + b1 / out.sf[1]) * out.nst[2] + b2 / out.sf[2];
            const int c = out.super_count[st];
            if (c <= out.super_cap) {
                src = out.super_list + (size_t)st * out.super_cap;
                nsrc = c;
            }
        }
        const int ncand = build_candidates<D>(sd, eig, wmax, blo, bhi, src, nsrc, s_list, kCullCap,
                                              s_cnt, s_red, &Utile);
        full = ncand > kCullCap;
        nscan = full ? g.n : ncand;
        ncand_kept = ncand;
        if (full || ncand >= g.n) Utile = INFINITY;  // no seed was left out
        if (out.adaptive && !full && !g.mass && !out.rel_gap) {
            const int own = box_owner<D>(sd, wmax, blo, bhi, s_list, ncand, s_red, sm.redi);
            if (own >= 0) {
                credit_tile<D, P>(g, t, b0, b1, b2, own, out);
                return;
            }
        }
    }

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
    // cost of staged seed q at the pixels of this lane (2 fused
    // multiply-adds per pixel after 3 (2D) or 7 (3D) per seed)
    auto lane_coef = [&](int q, float &a00, float &beta, float &alpha) {
        const float4 c0 = sC[0][q];
        const float4 c1 = sC[1][q];
        if constexpr (D == 2) {
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
    };
    // padding entries (and the dummy slot) cost 1.7e38 everywhere
    auto pad = [&](int q) {
        sC[0][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (D == 2) {
            sC[1][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
        } else {
            sC[1][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            sC[2][q] = make_float4(0.0f, 1.7e38f, 0.0f, 0.0f);
        }
    };
    auto stage = [&](int base, int cnt, int padded) {
        if (threadIdx.x == 0) pad(kDummy);
        for (int q = threadIdx.x; q < padded; q += kThreads) {
            if (q >= cnt) {
                pad(q);
                continue;
            }
            const int i = full ? base + q : s_list[base + q];
            double qd[6], ld[3], cd, ed[3], wpd;
            seed_terms<D>(sd, i, anc, wmax, qd, ld, &cd, ed, &wpd);
            float lmn = 0.0f, lmx = 0.0f;
            if constexpr (CULL) {
                // rounded outwards: the FP32 bounds of the wave lists stay bounds
                lmn = (float)eig[2 * (size_t)i] * (1.0f - 0x1p-20f);
                lmx = (float)eig[2 * (size_t)i + 1] * (1.0f + 0x1p-20f);
                sm.sB[q] = make_float4((float)ed[0], (float)ed[1], D == 3 ? (float)ed[2] : 0.0f, (float)wpd);
            }
            if constexpr (D == 2) {
                sC[0][q] = make_float4((float)qd[0], (float)qd[1], (float)qd[2], (float)ld[0]);
                sC[1][q] = make_float4((float)ld[1], (float)cd, lmn, lmx);
            } else {
                sC[0][q] = make_float4((float)qd[0], (float)qd[1], (float)qd[2], (float)ld[0]);
                sC[1][q] = make_float4((float)qd[3], (float)qd[4], (float)qd[5], (float)ld[1]);
                sC[2][q] = make_float4((float)ld[2], (float)cd, lmn, lmx);
            }
        }
    };
    float fb[P], fs[P];  // the two smallest costs of each pixel
    int pos[P];          // scan position of the best seed
    bool lost[P];        // the winner was not found again (never expected)
#pragma unroll
    for (int p = 0; p < P; ++p) {
        fb[p] = INFINITY;
        fs[p] = INFINITY;
        pos[p] = 0;
        lost[p] = false;
    }
    // Short scan of the staged positions idx(j), j < c16 (a multiple of 16).
    // Only the first c4 (a multiple of 4) positions are scanned: the lists
    // are padded to 16, but a short list wastes at most 3 slots.
    bool keyed = false;  // the short scan ran: its costs lost their low 4 bits
    auto key_scan = [&](int c4, auto idx) {
        keyed = true;
        int best[P], second[P], blk[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            best[p] = 0x7fffffff;
            second[p] = 0x7fffffff;
            blk[p] = 0;
        }
        for (int q0 = 0; q0 < c4; q0 += 16) {
            int old[P];
#pragma unroll
            for (int p = 0; p < P; ++p) old[p] = best[p];
            for (int r4 = 0; r4 < 16 && q0 + r4 < c4; r4 += 4) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int r = r4 + rr;
                    float a00, beta, alpha;
                    lane_coef(idx(q0 + r), a00, beta, alpha);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                        const int key = (__float_as_int(c) & ~15) | r;
                        second[p] = med3i(best[p], key, second[p]);
                        best[p] = min(best[p], key);
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) blk[p] = (best[p] != old[p]) ? q0 : blk[p];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            pos[p] = blk[p] + (best[p] & 15);
            fb[p] = __int_as_float(best[p]);
            fs[p] = __int_as_float(second[p]);
        }
    };
    // Long scan of one staged chunk (positions idx(j), j < c16), merged into
    // the running top two; winners found here get scan position base + j.
    auto group_scan = [&](int c16, auto idx, int base) {
        int blk[P];
#pragma unroll
        for (int p = 0; p < P; ++p) blk[p] = -1;
        for (int q0 = 0; q0 < c16; q0 += 16) {
            float m[P];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float a00, beta, alpha;
                lane_coef(idx(q0 + r), a00, beta, alpha);
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                    m[p] = r == 0 ? c : fminf(m[p], c);
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                // top two of the group minima and the group of the best (a
                // select on the comparison, which needs no canonicalised
                // operand as a minimum would)
                fs[p] = __builtin_amdgcn_fmed3f(fb[p], m[p], fs[p]);
                const bool better = m[p] < fb[p];
                blk[p] = better ? q0 : blk[p];
                fb[p] = better ? m[p] : fb[p];
            }
        }
        // the winners found in this chunk: which seed of the group, and the
        // second-smallest cost inside the group
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (blk[p] < 0) continue;
            float s2 = INFINITY;
            int ix = -1;
            for (int r = 0; r < 16; ++r) {
                float a00, beta, alpha;
                lane_coef(idx(blk[p] + r), a00, beta, alpha);
                const float c = fmaf(fmaf(a00, u0[p], beta), u0[p], alpha);
                const bool hit = ix < 0 && c == fb[p];
                ix = hit ? r : ix;
                s2 = hit ? s2 : fminf(s2, c);
            }
            lost[p] = ix < 0;
            pos[p] = base + blk[p] + max(ix, 0);
            fs[p] = fminf(fs[p], s2);
        }
    };
    auto ident = [](int j) { return j; };
    // per-wave lists: candidates of the tile, staged in one chunk
    const bool per_wave = CULL && !full && nscan <= kVecChunk;
    int *wl = sm.wl[threadIdx.x >> 6];
    int cntw = -1;  // this wave's list length; -1: scan the tile's list
    if (per_wave) {
        const int padded = (nscan + 15) & ~15;
        __syncthreads();
        stage(0, nscan, padded);
        __syncthreads();
        // the wave's box in the tile-local coordinates of the scan, and FP32
        // bounds from the staged data, widened by a relative 1e-4 (far above
        // their rounding), so the wave list keeps every seed that can win
        float wlo[3] = {0.0f, 0.0f, 0.0f}, whi[3] = {0.0f, 0.0f, 0.0f};
        {
            const int k0w[3] = {t.org[0], t.org[1], t.org[2]};
            const int extw[3] = {wave_ext(D, P, 0), wave_ext(D, P, 1), wave_ext(D, P, 2)};
            for (int d = 0; d < D; ++d) {
                const int a = k0w[d], b = max(a, min(a + extw[d], g.grid[d]) - 1);
                wlo[d] = ((float)(a - t.anc[d]) + 0.5f) * s[d];
                whi[d] = ((float)(b - t.anc[d]) + 0.5f) * s[d];
            }
        }
        auto wbounds = [&](int q, float &lb, float &ub) {
            const float4 b = sm.sB[q];
            const float4 ce = sC[VecCfg<D, CULL>::kRows - 1][q];  // .z, .w: eigenvalue range
            const float e[3] = {b.x, b.y, b.z};
            float dist2 = 0.0f, far2 = 0.0f;
            for (int d = 0; d < D; ++d) {
                const float dd = fmaxf(0.0f, fmaxf(wlo[d] - e[d], e[d] - whi[d]));
                const float fd = fmaxf(e[d] - wlo[d], whi[d] - e[d]);
                dist2 = fmaf(dd, dd, dist2);
                far2 = fmaf(fd, fd, far2);
            }
            float l = ce.z * dist2, h = ce.w * far2;
            const float slack = 1e-4f * (fabsf(l) + (float)D * fabsf(h) + fabsf(b.w)) + 1e-30f;
            if constexpr (D == 2) {
                // the exact range of the quadratic form, as cull_bounds
                const float4 c0 = sC[0][q];  // a00, 2 a01, a11
                quad_box_range2<float>(c0.x, c0.y, c0.z, wlo[0] - e[0], whi[0] - e[0], wlo[1] - e[1],
                                       whi[1] - e[1], &l, &h);
            } else {
                // the exact maximum: the form is convex, so at a corner
                const float4 c0 = sC[0][q];  // a00, 2 a01, 2 a02
                const float4 c1 = sC[1][q];  // a11, 2 a12, a22
                float hm = 0.0f;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const float d0 = ((v & 1) ? whi[0] : wlo[0]) - e[0];
                    const float d1 = ((v & 2) ? whi[1] : wlo[1]) - e[1];
                    const float d2 = ((v & 4) ? whi[2] : wlo[2]) - e[2];
                    const float qv = fmaf(fmaf(c0.x, d0, fmaf(c0.y, d1, c0.z * d2)), d0,
                                          fmaf(fmaf(c1.x, d1, c1.y * d2), d1, c1.z * d2 * d2));
                    hm = fmaxf(hm, qv);
                }
                h = hm;
            }
            lb = l - b.w - slack;
            ub = h - b.w + slack;
        };
        float um = INFINITY;
        for (int q = t.lane; q < nscan; q += 64) {
            float lb, ub;
            wbounds(q, lb, ub);
            um = fminf(um, ub);
        }
        um = wave_min(um);
        int c = 0;
        for (int q0 = 0; q0 < nscan; q0 += 64) {
            const int q = q0 + t.lane;
            bool cand = false;
            if (q < nscan) {
                float lb, ub;
                wbounds(q, lb, ub);
                cand = lb <= um;
            }
            const unsigned long long m = __ballot(cand);
            const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (cand && c + below < kWaveCap) wl[c + below] = q;
            c += (int)__popcll(m);
        }
        const int c16 = (c + 15) & ~15;
        if (c > 0 && c16 <= kWaveCap) {
            for (int j = c + t.lane; j < c16; j += 64) wl[j] = kDummy;
            cntw = c;
            if (c < nscan) Uwave = um;  // some of the tile's candidates were left out
        }
        // the list is read back by other lanes of the wave only
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (cntw >= 0) {
            const int c16w = (cntw + 15) & ~15;
            auto widx = [&](int j) { return wl[j]; };
            if (cntw >= kGroupScan) group_scan(c16w, widx, 0);
            else key_scan((cntw + 3) & ~3, widx);
        } else if (nscan >= kGroupScan) {
            group_scan(padded, ident, 0);
        } else {
            key_scan((nscan + 3) & ~3, ident);
        }
    } else if (nscan >= kGroupScan) {
        for (int base = 0; base < nscan; base += kVecChunk) {
            const int cnt = min(kVecChunk, nscan - base);
            const int padded = (cnt + 15) & ~15;
            __syncthreads();
            stage(base, cnt, padded);
            __syncthreads();
            group_scan(padded, ident, base);
        }
    } else {
        const int padded = (nscan + 15) & ~15;
        __syncthreads();
        stage(0, nscan, padded);
        __syncthreads();
        key_scan((nscan + 3) & ~3, ident);
    }
    const float sab = dslack_abs(g, wmax, ct), skb = kslack(ct);
    const float kbits = keyed ? 0x1p-18f : 0.0f;
    bool flag[P];
    int lab[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (cntw >= 0) {
            lab[p] = s_list[wl[min(pos[p], cntw - 1)]];
        } else {
            const int ps = min(pos[p], nscan - 1);
            lab[p] = full ? ps : s_list[ps];
        }
        const float r2 = pixel_r2(ct, u0[p], u1, u2);
        const float bb = fmaxf(fb[p], 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float thr = 2.0f * e32_bound(B1, sqrtf(r2), r2) + kbits * fmaxf(fabsf(fb[p]), fabsf(fs[p])) +
                          sab + skb * (B1 + r2);
        flag[p] = lost[p] || !((fs[p] - fb[p]) > thr);
        if (out.rel_gap && act[p] && !flag[p]) {
            // the winner costs at most c1u; a scanned seed at least fs minus
            // its bound, one left out of the lists more than the lists' U
            const float c1u = (fb[p] + 0x1p-19f * fabsf(fb[p]) + e32_bound(B1, sqrtf(r2), r2) + sab +
                               skb * (B1 + r2)) * (1.0f + 0x1p-20f);
            const float f2 = pad_inf(fs[p]);
            const float bs = fmaxf(f2, 0.0f);
            const float B2 = bs + 0x1p-10f * (bs + r2);
            float c2l = f2 == INFINITY
                            ? f2
                            : f2 - 0x1p-19f * fabsf(f2) - e32_bound(B2, sqrtf(r2), r2) - sab - skb * (B2 + r2);
            const float uc = fminf((float)Utile, Uwave);
            c2l = fminf(c2l, (uc == INFINITY ? uc : uc - 0x1p-20f * fabsf(uc))) * (1.0f - 0x1p-20f);
            out.rel_gap[pixel_index<D>(g, t.k0w + p, t)] = fs[p] > 0.0f ? gap_lower(c1u, c2l) : 0.0f;
        }
    }
    PassOut o = out;
    if (CULL && out.tile_lists) {
        // keep the candidates for the re-check of this tile's queued pixels
        const int tid = ((b0 * out.ntile[1]) + b1) * out.ntile[2] + b2;
        o.tile_id = tid;
        const bool keep = !full && ncand_kept <= out.list_cap;
        if (keep)
            for (int q = threadIdx.x; q < ncand_kept; q += kThreads)
                out.tile_lists[(size_t)tid * out.list_cap + q] = s_list[q];
        if (threadIdx.x == 0) {
            out.tile_count[tid] = keep ? ncand_kept : out.list_cap + 1;
            if (out.tile_U) out.tile_U[tid] = keep ? Utile : INFINITY;
        }
    }
    tile_epilogue<D, P>(g, t, act, lab, flag, o, qcount);
}


// ------------------------------------------------------------ bf16 helpers

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

// round to nearest even (finite inputs)
__device__ inline unsigned short bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// ------------------------------------------- hybrid matrix-core / vector tile

// Single precision over every seed, the work split between the two units.
// The cost of seed i at a pixel, in coordinates u about the tile anchor, is
// a quadratic in u0 whose coefficients depend on the pixel's other axes:
//   C = a00 u0^2 + beta u0 + alpha,
//   3D: beta  = 2a01 u1 + 2a02 u2 + l0,
//       alpha = a11 u1^2 + 2a12 u1 u2 + a22 u2^2 + l1 u1 + l2 u2 + c,
//   2D: beta  = 2a01 u1 + l0,  alpha = a11 u1^2 + l1 u1 + c
// (l = -2 A e, c = e^T A e - w', as seed_terms).  For 32 seeds x 32 positions
// (u1, u2) the matrix cores form beta and alpha, one
// v_mfma_f32_32x32x16_bf16 each: the coefficients split exactly into three
// bf16 parts against exact small-integer features (hyb_stage).  The vector
// ALU then evaluates the quadratic along axis 0 for rows placed
// symmetrically about the anchor, u0 = +-(j + 1/2) s0: a row pair shares
// q = a00 u0^2 + alpha and takes C = q +- beta u0, so 1.5 fused multiply-adds
// per pair and no per-seed coefficient work on the ALU.  The accumulator
// layout gives lane l the block rows 8 (r / 4) + 4 h + r % 4 (h = l / 32) at
// position l % 32: the two half-waves see the same pixels against the two
// halves of every block.  The seeds are scanned in the order of a
// space-filling curve (k_seed_order), and the running minimum is kept per
// kHybSB consecutive ones (a super-block, a compact region of the box),
// with the runner-up and that super-block's index.  At the
// end the two halves exchange their minima, so that only the pixel's true
// winning super-block is searched, once per distinct one in the wave: its
// products are formed again (the same operands, so the same bits) and the
// half holding the best cost finds the seed attaining it.
//
// Tiles (HybCfg): 3D 16 x 16 x 8 pixels, wave w covering the 8 row pairs
// and 4 x 8 positions (axis 1 from 4 w, axis 2); 2D 32 x 32 pixels, wave w
// covering row pairs 4 w .. 4 w + 3 and the tile's 32 positions.  After the
// half-waves are merged, lane l owns its pairs' rows below the anchor
// (h = 0) or above it (h = 1) at its position: NJ consecutive rows.
//
// Rounding bound (relative roundings of 2^-24 on each monomial's path to
// the computed cost, S the sum of the monomials' magnitudes, S <= C +
// 4 r sqrt(C) + 4 r^2 as for the vector tile): the coefficient's FP32
// rounding (1; the bf16 split, the integer features and their products are
// exact), the matrix-core sum (alpha: the start c - c_hi and its products,
// 16 in 3D and 10 in 2D, each addition possibly rounded), the two fused
// multiply-adds.  3D: at most 19 (beta's terms 11, a00 u0^2 5), so
// |C_fp32 - C| <= gamma_19 S < 1.19 2^-20 S, within hyb_bound (1.3125 2^-20
// S); 2D: at most 13, within e32_bound.
constexpr int kHybSB = 64;  // seeds per running-minimum group (super-block): one per lane

template <int D> struct HybCfg;
template <> struct HybCfg<3> {
    static constexpr int kRows = kHybRows3;  // tile rows along axis 0
    static constexpr int kPairs = 8;         // row pairs per lane
    static constexpr int kChunk = 512;       // seeds staged per chunk (a multiple of kHybSB)
};
template <> struct HybCfg<2> {
    static constexpr int kRows = kHybRows2;
    static constexpr int kPairs = 4;
    static constexpr int kChunk = 512;
};

// LDS of the hybrid tile: per staged seed its bf16 operand slots, group
// 2 m + h holding slots 8 h .. 8 h + 7 of product m (0: beta, 1: alpha), and
// its FP32 a00 and c - c_hi.  After the scan each wave re-stages one
// super-block at a time into its own 64 positions of the same arrays.
template <int D>
struct HybSmem {
    static constexpr int C = HybCfg<D>::kChunk;
    ushort8 a[4][C];
    float a00[C];
    float crest[C];
};

// An FP32 value as the exact sum of three bf16 parts (hi, mid, lo: 8
// significant bits each; each difference is exact in FP32).
__device__ inline void bf16_split3(float f, unsigned short *out) {
    const unsigned short hi = bf16_bits(f);
    const float r = f - bf16_value(hi);
    const unsigned short mid = bf16_bits(r);
    out[0] = hi;
    out[1] = mid;
    out[2] = bf16_bits(r - bf16_value(mid));
}

// The operand slots of one seed.  In tile-local half-pixel units
// o_d = 2 (k_d - anchor_d) + 1 (odd integers: 3D |o_1| <= 15, |o_2| <= 7;
// 2D |o_1| <= 31) the position's features are exact bf16 values (2D: o1^2,
// up to 961, as the sum of two, f2 = f2_hi + f2_lo) and the coefficients
// carry the half spacings h_d = s_d / 2:
//   3D beta  = (2a01 h1) o1 + (2a02 h2) o2 + l0,
//      alpha = (a11 h1^2) o1^2 + (2a12 h1 h2) o1 o2 + (a22 h2^2) o2^2
//              + (l1 h1) o1 + (l2 h2) o2 + c;
//   2D beta  = (2a01 h1) o1 + l0,  alpha = (a11 h1^2) o1^2 + (l1 h1) o1 + c.
// Each coefficient is rounded once to FP32 and split exactly into bf16 hi,
// mid and lo parts, one slot each (2D: a11's parts against f2_hi and again
// against f2_lo): 3D beta slots 0-8, alpha slots 0-14 and c_hi in 15; 2D
// beta slots 0-5, alpha slots 0-8 and c_hi in 9; the rest zero.  c - c_hi
// (exact in FP32) starts the alpha accumulator.  Padding seeds cost 1.7e38.
template <int D>
__device__ inline void hyb_stage(const Seeds &sd, int i, bool real, const double *anc, double wmax,
                                 double h1, double h2, ushort8 (&grp)[4], float &a00, float &crest) {
    constexpr int CHI = D == 3 ? 31 : 25;  // slot of c_hi (alpha's slots start at 16)
    unsigned short sl[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) sl[k] = 0;
    if (!real) {
        sl[CHI] = bf16_bits(1.7e38f);
        a00 = 0.0f;
        crest = 0.0f;
    } else {
        double qd[6], ld[3], cd, ed[3], wpd;
        seed_terms<D>(sd, i, anc, wmax, qd, ld, &cd, ed, &wpd);
        if constexpr (D == 3) {
            // qd = (a00, 2a01, 2a02, a11, 2a12, a22)
            const float cb[3] = {(float)(qd[1] * h1), (float)(qd[2] * h2), (float)ld[0]};
            const float ca[5] = {(float)(qd[3] * h1 * h1), (float)(qd[4] * h1 * h2), (float)(qd[5] * h2 * h2),
                                 (float)(ld[1] * h1), (float)(ld[2] * h2)};
#pragma unroll
            for (int k = 0; k < 3; ++k) bf16_split3(cb[k], sl + 3 * k);
#pragma unroll
            for (int k = 0; k < 5; ++k) bf16_split3(ca[k], sl + 16 + 3 * k);
        } else {
            // qd = (a00, 2a01, a11)
            bf16_split3((float)(qd[1] * h1), sl);
            bf16_split3((float)ld[0], sl + 3);
            bf16_split3((float)(qd[2] * h1 * h1), sl + 16);
            sl[19] = sl[16];
            sl[20] = sl[17];
            sl[21] = sl[18];
            bf16_split3((float)(ld[1] * h1), sl + 22);
        }
        const float cc = (float)cd;
        sl[CHI] = bf16_bits(cc);
        crest = cc - bf16_value(sl[CHI]);
        a00 = (float)qd[0];
    }
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
        ushort8 u;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) u[jj] = sl[8 * gq + jj];
        grp[gq] = u;
    }
}

// Rounding bound of the hybrid tile's costs: 2D that of the vector tile
// (e32_bound); 3D 1.3125 times it, for its longer matrix-core sum.
template <int D>
__device__ inline float hyb_bound(float B, float r, float r2) {
    return (D == 3 ? 0x1.5p-20f : 0x1p-20f) * (B + 4.0f * r * sqrtf(B) + 4.0f * r2);
}

// a wave-uniform float in a scalar register
__device__ inline float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

template <int D>
__device__ inline void hyb_tile(const Geo &g, const Seeds &sd, double wmax, Cert ct, int b0, int b1, int b2,
                                HybSmem<D> &sm, const PassOut &out, unsigned *qcount) {
    using Cfg = HybCfg<D>;
    constexpr int NJ = Cfg::kPairs;   // row pairs of a lane
    constexpr int NP = 2 * NJ;        // pixels a lane evaluates
    constexpr int CH = Cfg::kChunk;
    const int lane = __lane_id();
    const int half = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    Tile<D> t;
    t.lane = lane;
    int j0;  // first row pair of this wave
    if constexpr (D == 3) {
        t.org[0] = b0 * Cfg::kRows;
        t.org[1] = b1 * 16 + wave * 4;
        t.org[2] = b2 * 8;
        t.anc[1] = b1 * 16 + 8;
        t.anc[2] = b2 * 8 + 4;
        t.k[1] = t.org[1] + (col >> 3);
        t.k[2] = t.org[2] + (col & 7);
        j0 = 0;
    } else {
        t.org[0] = b0 * Cfg::kRows;
        t.org[1] = b1 * 32;
        t.org[2] = 0;
        t.anc[1] = b1 * 32 + 16;
        t.anc[2] = 0;
        t.k[1] = t.org[1] + col;
        t.k[2] = 0;
        j0 = wave * NJ;
    }
    t.anc[0] = b0 * Cfg::kRows + Cfg::kRows / 2;
    t.k0w = half ? t.anc[0] + j0 : t.anc[0] - j0 - NJ;  // the rows this lane owns at the end
    t.k[0] = t.k0w;
    float s[3];
    double anc[3];
    for (int d = 0; d < D; ++d) {
        s[d] = (float)g.s[d];
        anc[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
    }
    // rows: uj[j] = (j0 + j + 1/2) s0 above the anchor, -uj[j] below
    float uj[NJ], usq[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float u = ((float)(j0 + j) + 0.5f) * s[0];
        uj[j] = uniform_f(u);
        usq[j] = uniform_f(u * u);
    }
    const float u1 = ((float)(t.k[1] - t.anc[1]) + 0.5f) * s[1];
    const float u2 = D == 3 ? ((float)(t.k[2] - t.anc[2]) + 0.5f) * s[2] : 0.0f;
    // operand B: the bf16 feature slots of this lane's position (half h
    // supplies slots 8 h .. 8 h + 7), as hyb_stage lays out the coefficients
    bf16x8 fbB, fbA;
    {
        float fB[16], fA[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) fB[k] = fA[k] = 0.0f;
        const float o1 = (float)(2 * (t.k[1] - t.anc[1]) + 1);
        if constexpr (D == 3) {
            const float o2 = (float)(2 * (t.k[2] - t.anc[2]) + 1);
            const float fb3[3] = {o1, o2, 1.0f}, fa3[5] = {o1 * o1, o1 * o2, o2 * o2, o1, o2};
#pragma unroll
            for (int k = 0; k < 9; ++k) fB[k] = fb3[k / 3];
#pragma unroll
            for (int k = 0; k < 15; ++k) fA[k] = fa3[k / 3];
            fA[15] = 1.0f;
        } else {
            const float f2 = o1 * o1, f2h = bf16_value(bf16_bits(f2)), f2l = f2 - f2h;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                fB[k] = o1;
                fB[3 + k] = 1.0f;
                fA[k] = f2h;
                fA[3 + k] = f2l;
                fA[6 + k] = o1;
            }
            fA[9] = 1.0f;
        }
        ushort8 uB, uA;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            uB[jj] = bf16_bits(half ? fB[8 + jj] : fB[jj]);
            uA[jj] = bf16_bits(half ? fA[8 + jj] : fA[jj]);
        }
        fbB = __builtin_bit_cast(bf16x8, uB);
        fbA = __builtin_bit_cast(bf16x8, uA);
    }
    const double h1 = 0.5 * g.s[1], h2 = D == 3 ? 0.5 * g.s[2] : 0.0;
    // the seed at scan position q (the scan follows out.seed_order)
    auto seed_at = [&](int q) { return out.seed_order ? out.seed_order[q] : q; };
    // seed i (padding unless real) into LDS position pos
    auto stage_at = [&](int pos, int i, bool real) {
        ushort8 gq[4];
        float a0, cr;
        hyb_stage<D>(sd, i, real, anc, wmax, h1, h2, gq, a0, cr);
#pragma unroll
        for (int k = 0; k < 4; ++k) sm.a[k][pos] = gq[k];
        sm.a00[pos] = a0;
        sm.crest[pos] = cr;
    };
    // beta and alpha of the 16 seeds (rows of this half) of the block staged
    // at positions pos .. pos + 31, at the lane's position: one
    // v_mfma_f32_32x32x16_bf16 each, alpha's accumulator starting from the
    // seeds' c - c_hi
    auto products = [&](int pos, floatx16 &bet, floatx16 &alp) {
        const bf16x8 ab = __builtin_bit_cast(bf16x8, sm.a[half][pos + col]);
        const bf16x8 aa = __builtin_bit_cast(bf16x8, sm.a[2 + half][pos + col]);
        floatx16 ci;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const float4 v = *reinterpret_cast<const float4 *>(&sm.crest[pos + 8 * qq + 4 * half]);
            ci[4 * qq] = v.x; ci[4 * qq + 1] = v.y; ci[4 * qq + 2] = v.z; ci[4 * qq + 3] = v.w;
        }
        bet = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, fbB, floatx16{}, 0, 0, 0);
        alp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, fbA, ci, 0, 0, 0);
    };
    // pixel 2 j + sgn: row anchor + j0 + j (sgn 0) or anchor - 1 - j0 - j (sgn 1)
    float fb[NP], fs[NP];
    int blk[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        fb[p] = INFINITY;
        fs[p] = INFINITY;
        blk[p] = 0;
    }

    for (int base = 0; base < g.n; base += CH) {
        const int cnt = min(CH, g.n - base);
        const int padded = (cnt + kHybSB - 1) & ~(kHybSB - 1);
        __syncthreads();
        for (int q = threadIdx.x; q < padded; q += kThreads)
            stage_at(q, q < cnt ? seed_at(base + q) : 0, q < cnt);
        __syncthreads();
        for (int sb = 0; sb < padded; sb += kHybSB) {
            float m[NP];
#pragma unroll
            for (int hb = 0; hb < kHybSB / 32; ++hb) {
                const int cb = sb + 32 * hb;
                floatx16 bet, alp;
                products(cb, bet, alp);
                float a0[16];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const float4 v = *reinterpret_cast<const float4 *>(&sm.a00[cb + 8 * qq + 4 * half]);
                    a0[4 * qq] = v.x; a0[4 * qq + 1] = v.y; a0[4 * qq + 2] = v.z; a0[4 * qq + 3] = v.w;
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const float q = fmaf(a0[r], usq[j], alp[r]);
                        const float cp = fmaf(bet[r], uj[j], q);
                        const float cm = fmaf(-bet[r], uj[j], q);
                        const bool first = hb == 0 && r == 0;
                        m[2 * j] = first ? cp : fminf(m[2 * j], cp);
                        m[2 * j + 1] = first ? cm : fminf(m[2 * j + 1], cm);
                    }
                }
            }
            const int gsb = (base + sb) / kHybSB;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                fs[p] = __builtin_amdgcn_fmed3f(fb[p], m[p], fs[p]);
                const bool better = m[p] < fb[p];
                blk[p] = better ? gsb : blk[p];
                fb[p] = better ? m[p] : fb[p];
            }
        }
    }

    // merge the half-waves' minima: lanes l and l ^ 32 hold the same pixels
    // against the two halves of every block, so after one exchange both know
    // each pixel's best cost, the super-block it lies in and the runner-up
    // among the super-block minima; bit p of `win` marks the pixels whose best
    // lies in this lane's half (both halves on equal costs in one super-block;
    // on equal costs in two, the lower super-block, and the certificate flags
    // the pixel either way)
    unsigned win = 0u;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const float ob = __shfl_xor(fb[p], 32);
        const float os = __shfl_xor(fs[p], 32);
        const int oi = __shfl_xor(blk[p], 32);
        const bool other = ob < fb[p] || (ob == fb[p] && oi < blk[p]);
        win |= (other ? 0u : 1u) << p;
        fs[p] = fminf(fmaxf(fb[p], ob), fminf(fs[p], os));
        fb[p] = fminf(fb[p], ob);
        blk[p] = other ? oi : blk[p];
    }

    // the seed inside each winning super-block: the wave forms the products
    // of one winning super-block at a time again (its smallest unresolved
    // one first) and each lane looks, among the costs of its half, for the
    // best of the pixels it won: the first seed attaining it and the smallest
    // of the other costs; a resolved pixel's blk holds its seed from then on
    unsigned done = 0u;  // bit p: resolved
    unsigned lostm = 0u; // bit p: the best cost was not found again (never expected)
    __syncthreads();     // every wave is done with the staged chunk
    for (;;) {
        int mine = 0x7fffffff;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (!(done >> p & 1u)) mine = min(mine, blk[p]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mine = min(mine, __shfl_xor(mine, o));
        const int wb = __builtin_amdgcn_readfirstlane(mine);
        if (wb == 0x7fffffff) break;
        unsigned want = 0u;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (!(done >> p & 1u) && blk[p] == wb) want |= 1u << p;
        done |= want;
        want &= win;
        // the super-block's 64 seeds, one per lane, in the wave's own 64
        // positions of the staging area
        {
            const int i = wb * kHybSB + lane;
            stage_at(64 * wave + lane, i < g.n ? seed_at(i) : 0, i < g.n);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the lane's pixels in groups of 8 (4 row pairs), the products formed
        // again for each group, to bound the registers held; a group that no
        // lane of the wave wants is skipped
#pragma unroll
        for (int grp = 0; grp < NP / 8; ++grp) {
            if (!__ballot((want >> (8 * grp) & 0xffu) != 0u)) continue;
            float mn[8], s2[8];
            int ix[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                mn[e] = INFINITY;
                s2[e] = INFINITY;
                ix[e] = 0;
            }
#pragma unroll 1
            for (int hb = 0; hb < 2; ++hb) {
                const int pos = 64 * wave + 32 * hb;
                floatx16 bet, alp;
                products(pos, bet, alp);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float a0 = sm.a00[pos + 8 * (r >> 2) + 4 * half + (r & 3)];
                    const int k = 16 * hb + r;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int j = 4 * grp + jj;
                        // the main scan's operations on the same operands
                        const float q = fmaf(a0, usq[j], alp[r]);
                        const float c2[2] = {fmaf(bet[r], uj[j], q), fmaf(-bet[r], uj[j], q)};
#pragma unroll
                        for (int sg = 0; sg < 2; ++sg) {
                            const int e = 2 * jj + sg;
                            const float c = c2[sg];
                            // best and second best so far, first index of the best
                            s2[e] = __builtin_amdgcn_fmed3f(mn[e], c, s2[e]);
                            ix[e] = c < mn[e] ? k : ix[e];
                            mn[e] = fminf(mn[e], c);
                        }
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int p = 8 * grp + e;
                if (!(want >> p & 1u)) continue;
                if (mn[e] != fb[p]) lostm |= 1u << p;
                // ix = 16 (block of 32 within the super-block) + r
                const int blk32 = ix[e] >> 4, r = ix[e] & 15;
                blk[p] = wb * kHybSB + 32 * blk32 + 8 * (r >> 2) + 4 * half + (r & 3);
                fs[p] = fminf(fs[p], s2[e]);
            }
        }
        // the area is rewritten by the next super-block
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // lane h keeps its pairs' rows below the anchor (h = 0) or above it
    // (h = 1), in row order p from t.k0w: h = 1 owns pixel (j = p, +), h = 0
    // pixel (j = NJ - 1 - p, -); the partner's seed and runner-up of those
    // pixels arrive by a swap across the half-waves
    const bool lane_ok = lane_in_grid<D>(g, t);
    const float sab = dslack_abs(g, wmax, ct), skb = kslack(ct);
    const unsigned owin = (unsigned)__shfl_xor((int)win, 32);
    const unsigned olost = (unsigned)__shfl_xor((int)lostm, 32);
    bool act[NJ], flag[NJ];
    int lab[NJ];
#pragma unroll
    for (int p = 0; p < NJ; ++p) {
        const int pa = 2 * p, pb = 2 * (NJ - 1 - p) + 1;  // (p, +) and (NJ - 1 - p, -)
        const int pm = half ? pa : pb;
        const float nb = fb[pm];  // equal in both halves
        const float ms = fs[pm];
        const int mi = blk[pm];
        const float os = __shfl_xor(half ? fs[pb] : fs[pa], 32);
        const int oi = __shfl_xor(half ? blk[pb] : blk[pa], 32);
        const bool mw = (win >> pm) & 1u, ow = (owin >> pm) & 1u;
        const float ns = fminf(ms, os);
        lab[p] = seed_at(min(mw && ow ? min(mi, oi) : mw ? mi : oi, g.n - 1));
        act[p] = lane_ok && t.k0w + p < g.grid[0];
        const float u0 = half ? uj[p] : -uj[NJ - 1 - p];
        const float r2 = pixel_r2(ct, u0, u1, u2);
        const float bb = fmaxf(nb, 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float e1 = hyb_bound<D>(B1, sqrtf(r2), r2);
        const float thr = 2.0f * e1 + sab + skb * (B1 + r2);
        flag[p] = ((lostm | olost) >> pm & 1u) || !((ns - nb) > thr);
        if (out.rel_gap && act[p] && !flag[p]) {
            const float c1u = (nb + 0x1p-19f * fabsf(nb) + e1 + sab + skb * (B1 + r2)) * (1.0f + 0x1p-20f);
            const float f2 = pad_inf(ns);
            const float bs = fmaxf(f2, 0.0f);
            const float B2 = bs + 0x1p-10f * (bs + r2);
            const float c2l = f2 == INFINITY ? f2
                              : (f2 - 0x1p-19f * fabsf(f2) - hyb_bound<D>(B2, sqrtf(r2), r2) - sab - skb * (B2 + r2)) *
                                    (1.0f - 0x1p-20f);
            out.rel_gap[pixel_index<D>(g, t.k0w + p, t)] = ns > 0.0f ? gap_lower(c1u, c2l) : 0.0f;
        }
    }
    tile_epilogue<D, NJ>(g, t, act, lab, flag, out, qcount);
}

// ------------------------------------------------------- bf16 matrix cores

// Slots of the bf16 dot product.  In tile-local half-pixel units
// v_d = 2 (k_d - anchor_d) + 1 (odd integers) the features are small
// integers, and every one of them is exactly a bf16 "hi" plus a bf16 "lo"
// part; each coefficient c is split as c_hi + c_lo (16 significant bits).
// A quadratic term c f takes three slots (c_hi f_hi, c_hi f_lo, c_lo f_hi),
// a linear one two (c_hi f, c_lo f), the constant three (c_hi + c_mid +
// c_lo, 24 significant bits: the constant carries the weight offset
// w_max - w, often the largest term).  2D: 3 x 3 + 2 x 2 + 3 = 16 slots (one
// 32x32x16 MFMA); 3D: 6 x 3 + 3 x 2 + 3 = 27 (two).
template <int D> struct Bf16Slots {
    static constexpr int NQ = D == 2 ? 3 : 6;   // quadratic features
    static constexpr int NL = D;                // linear features
    static constexpr int SLOTS = D == 2 ? 16 : 32;
    static constexpr int NM = SLOTS / 16;       // MFMAs per 32x32 block
    static_assert(3 * NQ + 2 * NL + 3 <= SLOTS, "bf16 slots");
};

// The coefficient side of the slots for one seed: c[0..NQ) quadratic,
// c[NQ..NQ+NL) linear, c[NQ+NL] constant.
template <int D>
__device__ inline void bf16_seed_slots(const float *c, unsigned short *out) {
    using SL = Bf16Slots<D>;
    int q = 0;
#pragma unroll
    for (int k = 0; k < SL::NQ + SL::NL + 1; ++k) {
        const unsigned short hi = bf16_bits(c[k]);
        const float rest = c[k] - bf16_value(hi);  // exact
        const unsigned short lo = bf16_bits(rest);
        out[q++] = hi;
        if (k < SL::NQ) out[q++] = hi;  // against f_lo
        if (k == SL::NQ + SL::NL) {
            // the constant: hi + mid + lo, each difference exact
            out[q++] = lo;
            out[q++] = bf16_bits(rest - bf16_value(lo));
        } else {
            out[q++] = lo;
        }
    }
#pragma unroll
    for (; q < SL::SLOTS; ++q) out[q] = 0;
}

// The feature side of the slots for one pixel: f as for the coefficients.
template <int D>
__device__ inline void bf16_pixel_slots(const float *f, unsigned short *out) {
    using SL = Bf16Slots<D>;
    int q = 0;
#pragma unroll
    for (int k = 0; k < SL::NQ + SL::NL + 1; ++k) {
        const unsigned short hi = bf16_bits(f[k]);
        if (k < SL::NQ) {
            const unsigned short lo = bf16_bits(f[k] - bf16_value(hi));
            out[q++] = hi;  // c_hi f_hi
            out[q++] = lo;  // c_hi f_lo
            out[q++] = hi;  // c_lo f_hi
        } else {
            out[q++] = hi;  // c_hi f (exact)
            out[q++] = hi;  // c_lo f
            if (k == SL::NQ + SL::NL) out[q++] = hi;  // the constant's third part
        }
    }
#pragma unroll
    for (; q < SL::SLOTS; ++q) out[q] = 0;
}

// LDS of the bf16 tile: per staged seed its bf16 slots (the matrix-core
// operand, seed-major so that a lane reads its 8 slots with one 16-byte
// load) and its FP32 coefficients in the layout of the vector tile
// (a00, 2a01, a11, -2(Ae)_0 | -2(Ae)_1, e^T A e - w' in 2D; the 3D rows
// hold a00, 2a01, 2a02, -2(Ae)_0 | a11, 2a12, a22, -2(Ae)_1 | -2(Ae)_2,
// e^T A e - w'); with candidate lists, the tile's list.
template <int D, int C, bool CULL>
struct Bf16Smem {
    static constexpr int kChunk = C;
    ushort8 sA[C * Bf16Slots<D>::SLOTS / 8];
    float4 sF4[D - 1][C];
    float2 sF2[C];
    int list[CULL ? kCullCap : 1];
    double red[kWaves];
    int redi[kWaves];
    int cnt;
};

// Rows per lane of the bf16 tile: 4 in 2D, 2 in 3D (its two matrix-core
// operands per block need twice the registers).
template <int D> struct Bf16Rows { static constexpr int value = D == 2 ? 4 : 2; };

// The bf16 tier of one tile, in the vector tile's geometry (tile_at: P
// pixels per lane along axis 0), so that it shares the candidate lists, the
// super-tiles and the re-check's tile layout.  A wave's pixels form 2P
// groups of 32: group 2r + c holds pixel r of lanes 32c .. 32c + 31, its
// column col that of lane 32c + col.  A 32-seed x 32-pixel block of costs
// is one (2D) or two (3D) v_mfma_f32_32x32x16_bf16 with the seeds on rows,
// so each lane holds 16 costs of one pixel (its column in the group)
// against 16 seeds (rows 8(r/4) + 4h + r%4 for the lane half h).  Those 16
// form a group:
//  * scan: per block and pixel group, the group minimum by 3-input integer
//    minima of the costs' bits (integer order is float order for the
//    non-negative costs; mixed-sign or negative near-ties fail the
//    certificate below), then the two smallest group minima and the group
//    of the best -- 12 operations per 16 pairs;
//  * at the end of each staged chunk the winning group of each pixel (over
//    both lane halves) is evaluated again in FP32 with the vector tile's
//    formulas, 8 seeds per lane half: this gives the label (the index is
//    kept in the low 4 bits of the FP32 cost) and the second-smallest cost
//    inside the group;
//  * certificate: with fb, fs the best and second FP32 costs of the winning
//    group and so the smallest bf16 group minimum of every other group, a
//    pixel is settled when fs - fb > 2 rho32 T + 2^-18 max|.| (as the FP32
//    tier) and so - fb > 2 rho16 T + 2^-18 max|.| (both plus the slack of
//    the double costs), rho32 = 2^-18 the bound of the FP32 costs and
//    rho16 = 2^-15 that of the bf16 costs.  Per monomial c f (c its FP32
//    coefficient in half-pixel units, f its integer feature): the
//    coefficient is within 2^-24 (1 + 2^-50) of its value; rounding to 8
//    significant bits gives |c - c_hi| <= 2^-8 |c| and |c - c_hi - c_lo|
//    <= 2^-16 |c|; f = f_hi + f_lo exactly (|v| < 64, so f < 2^12); the
//    slots hold c_hi f_hi + c_hi f_lo + c_lo f_hi = (c_hi + c_lo) f -
//    c_lo f_lo with |c_lo f_lo| <= 2^-16 (1 + 2^-8) |c f|; every product of
//    two bf16 numbers is exact in FP32; the accumulation of at most 31
//    products (two blocks of 16 slots in 3D, 15 in 2D) adds at most
//    gamma_31 < 2^-19 of sum |c f|.  So |C_bf16 - C| <= (2^-15 + 2^-19 +
//    2^-23) S (to first order) <= 1.07 2^-15 S, and S <= T / 1.13 as above: the
//    error is within rho16 T for any symmetric positive definite A_i.
//    Any seed that could beat the label would contradict one of the two
//    gaps, as in the single-tier argument; a negative bf16 minimum among
//    the other groups (integer order reversed) leaves so <= 0 < fb + the
//    gap, so such pixels are never settled.  Other pixels go to the double
//    re-check.
// The features are exact bf16 hi + lo pairs: in half-pixel units they are
// integers below 2^12 (|v| < 64).  With CULL the tile scans its candidate
// list (built as the vector tile builds it, from its super-tile's list
// when there is one) and keeps it for the re-check.
template <int D, int P, int C, bool CULL>
__device__ inline void bf16_tile(const Geo &g, const Seeds &sd, double wmax, Cert ct,
                                 const double *eig, int b0, int b1, int b2,
                                 Bf16Smem<D, C, CULL> &sm, const PassOut &out, unsigned *qcount) {
    using SL = Bf16Slots<D>;
    static_assert(C % 32 == 0, "bf16 staging");
    constexpr int NG = 2 * P;  // 32-pixel groups per wave: gi = 2 r + c
    constexpr int E0 = tile_ext(D, P, 0), E1 = tile_ext(D, P, 1), E2 = tile_ext(D, P, 2);
    constexpr int kQ = SL::SLOTS / 8;  // 16-byte operand pieces per seed
    constexpr float kPad = 1.7e38f;

    const Tile<D> t = tile_at<D, P>(b0, b1, b2);
    const int lane = t.lane;
    const int half = lane >> 5, col = lane & 31;

    double ancd[3];
    float s[3];
    for (int d = 0; d < D; ++d) {
        ancd[d] = g.lo[d] + (double)t.anc[d] * g.s[d];
        s[d] = (float)g.s[d];
    }
    // the pixels of column col of each group: those of lane L = 32 c + col
    // of the wave (its first row k0c[c], its other indices), in FP32 and in
    // half-pixel units
    float u1c[2], u2c[2], v1c[2], v2c[2];
    int k0c[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        int k1, k2;
        lane_pixel<D, P>(t.org, 32 * c + col, k0c[c], k1, k2);
        u1c[c] = ((float)(k1 - t.anc[1]) + 0.5f) * s[1];
        u2c[c] = D == 3 ? ((float)(k2 - t.anc[2]) + 0.5f) * s[2] : 0.0f;
        v1c[c] = (float)(2 * (k1 - t.anc[1]) + 1);
        v2c[c] = D == 3 ? (float)(2 * (k2 - t.anc[2]) + 1) : 0.0f;
    }
    // matrix-core operand B (this lane's half of the pixel slots) per group
    bf16x8 bf[NG][SL::NM];
    float u0[NG];
#pragma unroll
    for (int r = 0; r < P; ++r) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int k0 = k0c[c] + r;
            u0[2 * r + c] = ((float)(k0 - t.anc[0]) + 0.5f) * s[0];
            const float v0 = (float)(2 * (k0 - t.anc[0]) + 1);
            const float v1 = v1c[c], v2 = v2c[c];
            float f[10];
            if (D == 2) {
                f[0] = v0 * v0; f[1] = v0 * v1; f[2] = v1 * v1;
                f[3] = v0; f[4] = v1; f[5] = 1.0f;
            } else {
                f[0] = v0 * v0; f[1] = v0 * v1; f[2] = v0 * v2;
                f[3] = v1 * v1; f[4] = v1 * v2; f[5] = v2 * v2;
                f[6] = v0; f[7] = v1; f[8] = v2; f[9] = 1.0f;
            }
            unsigned short sl[SL::SLOTS];
            bf16_pixel_slots<D>(f, sl);
#pragma unroll
            for (int m = 0; m < SL::NM; ++m) {
                ushort8 u;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) u[jj] = half ? sl[16 * m + 8 + jj] : sl[16 * m + jj];
                bf[2 * r + c][m] = __builtin_bit_cast(bf16x8, u);
            }
        }
    }

    // ---- the candidate list, from the super-tile's list when it has one
    int nscan = g.n;
    bool full = true;
    int ncand_kept = 0;
    double Utile = INFINITY;  // no seed left out of the tile's list costs less
    if (CULL) {
        double blo[3], bhi[3];
        const int ext[3] = {E0, E1, E2};
        const int k0[3] = {t.anc[0] - E0 / 2, t.anc[1] - E1 / 2, D == 3 ? t.anc[2] - E2 / 2 : 0};
        cull_box<D>(g, k0, ext, blo, bhi);
        const int *src = nullptr;
        int nsrc = g.n;
        if (out.super_list) {
            const int st = ((b0 / out.sf[0]) * out.nst[1] + b1 / out.sf[1]) * out.nst[2] + b2 / out.sf[2];
            const int c = out.super_count[st];
            if (c <= out.super_cap) {
                src = out.super_list + (size_t)st * out.super_cap;
                nsrc = c;
            }
        }
        const int ncand = build_candidates<D>(sd, eig, wmax, blo, bhi, src, nsrc, sm.list, kCullCap, sm.cnt,
                                              sm.red, &Utile);
        full = ncand > kCullCap;
        nscan = full ? g.n : ncand;
        ncand_kept = ncand;
        if (full || ncand >= g.n) Utile = INFINITY;  // no seed was left out
        if (out.adaptive && !full && !g.mass && !out.rel_gap) {
            const int own = box_owner<D>(sd, wmax, blo, bhi, sm.list, ncand, sm.red, sm.redi);
            if (own >= 0) {
                credit_tile<D, P>(g, t, b0, b1, b2, own, out);
                return;
            }
        }
    }

    // staging of scan positions [base, base + cnt), padded to a multiple of
    // 32 with entries that cost 1.7e38 everywhere
    auto stage = [&](int base, int cnt, int padded) {
        for (int q = threadIdx.x; q < padded; q += kThreads) {
            float c[10];  // bf16-slot coefficients (half-pixel units)
            if (q >= cnt) {
#pragma unroll
                for (int z = 0; z < 10; ++z) c[z] = 0.0f;
                c[SL::NQ + SL::NL] = kPad;
                for (int r = 0; r < D - 1; ++r) sm.sF4[r][q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                sm.sF2[q] = make_float2(0.0f, kPad);
            } else {
                const int i = (CULL && !full) ? sm.list[base + q] : base + q;
                double qd[6], ld[3], cd, ed[3], wpd;
                seed_terms<D>(sd, i, ancd, wmax, qd, ld, &cd, ed, &wpd);
                const double h0 = 0.5 * g.s[0], h1 = 0.5 * g.s[1], h2 = D == 3 ? 0.5 * g.s[2] : 0.0;
                if (D == 2) {
                    sm.sF4[0][q] = make_float4((float)qd[0], (float)qd[1], (float)qd[2], (float)ld[0]);
                    sm.sF2[q] = make_float2((float)ld[1], (float)cd);
                    c[0] = (float)(qd[0] * h0 * h0); c[1] = (float)(qd[1] * h0 * h1);
                    c[2] = (float)(qd[2] * h1 * h1);
                    c[3] = (float)(ld[0] * h0); c[4] = (float)(ld[1] * h1); c[5] = (float)cd;
                } else {
                    sm.sF4[0][q] = make_float4((float)qd[0], (float)qd[1], (float)qd[2], (float)ld[0]);
                    sm.sF4[D - 2][q] = make_float4((float)qd[3], (float)qd[4], (float)qd[5], (float)ld[1]);
                    sm.sF2[q] = make_float2((float)ld[2], (float)cd);
                    c[0] = (float)(qd[0] * h0 * h0); c[1] = (float)(qd[1] * h0 * h1);
                    c[2] = (float)(qd[2] * h0 * h2); c[3] = (float)(qd[3] * h1 * h1);
                    c[4] = (float)(qd[4] * h1 * h2); c[5] = (float)(qd[5] * h2 * h2);
                    c[6] = (float)(ld[0] * h0); c[7] = (float)(ld[1] * h1); c[8] = (float)(ld[2] * h2);
                    c[9] = (float)cd;
                }
            }
            unsigned short sl[SL::SLOTS];
            bf16_seed_slots<D>(c, sl);
#pragma unroll
            for (int m = 0; m < kQ; ++m) {
                ushort8 u;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) u[jj] = sl[8 * m + jj];
                sm.sA[q * kQ + m] = u;
            }
        }
    };
    // FP32 cost of staged seed q at the pixel (v0, v1, v2) (tile-local
    // coordinates; the vector tile's formulas)
    auto cost32 = [&](int q, float v0, float v1, float v2) {
        const float4 c0 = sm.sF4[0][q];
        const float2 cl = sm.sF2[q];
        float beta, alpha;
        if constexpr (D == 2) {
            beta = fmaf(c0.y, v1, c0.w);
            alpha = fmaf(fmaf(c0.z, v1, cl.x), v1, cl.y);
        } else {
            const float4 c1 = sm.sF4[D - 2][q];
            beta = fmaf(c0.y, v1, fmaf(c0.z, v2, c0.w));
            alpha = fmaf(fmaf(c1.x, v1, fmaf(c1.y, v2, c1.w)), v1, fmaf(fmaf(c1.z, v2, cl.x), v2, cl.y));
        }
        return fmaf(fmaf(c0.x, v0, beta), v0, alpha);
    };

    // group minima (bf16 costs as integers): best, second, block of the best
    int best[NG], second[NG], blk[NG];
    // the winning group evaluated in FP32: scan position, best and second keys
    int lab[NG], kb[NG], ks[NG];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        best[gi] = 0x7fffffff;
        second[gi] = 0x7fffffff;
        blk[gi] = -1;
        lab[gi] = 0;
        kb[gi] = 0x7fffffff;
        ks[gi] = 0x7fffffff;
    }
    for (int base = 0; base < nscan; base += C) {
        const int cnt = min(C, nscan - base);
        const int padded = (cnt + 31) & ~31;
        __syncthreads();
        stage(base, cnt, padded);
        __syncthreads();
        for (int cb = 0; cb < padded; cb += 32) {
            bf16x8 av[SL::NM];
#pragma unroll
            for (int m = 0; m < SL::NM; ++m)
                av[m] = __builtin_bit_cast(bf16x8, sm.sA[(cb + col) * kQ + 2 * m + half]);
            floatx16 acc[NG];
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                acc[gi] = floatx16{};
#pragma unroll
                for (int m = 0; m < SL::NM; ++m)
                    acc[gi] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bf[gi][m], acc[gi], 0, 0, 0);
            }
            const int gblk = base + cb;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                int k[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) k[r] = __float_as_int(acc[gi][r]);
                const int t0 = min(min(k[0], k[1]), k[2]);
                const int t1 = min(min(k[3], k[4]), k[5]);
                const int t2 = min(min(k[6], k[7]), k[8]);
                const int t3 = min(min(k[9], k[10]), k[11]);
                const int t4 = min(min(k[12], k[13]), k[14]);
                const int m = min(min(min(t0, t1), t2), min(min(t3, t4), k[15]));
                second[gi] = med3i(best[gi], m, second[gi]);
                blk[gi] = m < best[gi] ? gblk : blk[gi];
                best[gi] = min(best[gi], m);
            }
        }
        // the pixel's winning group (ties to lane half 0); where it was
        // found in this chunk, evaluate it again in FP32
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            const int pb = __shfl_xor(best[gi], 32);
            const int pblk = __shfl_xor(blk[gi], 32);
            const bool other = half == 0 ? pb < best[gi] : pb <= best[gi];
            const int wblk = other ? pblk : blk[gi];
            const int wh = other ? 1 - half : half;
            const bool need = wblk >= base;
            if (__ballot(need)) {
                // rows r = 8 half .. 8 half + 7 of the group: seeds
                // wblk + 8 (r / 4) + 4 wh + r % 4
                const int q0 = max(wblk - base, 0) + 4 * wh + 16 * half;
                int bk = 0x7fffffff, s2 = 0x7fffffff;
#pragma unroll
                for (int rr = 0; rr < 8; ++rr) {
                    const int q = q0 + 8 * (rr >> 2) + (rr & 3);
                    const float c = cost32(q, u0[gi], u1c[gi & 1], u2c[gi & 1]);
                    const int key = (__float_as_int(c) & ~15) | (8 * half + rr);
                    s2 = med3i(bk, key, s2);
                    bk = min(bk, key);
                }
                const int ob = __shfl_xor(bk, 32);
                const int os = __shfl_xor(s2, 32);
                const int nb = min(bk, ob);
                const int ns = min(max(bk, ob), min(s2, os));
                if (need) {
                    const int r = nb & 15;
                    lab[gi] = wblk + 8 * (r >> 2) + 4 * wh + (r & 3);
                    kb[gi] = nb;
                    ks[gi] = ns;
                }
            }
        }
    }

    const float sab = dslack_abs(g, wmax, ct), skb = kslack(ct);
    // lane l takes to the epilogue the groups of its own column half (the
    // pixels of column l % 32 of those groups are its own)
    const bool lane_ok = lane_in_grid<D>(g, t);
    bool act[P], flag[P];
    int labe[P];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int pb = __shfl_xor(best[gi], 32);
        const int ps = __shfl_xor(second[gi], 32);
        const int so = min(max(best[gi], pb), min(second[gi], ps));
        const float fb = __int_as_float(kb[gi]), fs = __int_as_float(ks[gi]);
        const float fo = __int_as_float(so);
        const float r2 = pixel_r2(ct, u0[gi], u1c[gi & 1], u2c[gi & 1]);
        const float rr = sqrtf(r2);
        const float bb = fmaxf(fb, 0.0f);
        const float B1 = bb + 0x1p-10f * (bb + r2);
        const float e32 = e32_bound(B1, rr, r2), e16 = e16_bound(B1, rr, r2);
        const float slack = sab + skb * (B1 + r2);
        const float thr32 = 2.0f * e32 + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fs)) + slack;
        const float thr16 = e32 + e16 + 0x1p-18f * fmaxf(fabsf(fb), fabsf(fo)) + slack;
        const bool settled = (fs - fb) > thr32 && (fo - fb) > thr16;
        const int r = gi >> 1;
        if ((gi & 1) == half) {
            const int pos = min(lab[gi], nscan - 1);
            act[r] = lane_ok && (t.k0w + r) < g.grid[0];
            flag[r] = !settled;
            labe[r] = (CULL && !full) ? sm.list[pos] : min(pos, g.n - 1);
            if (out.rel_gap && act[r] && settled) {
                // the winner costs at most c1u; the rest of its group at
                // least fs, the other groups at least fo, each less its bound,
                // and a seed left out of the list more than U
                const float c1u = (fb + 0x1p-19f * fabsf(fb) + e32 + slack) * (1.0f + 0x1p-20f);
                const float f2 = pad_inf(fs), fo2 = pad_inf(fo);
                const float bs = fmaxf(f2, 0.0f), bo = fmaxf(fo2, 0.0f);
                const float Bs = bs + 0x1p-10f * (bs + r2), Bo = bo + 0x1p-10f * (bo + r2);
                const float cs = f2 == INFINITY
                                     ? f2
                                     : f2 - 0x1p-19f * fabsf(f2) - e32_bound(Bs, rr, r2) - sab - skb * (Bs + r2);
                const float co = fo2 == INFINITY ? fo2 : fo2 - e16_bound(Bo, rr, r2) - sab - skb * (Bo + r2);
                const float uc = (float)Utile;
                const float c2l = fminf(fminf(cs, co), (uc == INFINITY ? uc : uc - 0x1p-20f * fabsf(uc))) * (1.0f - 0x1p-20f);
                out.rel_gap[pixel_index<D>(g, t.k0w + r, t)] =
                    (fs > 0.0f && fo > 0.0f) ? gap_lower(c1u, c2l) : 0.0f;
            }
        }
    }
    PassOut o = out;
    if (CULL && out.tile_lists) {
        // keep the candidates for the re-check of this tile's queued pixels
        const int tid = ((b0 * out.ntile[1]) + b1) * out.ntile[2] + b2;
        o.tile_id = tid;
        const bool keep = !full && ncand_kept <= out.list_cap;
        if (keep)
            for (int q = threadIdx.x; q < ncand_kept; q += kThreads)
                out.tile_lists[(size_t)tid * out.list_cap + q] = sm.list[q];
        if (threadIdx.x == 0) {
            out.tile_count[tid] = keep ? ncand_kept : out.list_cap + 1;
            if (out.tile_U) out.tile_U[tid] = keep ? Utile : INFINITY;
        }
    }
    tile_epilogue<D, P>(g, t, act, labe, flag, o, qcount);
}

// ------------------------------------------------------- double re-check

// Seeds staged in LDS for the double re-check: x, the upper triangle of A
// (row by row) and w of up to S seeds, and their seed numbers.
template <int D, int S>
struct StagedSeeds {
    static constexpr int kSeeds = S;
    static constexpr int kTri = D * (D + 1) / 2;
    int idx[S];
    double x[D][S];
    double a[kTri][S];
    double w[S];
};

// Stage seed `i` at position q (every thread of the block calls it for its
// positions; a barrier must follow before the reads).
template <int D, int S>
__device__ inline void stage_seed(StagedSeeds<D, S> &sm, const Seeds &sd, int q, int i) {
    const double *xi = sd.x + (size_t)i * D;
    const double *ai = sd.A + (size_t)i * D * D;
    int t = 0;
    for (int r = 0; r < D; ++r) {
        sm.x[r][q] = xi[r];
        for (int c = r; c < D; ++c, ++t) sm.a[t][q] = ai[r * D + c];
    }
    sm.w[q] = sd.w[i];
    sm.idx[q] = i;
}

// The double cost of the staged seed at position q at y, in the expression
// order of exact_cost (the same roundings, so the same value).
template <int D, int S>
__device__ inline double staged_cost(const StagedSeeds<D, S> &sm, int q, const double *y) {
    double dd[D];
#pragma unroll
    for (int e = 0; e < D; ++e) dd[e] = y[e] - sm.x[e][q];
    double qf = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
        double row = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int lo = e < c ? e : c, hi = e < c ? c : e;
            const int tix = lo * D - lo * (lo - 1) / 2 + (hi - lo);  // (lo, hi) packed
            const double t = sm.a[tix][q] * dd[c];
            row = (c == 0) ? t : row + t;
        }
        const double t = dd[e] * row;
        qf = (e == 0) ? t : qf + t;
    }
    return qf - sm.w[q];
}

// Grid index k and centre y of pixel j (eq. (2.6)).
template <int D>
__device__ inline void pixel_of(const Geo &g, uint32_t j, int *k, double *y) {
    uint32_t r = j;
    for (int d = D - 1; d >= 0; --d) {
        k[d] = (int)(r % (uint32_t)g.grid[d]);
        r /= (uint32_t)g.grid[d];
    }
    for (int d = 0; d < D; ++d) y[d] = centre(g, d, k[d]);
}

// (value, seed) minimum over the G lanes of a group (G a power of two up to
// 64, groups aligned within the wave): the lowest seed among equal values.
__device__ inline void group_min(double &b, int &bi, int G) {
    for (int o = G / 2; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(b, o);
        const int oi = __shfl_xor(bi, o);
        if (ob < b || (ob == b && oi < bi)) {
            b = ob;
            bi = oi;
        }
    }
}

// The same with the runner-up value s (the smallest value other than the
// winner's, ties included) carried along.
__device__ inline void group_min2(double &b, int &bi, double &s, int G) {
    for (int o = G / 2; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(b, o);
        const int oi = __shfl_xor(bi, o);
        const double os = __shfl_xor(s, o);
        if (ob < b || (ob == b && oi < bi)) {
            s = fmin(os, b);
            b = ob;
            bi = oi;
        } else {
            s = fmin(s, ob);
        }
    }
}

// Orders this wave's LDS writes before its lanes' later reads (and earlier
// reads before later writes): the wave's own barrier.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Double re-check, by one wave, of the `count` queued pixels from queue
// position `start`, all of one tile, against the tile's candidate list
// (list[0, nlist), seed numbers) or, without one, every seed.  The
// candidates are staged in the wave's own LDS (sm) chunk by chunk; a group
// of G lanes takes one pixel (G the largest power of two, up to 64, that
// leaves a group for every pixel of the segment), lane r of the group scans
// the staged positions r, r + G, ...  The list holds every seed that can
// attain the minimum anywhere in the tile, exact ties included, so the
// (value, lowest seed) minimum equals that of a scan over every seed in the
// definition's order.  pixel_at(q) gives the pixel index at queue position
// q.  Every lane of the wave must call it.
//
// With rel_gap it also writes each pixel's relative top-two gap
// (gap_exact): the runner-up over the list, or, below it, the list's bound
// U (in the gauge w - w_max) under which no seed outside the list costs.
template <int D, int S, class PixelAt>
__device__ inline void recheck_segment(const Geo &g, const Seeds &sd, unsigned start, unsigned count,
                                       const int *list, int nlist, PixelAt pixel_at, int32_t *labels,
                                       uint64_t *mom, StagedSeeds<D, S> &sm, float *rel_gap = nullptr,
                                       double wmax = 0.0, double U = INFINITY) {
    const int lane = __lane_id();
    const int nseed = list ? nlist : g.n;
    int G = 64;
    while (G > 1 && (unsigned)(64 / G) < count) G >>= 1;
    const unsigned ngroups = (unsigned)(64 / G);
    const int grp = lane / G, r = lane % G;
    for (unsigned p0 = 0; p0 < count; p0 += ngroups) {
        const unsigned p = p0 + (unsigned)grp;
        const bool valid = p < count;
        const uint32_t j = valid ? pixel_at(start + p) : 0u;
        int k[3];
        double y[D];
        pixel_of<D>(g, j, k, y);
        double b = INFINITY, s2 = INFINITY;
        int bi = 0x7fffffff;
        for (int c0 = 0; c0 < nseed; c0 += S) {
            const int cnt = min(S, nseed - c0);
            wave_lds_sync();
            for (int q = lane; q < cnt; q += 64) stage_seed<D, S>(sm, sd, q, list ? list[c0 + q] : c0 + q);
            wave_lds_sync();
            for (int q = r; q < cnt; q += G) {
                const double c = staged_cost<D, S>(sm, q, y);
                const int i = sm.idx[q];
                if (c < b || (c == b && i < bi)) {
                    s2 = b;
                    b = c;
                    bi = i;
                } else {
                    s2 = fmin(s2, c);
                }
            }
        }
        if (rel_gap) group_min2(b, bi, s2, G);
        else group_min(b, bi, G);
        if (bi >= g.n) bi = 0;  // no finite cost (non-finite input, reported by the prep step)
        if (valid && r == 0) {
            if (labels) labels[j] = bi;
            if (mom) pixel_moments_add<D>(mom, bi, k, pixel_weight(g, j));
            if (rel_gap) {
                // a seed outside the list costs more than U - w_max (unshifted)
                const double su = U - wmax;
                rel_gap[j] = su < s2 ? gap_exact(b, su - 1e-9 * fabs(U), wmax) : gap_exact(b, s2, wmax);
            }
        }
    }
}

// Finalize of one cell from its exact moments (o = 2k + 1, y = lo + h o,
// h = s/2):
//   m_i, grad_i = v_i - m_i |P|                                  eq. (2.8)
//   centroid ybar = lo + h S_d / m                                 Alg. 3
//   sum_{cell} |y - x_i|^2_A = m |ybar - x_i|^2_A
//                              + sum_de A_de h_d h_e (S_de - S_d S_e / m)
// returns the cell's term of eq. (2.7), (v_i - m_i |P|) w_i + |P| sum |y - x_i|^2_A,
// and its relative volume error.  For other costs (g.power != 2) the term is
// v_i w_i and the finalize adds |P| sum_j q_j C_{H_j j} (eq. (2.7) written
// over pixels), summed by the assignment kernel.
template <int D>
__device__ inline double cell_final(const Geo &g, const Seeds &sd, const uint64_t *M, int i,
                                   double *grad_i, double *rel_i, double *ybar) {
    const uint64_t m = M[0];
    const double md = (double)m;
    const double vi = sd.v[i], wi = sd.w[i];
    const double gi = vi - md * g.munit;
    *grad_i = gi;
    *rel_i = fabs(gi) / vi;
    const double *a = sd.A + (size_t)i * D * D;
    double h[3];
    for (int d = 0; d < D; ++d) h[d] = 0.5 * g.s[d];
    double integral = 0.0;
    if (m > 0 && g.power != 2) {
        // other costs: the cell's share of sum_j |P_j| C_{H_j j} is summed
        // pixel by pixel (Scalars::gpix); here only the centroid and v_i w_i
        for (int d = 0; d < D; ++d) ybar[d] = g.lo[d] + h[d] * ((double)M[1 + d] / md);
        return vi * wi;
    }
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
        integral = g.munit * (md * q1 + q2);
    } else {
        for (int d = 0; d < D; ++d) ybar[d] = sd.x[(size_t)i * D + d];
        if (g.power != 2) return vi * wi;
    }
    return gi * wi + integral;
}

}  // namespace dev
}  // namespace apd
