// apd_kernels.hip -- gfx950 kernels of the APD hot path.
//
// One evaluation of the discretised dual problem (Section 2.3 of
// arXiv 2403.03571) is a chain of kernels on one stream:
//
//   k_prep        blocks of seeds, the last to finish combining their
//                 partials: gauge max of w, Gershgorin bound and
//                 eigenvalue ranges of the anisotropy matrices, input
//                 validation, zeroed moments (in a fit's graph it also
//                 takes the trial weights from pinned host memory).
//   k_super_cull  candidate lists of super-tiles (passes with lists).
//   k_assign_*    the O(N J) part (Algorithm 1): every pixel of a tile
//                 scans every seed (or the tile's candidates), keeps the
//                 argmin, and the tile reduces the exact integer moments of
//                 each cell it touched.  _fp64 evaluates
//                 C_ij = |y_j - x_i|^2_{A_i} - w_i exactly as the definition
//                 is written; _vec (FP32 vector ALU), _mfma (FP32 matrix
//                 cores) and _bf16 (bf16 matrix cores) evaluate it in local
//                 coordinates and queue every pixel whose top-two gap is
//                 within their rounding bound.
//   k_recheck_*   re-runs the scan of every queued pixel in double, in
//                 the definition's own expression order, so every label
//                 equals that of an exact double-precision argmin (_staged:
//                 every seed, staged in LDS; _seg: a tile's candidate list,
//                 staged once for all the tile's queued pixels).
//   k_finalize    blocks of cells, the last to finish combining them:
//                 objective (2.7), gradient (2.8), maximum relative volume
//                 error, centroids, from the moments.
//
// The whole file is built with -ffp-contract=off: the double-precision
// costs are evaluated without fused multiply-adds, and the single-precision
// path fuses only where it says so (fmaf).
#include "apd_device.h"

#include <math.h>

#include <algorithm>

namespace apd {
namespace {

using namespace dev;

// ------------------------------------------------------------- k_prep

constexpr int kRedThreads = 256;
constexpr int kRedWaves = kRedThreads / 64;

// Seeds [lo, hi) of block b when n seeds are split over gridDim.x blocks.
__device__ inline void block_range(int n, int *lo, int *hi) {
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    *lo = min(n, (int)blockIdx.x * per);
    *hi = min(n, *lo + per);
}

// True in the last block to finish; its partials and those of every other
// block are then visible to it.
__device__ inline bool last_block(unsigned *ticket) {
    __shared__ bool s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (s_last) __threadfence();
    return s_last;
}

// Validation, max_i w_i, sum_i v_i, the Gershgorin bound of the largest
// eigenvalue, the eigenvalue ranges (culling) and the zeroed moments, over
// blocks of seeds.
template <int D>
__global__ __launch_bounds__(kRedThreads) void k_prep(Geo g, Seeds sd, Scalars *sc, uint64_t *mom,
                                                      double *eig, BlockParts *bp, const double *w_src) {
    constexpr int K = moments_per_cell(D);
    __shared__ double s_w[kRedWaves];
    __shared__ double s_v[kRedWaves];
    __shared__ float s_l[kRedWaves];
    __shared__ float s_k[kRedWaves];
    __shared__ int s_b[kRedWaves];
    const int tid = threadIdx.x;
    if (mom)
        for (size_t t = (size_t)blockIdx.x * kRedThreads + tid; t < (size_t)g.n * K;
             t += (size_t)gridDim.x * kRedThreads)
            mom[t] = 0ull;
    int i0, i1;
    block_range(g.n, &i0, &i1);
    double wm = -INFINITY, vs = 0.0;
    float lam = 0.0f, kap = 0.0f;
    int bad = 0;
    for (int i = i0 + tid; i < i1; i += kRedThreads) {
        double wi;
        if (w_src) {
            // the pass's weights, from the host; later kernels read sd.w
            wi = w_src[i];
            const_cast<double *>(sd.w)[i] = wi;
        } else {
            wi = sd.w[i];
        }
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
        double det = m2;
        if (D == 3) {
            det = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[1][2]) -
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
        double lg = 0.0;
        for (int r = 0; r < D; ++r) {
            double rs = 0.0;
            for (int c = 0; c < D; ++c) rs += fabs(u[r][c]);
            lg = fmax(lg, rs);
        }
        lam = fmaxf(lam, (float)lg);
        if (spd) kap = fmaxf(kap, (float)cond_bound(D, lg, det));
        if (sd.v) {
            const double vi = sd.v[i];
            if (!(vi > 0.0) || !isfinite(vi)) bad |= kBadV;
            vs += vi;
        }
    }
    // block reduction: a butterfly inside each wave, then the wave results
    // in wave order by thread 0 (whose slots 0 then hold the block's values)
    auto reduce = [&](double a, double v, float l, float kk, int b) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            a = fmax(a, __shfl_xor(a, o));
            v = v + __shfl_xor(v, o);
            l = fmaxf(l, __shfl_xor(l, o));
            kk = fmaxf(kk, __shfl_xor(kk, o));
            b = b | __shfl_xor(b, o);
        }
        __syncthreads();  // earlier readers of the slots are done
        if (__lane_id() == 0) {
            const int wv = tid >> 6;
            s_w[wv] = a;
            s_v[wv] = v;
            s_l[wv] = l;
            s_k[wv] = kk;
            s_b[wv] = b;
        }
        __syncthreads();
        if (tid == 0)
            for (int k = 1; k < kRedWaves; ++k) {
                s_w[0] = fmax(s_w[0], s_w[k]);
                s_v[0] = s_v[0] + s_v[k];
                s_l[0] = fmaxf(s_l[0], s_l[k]);
                s_k[0] = fmaxf(s_k[0], s_k[k]);
                s_b[0] = s_b[0] | s_b[k];
            }
    };
    reduce(wm, vs, lam, kap, bad);
    if (tid == 0) {
        bp->a[blockIdx.x] = s_w[0];
        bp->b[blockIdx.x] = s_v[0];
        bp->l[blockIdx.x] = s_l[0];
        bp->k[blockIdx.x] = s_k[0];
        bp->bad[blockIdx.x] = s_b[0];
    }
    if (!last_block(&bp->ticket)) return;
    const bool have = tid < (int)gridDim.x;
    reduce(have ? bp->a[tid] : -INFINITY, have ? bp->b[tid] : 0.0, have ? bp->l[tid] : 0.0f,
           have ? bp->k[tid] : 0.0f, have ? bp->bad[tid] : 0);
    if (tid == 0) {
        sc->wmax = s_w[0];
        sc->vsum = s_v[0];
        sc->lam = s_l[0] * 1.0001f;
        sc->kap = s_k[0] * 1.0001f;
        sc->bad = s_b[0];
        sc->qcount = 0u;
        sc->segcount = 0u;
        sc->credited = 0u;
        sc->gpix = 0.0;
        sc->g = 0.0;
        sc->maxrel = 0.0;
        sc->qtotal = 0ull;
        bp->ticket = 0u;
    }
}

// Zero n 32-bit words (a kernel rather than a memset, so that the call can
// sit inside a captured graph).
__global__ __launch_bounds__(256) void k_zero_words(unsigned *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

// sc->gpix = sum of part[0, n) in a fixed order: thread t sums t, t + 256, ...
// in order, then a tree over the threads (one block).
__global__ __launch_bounds__(256) void k_sum_parts(const double *part, int64_t n, Scalars *sc) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->gpix = red[0];
}

// sum_j mass[j] into sc->qtotal (after k_prep has zeroed it).
__global__ __launch_bounds__(256) void k_mass_total(int64_t J, const uint8_t *mass, Scalars *sc) {
    __shared__ unsigned long long red[256];
    unsigned long long s = 0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < J; j += (int64_t)gridDim.x * 256)
        s += mass[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&sc->qtotal, red[0]);
}

// Blocks for n seeds: one seed per thread up to kMaxParts blocks.
inline int red_blocks(int n) {
    return (int)std::min<int64_t>(kMaxParts, std::max<int64_t>(1, ((int64_t)n + kRedThreads - 1) / kRedThreads));
}

// ------------------------------------------------------ k_assign_fp64

// For costs other than the squared norm the block also sums its pixels'
// least costs, weighted by the pixel weights, in a fixed order (per lane,
// a butterfly in the wave, the waves in order) into out.cost_part.
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
    double best[kP], second[kP];
    int lab[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        best[p] = INFINITY;
        second[p] = INFINITY;
        lab[p] = 0;
    }
    for (int i = 0; i < g.n; ++i) {
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const double c = exact_cost<D>(sd.x, sd.A, sd.w, i, y[p], g.power);
            if (c < best[p]) {
                second[p] = best[p];
                best[p] = c;
                lab[p] = i;
            } else {
                second[p] = fmin(second[p], c);
            }
        }
    }
    bool flag[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        flag[p] = false;
        if (out.rel_gap && act[p])
            out.rel_gap[pixel_index<D>(g, t.k0w + p, t)] = gap_exact(best[p], second[p], sc->wmax);
    }
    if (out.cost_part) {
        __shared__ double s_part[kWaves];
        double sp = 0.0;
#pragma unroll
        for (int p = 0; p < kP; ++p)
            if (act[p]) sp += (double)pixel_weight(g, pixel_index<D>(g, t.k0w + p, t)) * best[p];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sp += __shfl_xor(sp, o);
        if (t.lane == 0) s_part[threadIdx.x >> 6] = sp;
        __syncthreads();
        if (threadIdx.x == 0) {
            const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            out.cost_part[b] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
        }
    }
    PassOut o = out;
    o.queue = nullptr;
    tile_epilogue<D>(g, t, act, lab, flag, o, nullptr);
}

// ------------------------------------------------ k_assign_fp32 / _cull

// One block per tile of the vector single-precision kernel
// (dev::vec_tile): every seed, or the tile's candidate seeds.
template <int D, bool CULL, int P>
__global__ __launch_bounds__(kThreads, (CULL && P == 4) ? 5 : 4) void k_assign_vec(Geo g, Seeds sd, Scalars *sc,
                                                        const double *eig, PassOut out) {
    __shared__ VecSmem<D, CULL> sm;
    if constexpr (D == 2)
        vec_tile<2, CULL, P>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, eig, blockIdx.y, blockIdx.x, 0, sm, out,
                             &sc->qcount);
    else
        vec_tile<3, CULL, P>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, eig, blockIdx.z, blockIdx.y, blockIdx.x, sm,
                             out, &sc->qcount);
}



// ------------------------------------------------------ k_assign_mfma

// One block per tile; the tile body (dev::mfma_tile) is shared with the
// batched persistent kernel.
template <int D>
__global__ __launch_bounds__(kThreads) void k_assign_mfma(Geo g, Seeds sd, Scalars *sc,
                                                         PassOut out) {
    __shared__ __attribute__((aligned(16))) float sC[kMfmaLds];
    if (D == 2)
        dev::mfma_tile<2>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, blockIdx.y, blockIdx.x, 0, sC, out, &sc->qcount);
    else
        dev::mfma_tile<3>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, blockIdx.z, blockIdx.y, blockIdx.x, sC, out,
                          &sc->qcount);
}

// ------------------------------------------------------ k_seed_order

// The seeds sorted by the Morton code of the box cell that holds them (16^3
// cells in 3D, 64^2 in 2D), by one block: counts per cell, an exclusive
// scan, then each seed's slot.  The hybrid kernel scans the seeds in this
// order, so that its super-blocks of 64 consecutive seeds cover compact
// regions and a wave's pixels fall in few of them (its winner search takes
// one round per distinct winning super-block).  Seeds of one cell take
// their slots in any order: the pass's labels, certificates and moments do
// not depend on it (an unflagged pixel's winner is the unique FP32 minimum;
// a flagged one is re-evaluated in double over every seed).
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 4096;

template <int D>
__device__ inline int seed_bin(const Geo &g, const Seeds &sd, int i) {
    constexpr int B = D == 3 ? 16 : 64;  // cells per axis
    constexpr int BITS = D == 3 ? 4 : 6;
    int q[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) {
        const double t = (sd.x[(size_t)i * D + d] - g.lo[d]) / (g.s[d] * (double)g.grid[d]);
        q[d] = t >= 0.0 ? (int)fmin(t * B, (double)(B - 1)) : 0;  // seeds outside the box clamp
    }
    int code = 0;
    for (int b = 0; b < BITS; ++b)
        for (int d = 0; d < D; ++d) code |= ((q[d] >> b) & 1) << (D * b + d);
    return code;
}

template <int D>
__global__ __launch_bounds__(kOrderThreads) void k_seed_order(Geo g, Seeds sd, int *ord) {
    __shared__ int cnt[kOrderBins];
    __shared__ int wex[kOrderThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int b = tid; b < kOrderBins; b += kOrderThreads) cnt[b] = 0;
    __syncthreads();
    for (int i = tid; i < g.n; i += kOrderThreads) atomicAdd(&cnt[seed_bin<D>(g, sd, i)], 1);
    __syncthreads();
    // exclusive scan: thread t holds cells 4t .. 4t + 3
    constexpr int PER = kOrderBins / kOrderThreads;
    int c[PER], sum = 0;
    for (int k = 0; k < PER; ++k) {
        c[k] = cnt[PER * tid + k];
        sum += c[k];
    }
    int inc = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wex[wave] = inc;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int w = 0; w < kOrderThreads / 64; ++w) {
            const int t = wex[w];
            wex[w] = run;
            run += t;
        }
    }
    __syncthreads();
    int off = wex[wave] + inc - sum;
    for (int k = 0; k < PER; ++k) {
        cnt[PER * tid + k] = off;
        off += c[k];
    }
    __syncthreads();
    for (int i = tid; i < g.n; i += kOrderThreads) ord[atomicAdd(&cnt[seed_bin<D>(g, sd, i)], 1)] = i;
}

// ------------------------------------------------------ k_assign_hyb

// One block per tile (dev::hyb_tile): 16 x 16 x 8 in 3D at three blocks per
// CU, so that the scan keeps its registers (at four, spills in the scan add
// about 4 GB of scratch traffic per launch on the 3D workload for the same
// time); 32 x 32 in 2D at four.
template <int D>
__global__ __launch_bounds__(kThreads, D == 3 ? 3 : 4) void k_assign_hyb(Geo g, Seeds sd, Scalars *sc,
                                                                          PassOut out) {
    __shared__ __attribute__((aligned(16))) HybSmem<D> sm;
    if constexpr (D == 3)
        hyb_tile<3>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, blockIdx.z, blockIdx.y, blockIdx.x, sm, out,
                    &sc->qcount);
    else
        hyb_tile<2>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, blockIdx.y, blockIdx.x, 0, sm, out, &sc->qcount);
}

// ------------------------------------------------------ k_assign_bf16

// One block per tile of the vector kernel's shape with P pixels per lane
// (dev::bf16_tile): every seed, or the tile's candidate seeds; seeds staged
// C at a time.
template <int D, int P, int C, bool CULL>
__global__ __launch_bounds__(kThreads) void k_assign_bf16(Geo g, Seeds sd, Scalars *sc,
                                                         const double *eig, PassOut out) {
    __shared__ dev::Bf16Smem<D, C, CULL> sm;
    const int b0 = D == 2 ? blockIdx.y : blockIdx.z;
    const int b1 = D == 2 ? blockIdx.x : blockIdx.y;
    const int b2 = D == 2 ? 0 : blockIdx.x;
    dev::bf16_tile<D, P, C, CULL>(g, sd, sc->wmax, Cert{sc->lam, sc->kap}, eig, b0, b1, b2, sm, out, &sc->qcount);
}

// --------------------------------------------------------- k_super_cull

// One block per super-tile (dev::super_tile_list).
template <int D>
__global__ __launch_bounds__(kThreads) void k_super_cull(Geo g, Seeds sd, const Scalars *sc,
                                                        const double *eig, PassOut out, int *list,
                                                        int *count) {
    __shared__ int s_cnt;
    __shared__ double s_red[kWaves];
    const int st = blockIdx.x;
    super_tile_list<D>(g, sd, sc->wmax, eig, out, st, list + (size_t)st * out.super_cap, count + st,
                       out.super_cap, s_cnt, s_red);
}

// ---------------------------------------------------------- k_recheck

// Seeds per staged chunk of the re-check kernels.
template <int D> struct RecheckChunk { static constexpr int value = D == 2 ? 1024 : 512; };
template <int D> struct SegChunk { static constexpr int value = 128; };  // per wave

// Re-check over every seed (passes without candidate lists): the seeds are
// staged in LDS chunk by chunk and a group of G lanes takes one queued
// pixel, G the largest power of two that still covers the whole queue in
// one round of the grid's waves (short queues spread each pixel over many
// lanes, long ones give every lane its own pixel); lane r of a group scans
// the staged seeds r, r + G, ... in increasing order, then the group takes
// the (value, lowest index) minimum.  The double cost is evaluated in the
// expression order of dev::exact_cost, so the labels are those of an exact
// double-precision argmin with ties to the lowest index.
template <int D>
__global__ __launch_bounds__(kThreads) void k_recheck_staged(Geo g, Seeds sd, const Scalars *sc,
                                                            PassOut out) {
    constexpr int S = RecheckChunk<D>::value;
    __shared__ StagedSeeds<D, S> sm;
    const unsigned nq = sc->qcount;
    const unsigned wslots = gridDim.x * kWaves;
    int G = 64;
    while (G > 1 && (unsigned long long)wslots * (unsigned)(64 / G) < nq) G >>= 1;
    const unsigned per_wave = 64u / (unsigned)G;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int n = g.n;
    for (unsigned base = 0; base < nq; base += wslots * per_wave) {
        // the whole block skips a round with none of its pixels
        const unsigned first = base + (unsigned)blockIdx.x * kWaves * per_wave;
        if (first >= nq) break;
        const unsigned pix = first + (unsigned)wave * per_wave + (unsigned)(lane / G);
        const bool valid = pix < nq;
        const uint32_t j = valid ? out.queue[pix] : 0u;
        int k[3];
        double y[D];
        pixel_of<D>(g, j, k, y);
        double b = INFINITY, s2 = INFINITY;
        int bi = 0x7fffffff;
        for (int c0 = 0; c0 < n; c0 += S) {
            const int cnt = min(S, n - c0);
            __syncthreads();
            for (int i = threadIdx.x; i < cnt; i += kThreads) stage_seed<D, S>(sm, sd, i, c0 + i);
            __syncthreads();
            for (int i = lane % G; i < cnt; i += G) {
                const double c = staged_cost<D, S>(sm, i, y);
                if (c < b) {
                    s2 = b;
                    b = c;
                    bi = c0 + i;
                } else {
                    s2 = fmin(s2, c);
                }
            }
        }
        if (out.rel_gap) group_min2(b, bi, s2, G);
        else group_min(b, bi, G);
        if (bi >= n) bi = 0;  // no finite cost (non-finite input, reported by the prep step)
        if (valid && lane % G == 0) {
            if (out.labels) out.labels[j] = bi;
            if (out.mom) dev::pixel_moments_add<D>(out.mom, bi, k, dev::pixel_weight(g, j));
            if (out.rel_gap) out.rel_gap[j] = dev::gap_exact(b, s2, sc->wmax);
        }
    }
}

// Re-check with the tiles' candidate lists: one wave per queue segment (the
// queued pixels of one tile), the tile's candidates staged once for all of
// them (dev::recheck_segment); a tile whose list overflowed scans every seed.
template <int D>
__global__ __launch_bounds__(kThreads) void k_recheck_seg(Geo g, Seeds sd, const Scalars *sc,
                                                         PassOut out) {
    constexpr int S = SegChunk<D>::value;
    __shared__ StagedSeeds<D, S> sm[kWaves];
    const unsigned nseg = sc->segcount;
    const int wave = threadIdx.x >> 6;
    for (unsigned s = blockIdx.x * kWaves + wave; s < nseg; s += gridDim.x * kWaves) {
        const QSeg seg = out.segs[s];
        const int cnt = out.tile_count[seg.tile];
        const int *list = cnt <= out.list_cap ? out.tile_lists + (size_t)seg.tile * out.list_cap : nullptr;
        const unsigned *queue = out.queue;
        const double U = (list && out.tile_U) ? out.tile_U[seg.tile] : INFINITY;
        recheck_segment<D, S>(g, sd, seg.start, seg.count, list, cnt, [&](unsigned q) { return queue[q]; },
                              out.labels, out.mom, sm[wave], out.rel_gap, sc->wmax, U);
    }
}

// -------------------------------------------------------- k_finalize

// Every cell's term of eq. (2.7) (dev::cell_final) and its relative volume
// error, over blocks of cells; the terms are summed in a fixed order
// (per block, then over blocks), so the objective is deterministic.
template <int D>
__global__ __launch_bounds__(kRedThreads) void k_finalize(Geo g, Seeds sd, const uint64_t *mom,
                                                          Scalars *sc, FinalOut out, BlockParts *bp) {
    constexpr int K = moments_per_cell(D);
    __shared__ double s_g[kRedWaves];
    __shared__ double s_m[kRedWaves];
    const int tid = threadIdx.x;
    int i0, i1;
    block_range(g.n, &i0, &i1);
    double gs = 0.0, mr = 0.0;
    for (int i = i0 + tid; i < i1; i += kRedThreads) {
        double gi, rel, ybar[3];
        gs += dev::cell_final<D>(g, sd, mom + (size_t)i * K, i, &gi, &rel, ybar);
        mr = fmax(mr, rel);
        if (out.grad) out.grad[i] = gi;
        if (out.counts) out.counts[i] = (int64_t)mom[(size_t)i * K];
        if (out.centroids)
            for (int d = 0; d < D; ++d) out.centroids[(size_t)i * D + d] = ybar[d];
    }
    // block reduction as in k_prep
    auto reduce = [&](double a, double m) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            a = a + __shfl_xor(a, o);
            m = fmax(m, __shfl_xor(m, o));
        }
        __syncthreads();
        if (__lane_id() == 0) {
            s_g[tid >> 6] = a;
            s_m[tid >> 6] = m;
        }
        __syncthreads();
        if (tid == 0)
            for (int k = 1; k < kRedWaves; ++k) {
                s_g[0] = s_g[0] + s_g[k];
                s_m[0] = fmax(s_m[0], s_m[k]);
            }
    };
    reduce(gs, mr);
    if (tid == 0) {
        bp->a[blockIdx.x] = s_g[0];
        bp->b[blockIdx.x] = s_m[0];
    }
    // this block's host writes (the gradient) reach the host before the
    // last block publishes the pass
    if (out.host_sc) __threadfence_system();
    if (!last_block(&bp->ticket)) return;
    const bool have = tid < (int)gridDim.x;
    reduce(have ? bp->a[tid] : 0.0, have ? bp->b[tid] : 0.0);
    if (tid == 0) {
        sc->g = g.power != 2 ? s_g[0] + g.munit * sc->gpix : s_g[0];
        sc->maxrel = s_m[0];
        bp->ticket = 0u;
        if (out.host_sc) {
            // every kernel of the pass before this one has finished; the
            // host waits for seq, so it goes last
            Scalars *h = out.host_sc;
            h->wmax = sc->wmax;
            h->vsum = sc->vsum;
            h->g = sc->g;
            h->maxrel = sc->maxrel;
            h->qcount = sc->qcount;
            h->segcount = sc->segcount;
            h->lam = sc->lam;
            h->bad = sc->bad;
            h->qtotal = sc->qtotal;
            h->credited = sc->credited;
            __threadfence_system();
            const unsigned n = ++bp->published;
            __hip_atomic_store(&out.host_sc->seq, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}


template <int D, int P = kP>
dim3 tile_grid(const Geo &g) {
    constexpr int E0 = tile_ext(D, P, 0), E1 = tile_ext(D, P, 1), E2 = tile_ext(D, P, 2);
    if (D == 2) return dim3((g.grid[1] + E1 - 1) / E1, (g.grid[0] + E0 - 1) / E0, 1);
    return dim3((g.grid[2] + E2 - 1) / E2, (g.grid[1] + E1 - 1) / E1, (g.grid[0] + E0 - 1) / E0);
}

// 8 pixels per lane halve the per-seed work of the lanes but give 2048-pixel
// tiles; below 1024 such tiles (4 waves per SIMD on 256 CUs) the 4-pixel
// form keeps the chip full.
template <int D, bool CULL>
hipError_t launch_vec(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                      const PassOut &out, hipStream_t st) {
    if (vec_pixels_per_lane(g, CULL) == 8)
        k_assign_vec<D, CULL, 8><<<tile_grid<D, 8>(g), kThreads, 0, st>>>(g, sd, sc, eig, out);
    else
        k_assign_vec<D, CULL, 4><<<tile_grid<D, 4>(g), kThreads, 0, st>>>(g, sd, sc, eig, out);
    return hipGetLastError();
}

}  // namespace

int vec_pixels_per_lane(const Geo &g, bool cull) {
    if (g.vec_p == 4 || g.vec_p == 8) return g.vec_p;
    // measured: with candidate lists the smaller wave boxes of 4 rows win
    // (fewer candidates per wave); over every seed, 8 rows halve the
    // per-seed work of a lane once the grid keeps the chip busy
    if (cull) return 4;
    int64_t J = 1;
    for (int d = 0; d < g.dim; ++d) J *= g.grid[d];
    return J >= 1024 * 2048 ? 8 : 4;
}

hipError_t launch_prep(const Geo &g, const Seeds &sd, Scalars *sc, uint64_t *mom, double *eig,
                       BlockParts *bp, hipStream_t st, const double *w_src) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    const int nb = red_blocks(g.n);
    if (g.dim == 2) k_prep<2><<<nb, kRedThreads, 0, st>>>(g, sd, sc, mom, eig, bp, w_src);
    else k_prep<3><<<nb, kRedThreads, 0, st>>>(g, sd, sc, mom, eig, bp, w_src);
    return hipGetLastError();
}

int64_t fp64_blocks(const Geo &g) {
    const dim3 b = g.dim == 2 ? tile_grid<2>(g) : tile_grid<3>(g);
    return (int64_t)b.x * b.y * b.z;
}

hipError_t launch_assign_fp64(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 2) k_assign_fp64<2><<<tile_grid<2>(g), kThreads, 0, st>>>(g, sd, sc, out);
    else k_assign_fp64<3><<<tile_grid<3>(g), kThreads, 0, st>>>(g, sd, sc, out);
    if (out.cost_part) k_sum_parts<<<1, 256, 0, st>>>(out.cost_part, fp64_blocks(g), sc);
    return hipGetLastError();
}

hipError_t launch_assign_fp32(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                              hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    return g.dim == 2 ? launch_vec<2, false>(g, sd, sc, nullptr, out, st)
                      : launch_vec<3, false>(g, sd, sc, nullptr, out, st);
}

hipError_t launch_super_cull(const Geo &g, const Seeds &sd, const Scalars *sc, const double *eig,
                             const PassOut &out, int *list, int *count, hipStream_t st) {
    (void)hipGetLastError();
    const int nb = out.nst[0] * out.nst[1] * out.nst[2];
    if (g.dim == 2) k_super_cull<2><<<nb, kThreads, 0, st>>>(g, sd, sc, eig, out, list, count);
    else k_super_cull<3><<<nb, kThreads, 0, st>>>(g, sd, sc, eig, out, list, count);
    return hipGetLastError();
}

hipError_t launch_assign_cull(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                              const PassOut &out, hipStream_t st) {
    (void)hipGetLastError();
    return g.dim == 2 ? launch_vec<2, true>(g, sd, sc, eig, out, st)
                      : launch_vec<3, true>(g, sd, sc, eig, out, st);
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

hipError_t launch_assign_hyb(const Geo &g, const Seeds &sd, Scalars *sc, const PassOut &out,
                             hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (g.dim == 3) {
        dim3 grid((g.grid[2] + 7) / 8, (g.grid[1] + 15) / 16, (g.grid[0] + kHybRows3 - 1) / kHybRows3);
        k_assign_hyb<3><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    } else {
        dim3 grid((g.grid[1] + 31) / 32, (g.grid[0] + kHybRows2 - 1) / kHybRows2);
        k_assign_hyb<2><<<grid, kThreads, 0, st>>>(g, sd, sc, out);
    }
    return hipGetLastError();
}

hipError_t launch_seed_order(const Geo &g, const Seeds &sd, int *ord, hipStream_t st) {
    (void)hipGetLastError();
    if (g.dim == 3) k_seed_order<3><<<1, kOrderThreads, 0, st>>>(g, sd, ord);
    else k_seed_order<2><<<1, kOrderThreads, 0, st>>>(g, sd, ord);
    return hipGetLastError();
}

// Seeds per staged chunk of the bf16 tile: 1024 in 2D over every seed
// (N = 1000 is one chunk), 256 in 3D or with candidate lists.
template <int D, int P, bool CULL>
static void launch_bf16(const Geo &g, Seeds sd, Scalars *sc, const double *eig, const PassOut &out,
                        hipStream_t st) {
    constexpr int C = (D == 2 && !CULL) ? 1024 : 256;
    k_assign_bf16<D, P, C, CULL><<<tile_grid<D, P>(g), kThreads, 0, st>>>(g, sd, sc, eig, out);
}

template <int D, bool CULL>
static void launch_bf16_rows(const Geo &g, Seeds sd, Scalars *sc, const double *eig, const PassOut &out,
                             hipStream_t st) {
    if (bf16_pixels_per_lane(g) == 4) launch_bf16<D, 4, CULL>(g, sd, sc, eig, out, st);
    else launch_bf16<D, 2, CULL>(g, sd, sc, eig, out, st);
}

// Pixel rows per lane of the bf16 tile: 4 in 2D and 2 in 3D (where the
// tile's two matrix-core operands per block take twice the registers), or
// half the pixels per lane set for the vector kernel (4 or 8).
int bf16_pixels_per_lane(const Geo &g) {
    if (g.vec_p == 4 || g.vec_p == 8) return g.vec_p / 2;
    return g.dim == 2 ? 4 : 2;
}

hipError_t launch_assign_bf16(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                              const PassOut &out, hipStream_t st) {
    (void)hipGetLastError();
    const bool cull = eig != nullptr;
    if (g.dim == 2) {
        if (cull) launch_bf16_rows<2, true>(g, sd, sc, eig, out, st);
        else launch_bf16_rows<2, false>(g, sd, sc, eig, out, st);
    } else {
        if (cull) launch_bf16_rows<3, true>(g, sd, sc, eig, out, st);
        else launch_bf16_rows<3, false>(g, sd, sc, eig, out, st);
    }
    return hipGetLastError();
}

hipError_t launch_recheck(const Geo &g, const Seeds &sd, const Scalars *sc, const PassOut &out,
                          hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    // a scan over every seed: stage the seeds in LDS (three blocks of 48 KB
    // or four of 40 KB per compute unit)
    if (!out.tile_lists) {
        if (g.dim == 2) k_recheck_staged<2><<<768, kThreads, 0, st>>>(g, sd, sc, out);
        else k_recheck_staged<3><<<1024, kThreads, 0, st>>>(g, sd, sc, out);
        return hipGetLastError();
    }
    // with the tiles' candidate lists: one wave per segment (a tile's
    // queued pixels), as many as fit on the chip (a segment is a short chain
    // of dependent loads, so concurrency sets the speed); waves past the
    // segments leave at once
    const int64_t tiles = (int64_t)out.ntile[0] * out.ntile[1] * out.ntile[2];
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + kWaves - 1) / kWaves, 2048));
    if (g.dim == 2) k_recheck_seg<2><<<nb, kThreads, 0, st>>>(g, sd, sc, out);
    else k_recheck_seg<3><<<nb, kThreads, 0, st>>>(g, sd, sc, out);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    (void)hipGetLastError();
    const size_t n = bytes / 4;
    const unsigned nb = (unsigned)std::min<size_t>(256, (n + 255) / 256);
    if (n) k_zero_words<<<nb, 256, 0, st>>>(static_cast<unsigned *>(p), n);
    return hipGetLastError();
}

hipError_t launch_mass_total(const Geo &g, Scalars *sc, hipStream_t st) {
    (void)hipGetLastError();
    int64_t J = 1;
    for (int d = 0; d < g.dim; ++d) J *= g.grid[d];
    const unsigned nb = (unsigned)std::min<int64_t>(1024, (J + 255) / 256);
    k_mass_total<<<nb, 256, 0, st>>>(J, g.mass, sc);
    return hipGetLastError();
}

hipError_t launch_finalize(const Geo &g, const Seeds &sd, const uint64_t *mom, Scalars *sc,
                           const FinalOut &out, BlockParts *bp, hipStream_t st) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    const int nb = red_blocks(g.n);
    if (g.dim == 2) k_finalize<2><<<nb, kRedThreads, 0, st>>>(g, sd, mom, sc, out, bp);
    else k_finalize<3><<<nb, kRedThreads, 0, st>>>(g, sd, mom, sc, out, bp);
    return hipGetLastError();
}

}  // namespace apd
