// apd_batch.hip -- many independent APD fits at once (Algorithm 2 of
// arXiv 2403.03571 for a batch of problems of uneven N and grid size).
//
// Every evaluation of every active instance is one replay of a captured
// HIP graph of five kernels:
//   kb_prep      block per instance: gauge max of the trial weights, zeroed
//                moments; block 0 resets the work counters.
//   kb_assign    persistent: blocks pull (instance, tile) work items from an
//                atomic counter over the concatenated tile lists (largest
//                instances first) and run the matrix-core tile of the
//                single-instance path on it; converged instances are skipped.
//   kb_recheck   persistent over one queue of (instance, pixel) entries:
//                the double re-check of near-tie pixels.
//   kb_finalize  block per instance: objective, gradient, max rel. error.
//   kb_lbfgs     block per instance: one step of the L-BFGS state machine
//                (the same specification as the host solver), which writes
//                the next trial weights or retires the instance.
// The host replays the graph and polls the number of active instances.
#include "../../include/apd.h"
#include "apd_batch.h"
#include "apd_device.h"

#include <math.h>

#include <algorithm>
#include <chrono>
#include <numeric>
#include <vector>

namespace apd {
namespace {

using namespace dev;

constexpr int kHist = 10;  // stored curvature pairs (the solver's memory)

// ------------------------------------------------------------ block helpers

__device__ inline double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kWaves; ++k) t += red[k];  // same order in every thread
    return t;
}

__device__ inline double block_max(double v, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (__lane_id() == 0) red[w] = v;
    __syncthreads();
    double t = red[0];
    for (int k = 1; k < kWaves; ++k) t = fmax(t, red[k]);
    return t;
}

// --------------------------------------------------------------- kb_setup

// Validation and the Gershgorin bound, once per batch.
template <int D>
__global__ __launch_bounds__(kThreads) void kb_setup(BInst *inst, BState *st) {
    __shared__ double red[kWaves];
    const int b = blockIdx.x;
    const BInst &I = inst[b];
    const int n = I.g.n;
    double lam = 0.0, vs = 0.0, kap = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += kThreads) {
        for (int d = 0; d < D; ++d)
            if (!isfinite(I.x[(size_t)i * D + d])) bad |= kBadX;
        const double *a = I.A + (size_t)i * D * D;
        double u[3][3];
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                u[r][c] = (r <= c) ? a[r * D + c] : a[c * D + r];
                if (!isfinite(u[r][c])) bad |= kBadA;
            }
        double det = u[0][0] * u[1][1] - u[0][1] * u[0][1];
        bool spd = u[0][0] > 0.0 && det > 0.0;
        if (D == 3) {
            det = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[1][2]) -
                  u[0][1] * (u[0][1] * u[2][2] - u[1][2] * u[0][2]) +
                  u[0][2] * (u[0][1] * u[1][2] - u[1][1] * u[0][2]);
            spd = spd && det > 0.0;
        }
        if (!spd) bad |= kBadSPD;
        double lg = 0.0;
        for (int r = 0; r < D; ++r) {
            double rs = 0.0;
            for (int c = 0; c < D; ++c) rs += fabs(u[r][c]);
            lg = fmax(lg, rs);
        }
        lam = fmax(lam, lg);
        if (spd) kap = fmax(kap, cond_bound(D, lg, det));
        double elo, ehi;
        eig_range<D>(u, &elo, &ehi);
        I.eig[2 * (size_t)i] = elo;
        I.eig[2 * (size_t)i + 1] = ehi;
        const double vi = I.v[i];
        if (!(vi > 0.0) || !isfinite(vi)) bad |= kBadV;
        vs += vi;
        if (!isfinite(I.wt[i])) bad |= kBadW;
    }
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    lam = block_max(lam, red);
    kap = block_max(kap, red);
    vs = block_sum(vs, red);
    if (bad) atomicOr(&s_bad, bad);
    __syncthreads();
    const int bits = s_bad;
    if (threadIdx.x == 0) {
        st[b].lam = (float)(lam * 1.0001);
        st[b].kap = (float)(kap * 1.0001);
        st[b].vsum = vs;
        st[b].bad = bits;
    }
}

// ---------------------------------------------------------------- kb_prep

template <int D>
__global__ __launch_bounds__(kThreads) void kb_prep(BInst *inst, BState *st, BCtl *ctl) {
    __shared__ double red[kWaves];
    constexpr int K = moments_per_cell(D);
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0) {
        ctl->next = 0u;
        ctl->qcount = 0u;
        ctl->segcount = 0u;
    }
    if (!st[b].active) return;
    const BInst &I = inst[b];
    const int n = I.g.n;
    for (int t = threadIdx.x; t < n * K; t += kThreads) I.mom[t] = 0ull;
    double wm = -INFINITY;
    for (int i = threadIdx.x; i < n; i += kThreads) wm = fmax(wm, I.wt[i]);
    wm = block_max(wm, red);
    if (threadIdx.x == 0) st[b].wmax = wm;
}

// -------------------------------------------------------------- kb_assign

__device__ inline int find_instance(const int64_t *tile0, int B, int64_t item) {
    int lo = 0, hi = B;  // tile0[lo] <= item < tile0[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile0[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One block per (instance, super-tile): the super-tile candidate lists of
// the active instances (dev::super_tile_list).
template <int D>
__global__ __launch_bounds__(kThreads) void kb_super(const BInst *inst, const BState *st,
                                                    const int64_t *super0, int B) {
    __shared__ int s_cnt;
    __shared__ double s_red[kWaves];
    const int64_t item = blockIdx.x;
    const int b = find_instance(super0, B, item);
    if (!st[b].active) return;
    const BInst &I = inst[b];
    const int local = (int)(item - super0[b]);
    Seeds sd{I.x, I.A, I.wt, I.v};
    PassOut out{nullptr, nullptr, nullptr};
    out.tp = I.tp;
    for (int d = 0; d < 3; ++d) {
        out.sf[d] = I.sf[d];
        out.nst[d] = I.nst[d];
    }
    super_tile_list<D>(I.g, sd, st[b].wmax, I.eig, out, local, I.super_lists + (size_t)local * kBatchSuperCap,
                       I.super_count + local, kBatchSuperCap, s_cnt, s_red);
}

// V: 0 fp32 matrix cores, 1 fp32 vector, 2 fp32 vector with candidate
// lists (8 pixels per lane), 3 bf16 matrix cores, 4 fp32 vector with
// candidate lists (4 pixels per lane), 5 bf16 matrix cores with candidate
// lists (both bf16 forms with Bf16Rows<D> pixel rows per lane; at two
// waves per SIMD the 2D form spills a few registers, and still runs the
// batched C4-type solve 1.5 times faster than at one wave -- measured)
template <int D, int V>
__global__ __launch_bounds__(kThreads, (D == 2 && V != 3 && V != 5) ? 4 : 2) void kb_assign(const BInst *inst, const BState *st,
                                                     const int64_t *tile0, int B, BCtl *ctl,
                                                     uint64_t *queue, QSeg *segs) {
    __shared__ union {
        float mf[kMfmaLds];
        VecSmem<D, V == 2 || V == 4> vec;
        Bf16Smem<D, 256, V == 5> bf;
    } sm;
    float *sC = sm.mf;
    __shared__ int64_t s_item;
    const int64_t total = tile0[B];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int64_t item = s_item;
        if (item >= total) break;
        const int b = find_instance(tile0, B, item);
        if (!st[b].active) continue;
        const BInst &I = inst[b];
        const int64_t local = item - tile0[b];
        Seeds sd{I.x, I.A, I.wt, I.v};
        PassOut out{nullptr, I.mom, nullptr};
        out.queue64 = queue;
        out.tag = (uint32_t)b;
        out.segs = segs;
        out.tile_id = (int)local;
        int b0, b1, b2 = 0;
        if (D == 2) {
            b0 = (int)(local / I.tiles1);
            b1 = (int)(local % I.tiles1);
        } else {
            const int per0 = I.tiles1 * I.tiles2;
            b0 = (int)(local / per0);
            const int r = (int)(local % per0);
            b1 = r / I.tiles2;
            b2 = r % I.tiles2;
        }
        if (V == 0) {
            mfma_tile<D>(I.g, sd, st[b].wmax, Cert{st[b].lam, st[b].kap}, b0, b1, b2, sC, out, &ctl->qcount);
        } else {
            constexpr bool kLists = V == 2 || V == 4 || V == 5;
            if (kLists && I.tile_lists) {
                out.tile_lists = I.tile_lists;
                out.tile_count = I.tile_count;
                out.list_cap = kBatchListCap;
                out.tp = I.tp;
                out.ntile[0] = I.tiles0;
                out.ntile[1] = I.tiles1;
                out.ntile[2] = I.tiles2;
                out.adaptive = true;  // single-candidate tiles credited whole
            }
            if (kLists && I.super_lists) {
                out.super_list = I.super_lists;
                out.super_count = I.super_count;
                out.super_cap = kBatchSuperCap;
                for (int d = 0; d < 3; ++d) {
                    out.sf[d] = I.sf[d];
                    out.nst[d] = I.nst[d];
                }
            }
            if constexpr (V == 3 || V == 5)
                bf16_tile<D, Bf16Rows<D>::value, 256, V == 5>(I.g, sd, st[b].wmax, Cert{st[b].lam, st[b].kap}, I.eig, b0, b1, b2,
                                                              sm.bf, out, &ctl->qcount);
            else
                vec_tile<D, kLists, V == 4 ? kP : kPv>(I.g, sd, st[b].wmax, Cert{st[b].lam, st[b].kap}, I.eig, b0, b1, b2,
                                                       sm.vec, out, &ctl->qcount);
        }
    }
}

// ------------------------------------------------------------- kb_recheck

template <int D>
__global__ __launch_bounds__(kThreads) void kb_recheck(const BInst *inst, const BCtl *ctl,
                                                      const uint64_t *queue, const QSeg *segs) {
    constexpr int S = 128;  // seeds per staged chunk, per wave
    __shared__ StagedSeeds<D, S> sm[kWaves];
    const unsigned nseg = ctl->segcount;
    const int wave = threadIdx.x >> 6;
    for (unsigned s = blockIdx.x * kWaves + wave; s < nseg; s += gridDim.x * kWaves) {
        // one tile's queued pixels against its candidate list (or every
        // seed of the instance: no lists, or an overflowed one), one wave
        const QSeg seg = segs[s];
        const BInst &I = inst[seg.tag];
        Seeds sd{I.x, I.A, I.wt, I.v};
        const int *list = nullptr;
        int cnt = 0;
        if (I.tile_lists) {
            cnt = I.tile_count[seg.tile];
            if (cnt <= kBatchListCap) list = I.tile_lists + (size_t)seg.tile * kBatchListCap;
        }
        recheck_segment<D, S>(I.g, sd, seg.start, seg.count, list, cnt,
                              [&](unsigned q) { return (uint32_t)queue[q]; }, nullptr, I.mom, sm[wave]);
    }
}

// ------------------------------------------------------------ kb_finalize

// f = -g~ and grad f = m|P| - v at the trial weights (into gt).
template <int D>
__global__ __launch_bounds__(kThreads) void kb_finalize(const BInst *inst, BState *st) {
    __shared__ double red[kWaves];
    constexpr int K = moments_per_cell(D);
    const int b = blockIdx.x;
    if (!st[b].active) return;
    const BInst &I = inst[b];
    const int n = I.g.n;
    Seeds sd{I.x, I.A, I.wt, I.v};
    double gs = 0.0, mr = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) {
        double gi, rel, ybar[3];
        gs += cell_final<D>(I.g, sd, I.mom + (size_t)i * K, i, &gi, &rel, ybar);
        mr = fmax(mr, rel);
        I.gt[i] = -gi;
    }
    gs = block_sum(gs, red);
    mr = block_max(mr, red);
    if (threadIdx.x == 0) {
        st[b].ftrial = -gs;
        st[b].crit_trial = mr;
    }
}

// --------------------------------------------------------------- kb_lbfgs

__device__ inline double project(double *v, int n, double *red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += v[i];
    s = block_sum(s, red) / (double)n;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kThreads) v[i] -= s;
    __syncthreads();
    return s;
}

__device__ inline double dot(const double *a, const double *b, int n, double *red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += a[i] * b[i];
    return block_sum(s, red);
}

// One step of the solver for instance blockIdx.x, after the evaluation at
// its trial point wt.  Specification (shared with the host solver): stop as
// soon as an evaluation meets max rel. error < eps; gradients projected on
// sum = 0; d by the two-loop recursion over at most kHist pairs with
// H0 = (s.y/y.y) I of the newest pair, or -gamma0 grad without pairs; Armijo
// (c1 = 1e-4) from the unit step, halving up to 30 times; pairs kept when
// s.y > 1e-10 |s||y|; a non-descent direction or a failed search clears the
// pairs and retries with the steepest step, whose own failure ends the solve.
__global__ __launch_bounds__(kThreads) void kb_lbfgs(const BInst *inst, BState *st, BCtl *ctl) {
    __shared__ double red[kWaves];
    __shared__ double alph[kHist];
    const int b = blockIdx.x;
    BState S = st[b];
    if (!S.active) return;
    const BInst &I = inst[b];
    const int n = I.g.n;
    double *w = I.w, *g = I.g_acc, *d = I.d, *wt = I.wt, *gt = I.gt;
    double *Sm = I.S, *Ym = I.Y, *rho = I.rho;
    const double eps = ctl->eps;
    S.evals += 1;
    const double ft = S.ftrial, critt = S.crit_trial;
    bool need_dir = false;
    int result = -1;  // -1: still running, else an apd_status

    auto copy_wt_to_w = [&]() {
        for (int i = threadIdx.x; i < n; i += kThreads) w[i] = wt[i];
        __syncthreads();
    };

    if (S.phase == 0) {  // the first evaluation, at w0
        S.f = ft;
        S.crit = critt;
        copy_wt_to_w();
        if (critt < eps) {
            result = APD_OK;
        } else {
            for (int i = threadIdx.x; i < n; i += kThreads) g[i] = gt[i];
            __syncthreads();
            project(g, n, red);
            need_dir = true;
        }
    } else if (critt < eps) {
        copy_wt_to_w();
        S.f = ft;
        S.crit = critt;
        S.iters += 1;
        result = APD_OK;
    } else if (ft <= S.f + 1e-4 * S.alpha * S.gd) {
        // accepted: curvature pair, then the new iterate
        project(gt, n, red);
        double sy = 0.0, ss = 0.0, yy = 0.0;
        for (int i = threadIdx.x; i < n; i += kThreads) {
            const double si = wt[i] - w[i], yi = gt[i] - g[i];
            sy += si * yi;
            ss += si * si;
            yy += yi * yi;
        }
        sy = block_sum(sy, red);
        ss = block_sum(ss, red);
        yy = block_sum(yy, red);
        if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
            int slot;
            if (S.npairs < kHist) {
                slot = (S.head + S.npairs) % kHist;
                S.npairs += 1;
            } else {
                slot = S.head;
                S.head = (S.head + 1) % kHist;
            }
            for (int i = threadIdx.x; i < n; i += kThreads) {
                Sm[(size_t)slot * n + i] = wt[i] - w[i];
                Ym[(size_t)slot * n + i] = gt[i] - g[i];
            }
            if (threadIdx.x == 0) rho[slot] = 1.0 / sy;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < n; i += kThreads) {
            w[i] = wt[i];
            g[i] = gt[i];
        }
        __syncthreads();
        S.f = ft;
        S.crit = critt;
        S.iters += 1;
        need_dir = true;
    } else {
        if (S.evals >= ctl->max_evals) {
            result = APD_ERR_NOT_CONVERGED;
        } else if (S.t + 1 < 30) {
            S.t += 1;
            S.alpha *= 0.5;
            for (int i = threadIdx.x; i < n; i += kThreads) wt[i] = w[i] + S.alpha * d[i];
        } else if (S.npairs > 0) {
            S.npairs = 0;
            S.head = 0;
            need_dir = true;
        } else {
            result = APD_ERR_LINESEARCH;
        }
    }

    if (need_dir) {
        if (S.iters >= ctl->max_iter || S.evals >= ctl->max_evals) {
            result = APD_ERR_NOT_CONVERGED;
        } else {
            for (int attempt = 0; attempt < 2; ++attempt) {
                if (S.npairs == 0) {
                    for (int i = threadIdx.x; i < n; i += kThreads) d[i] = -S.gamma0 * g[i];
                    __syncthreads();
                } else {
                    for (int i = threadIdx.x; i < n; i += kThreads) d[i] = g[i];
                    __syncthreads();
                    for (int k = S.npairs - 1; k >= 0; --k) {
                        const int sl = (S.head + k) % kHist;
                        const double a = rho[sl] * dot(Sm + (size_t)sl * n, d, n, red);
                        if (threadIdx.x == 0) alph[k] = a;
                        for (int i = threadIdx.x; i < n; i += kThreads) d[i] -= a * Ym[(size_t)sl * n + i];
                        __syncthreads();
                    }
                    const int nl = (S.head + S.npairs - 1) % kHist;
                    const double gam = dot(Sm + (size_t)nl * n, Ym + (size_t)nl * n, n, red) /
                                       dot(Ym + (size_t)nl * n, Ym + (size_t)nl * n, n, red);
                    for (int i = threadIdx.x; i < n; i += kThreads) d[i] *= gam;
                    __syncthreads();
                    for (int k = 0; k < S.npairs; ++k) {
                        const int sl = (S.head + k) % kHist;
                        const double beta = rho[sl] * dot(Ym + (size_t)sl * n, d, n, red);
                        const double a = alph[k];
                        for (int i = threadIdx.x; i < n; i += kThreads) d[i] += Sm[(size_t)sl * n + i] * (a - beta);
                        __syncthreads();
                    }
                    for (int i = threadIdx.x; i < n; i += kThreads) d[i] = -d[i];
                    __syncthreads();
                }
                const double gd = dot(g, d, n, red);
                if (gd < 0.0) {
                    S.gd = gd;
                    S.alpha = 1.0;
                    S.t = 0;
                    S.phase = 1;
                    for (int i = threadIdx.x; i < n; i += kThreads) wt[i] = w[i] + d[i];
                    break;
                }
                if (S.npairs > 0) {
                    S.npairs = 0;
                    S.head = 0;
                    continue;
                }
                result = APD_ERR_LINESEARCH;
                break;
            }
        }
    }
    if (result >= 0) {
        S.active = 0;
        S.status = result;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st[b] = S;
        if (result >= 0) atomicSub(&ctl->active, 1);
    }
}

// the first trial point: the caller's weights or zeros
__global__ __launch_bounds__(kThreads) void kb_init(const BInst *inst, const double *const *src,
                                                   int warm) {
    const int b = blockIdx.x;
    const BInst &I = inst[b];
    for (int i = threadIdx.x; i < I.g.n; i += kThreads) I.wt[i] = warm ? src[b][i] : 0.0;
}

// write the accepted iterate back to the caller's arrays
__global__ __launch_bounds__(kThreads) void kb_scatter(const BInst *inst, double *const *dst) {
    const int b = blockIdx.x;
    const BInst &I = inst[b];
    for (int i = threadIdx.x; i < I.g.n; i += kThreads) dst[b][i] = I.w[i];
}

}  // namespace

hipError_t launch_batch_setup(int dim, BInst *inst, BState *st, int B, hipStream_t s) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (dim == 2) kb_setup<2><<<B, kThreads, 0, s>>>(inst, st);
    else kb_setup<3><<<B, kThreads, 0, s>>>(inst, st);
    return hipGetLastError();
}

template <int D>
void batch_assign(int variant, dim3 grid, BInst *inst, BState *st, const int64_t *tile0, int B,
                  BCtl *ctl, uint64_t *queue, QSeg *segs, hipStream_t s) {
    switch (variant) {
    case 0: kb_assign<D, 0><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    case 1: kb_assign<D, 1><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    case 2: kb_assign<D, 2><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    case 4: kb_assign<D, 4><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    case 5: kb_assign<D, 5><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    default: kb_assign<D, 3><<<grid, kThreads, 0, s>>>(inst, st, tile0, B, ctl, queue, segs); break;
    }
}

hipError_t launch_batch_step(int dim, BInst *inst, BState *st, const int64_t *tile0, int B,
                             BCtl *ctl, uint64_t *queue, QSeg *segs, int grid_assign, int variant,
                             int recheck_blocks, const int64_t *super0, int64_t nsuper, hipStream_t s) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    if (dim == 2) {
        kb_prep<2><<<B, kThreads, 0, s>>>(inst, st, ctl);
        if (nsuper > 0) kb_super<2><<<(unsigned)nsuper, kThreads, 0, s>>>(inst, st, super0, B);
        batch_assign<2>(variant, grid_assign, inst, st, tile0, B, ctl, queue, segs, s);
        kb_recheck<2><<<recheck_blocks, kThreads, 0, s>>>(inst, ctl, queue, segs);
        kb_finalize<2><<<B, kThreads, 0, s>>>(inst, st);
    } else {
        kb_prep<3><<<B, kThreads, 0, s>>>(inst, st, ctl);
        if (nsuper > 0) kb_super<3><<<(unsigned)nsuper, kThreads, 0, s>>>(inst, st, super0, B);
        batch_assign<3>(variant, grid_assign, inst, st, tile0, B, ctl, queue, segs, s);
        kb_recheck<3><<<recheck_blocks, kThreads, 0, s>>>(inst, ctl, queue, segs);
        kb_finalize<3><<<B, kThreads, 0, s>>>(inst, st);
    }
    kb_lbfgs<<<B, kThreads, 0, s>>>(inst, st, ctl);
    return hipGetLastError();
}

hipError_t launch_batch_init(BInst *inst, double *const *src, int B, bool warm, hipStream_t s) {
    (void)hipGetLastError();
    kb_init<<<B, kThreads, 0, s>>>(inst, src, warm ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_batch_scatter(BInst *inst, double *const *dst, int B, hipStream_t s) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    kb_scatter<<<B, kThreads, 0, s>>>(inst, dst);
    return hipGetLastError();
}

}  // namespace apd
