// apd_ws.hip -- the learned warm start: a per-seed network that predicts the
// initial weights of Algorithm 2 (arXiv 2403.03571 starts from W_0 = 0).
//
// Features (2D), per seed i: its own (x_i, upper triangle of A_i, N v_i),
// the mean over its 16 nearest seeds (Euclidean, ties to the lower index)
// of (sqrt(N)(x_j - x_i), upper triangle of A_j, N v_j, N |x_j - x_i|^2_{A_i},
// N |x_j - x_i|^2_{A_j}), its distance to the box boundary along each axis
// scaled by sqrt(N / |Omega|), the volume deficit d_i = N (v_i - |C_i|) of
// its cell at W = 0 (the gradient (2.8) of one pass at zero weights), and the
// 1-, 2- and 3-fold repeated 16-neighbour means of d: 20 numbers.  The
// optimal weights respond to the deficit like the inverse of a graph
// Laplacian, which the repeated means reach beyond the nearest seeds.
// Network: 20 -> 128 -> 128 -> 128 -> 1, ReLU between layers, parameters
// one flat FP32 vector (per layer W [in][out] row-major, then b).
// Training: mean squared error against t_i = N (w*_i - mean w*), Adam.
// Prediction: w_i = (y_i - mean y) / N.
#include "../../include/apd.h"
#include "apd_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <string>

namespace apd {
namespace ws {

constexpr int kFeat = 20;
constexpr int kPoolHops = 3;
constexpr int kHid = 128;
constexpr int kNeigh = 16;
constexpr int64_t kParams = (int64_t)kFeat * kHid + kHid + 2 * ((int64_t)kHid * kHid + kHid) + kHid + 1;

const int64_t kParamCount = kParams;

// offsets of the layers in the flat vector
constexpr int64_t oW1 = 0, ob1 = oW1 + kFeat * kHid;
constexpr int64_t oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid;
constexpr int64_t oW3 = ob2 + kHid, ob3 = oW3 + kHid * kHid;
constexpr int64_t oW4 = ob3 + kHid, ob4 = oW4 + kHid;

namespace {

// ------------------------------------------------------------- features

// One wave per seed.  The 16 nearest seeds are found in 16 rounds: each
// round every lane scans its share of the seeds for the smallest
// (distance^2, index) pair above the previous round's, and a wave minimum
// picks the next neighbour (ties go to the lower index).
__global__ __launch_bounds__(256) void kw_features(int n, const double *__restrict__ x,
                                                   const double *__restrict__ A,
                                                   const double *__restrict__ v, double lo0,
                                                   double lo1, double hi0, double hi1, float *F,
                                                   int *nb) {
    const int lane = __lane_id();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;  // whole waves leave together
    const double xi0 = x[2 * i], xi1 = x[2 * i + 1];
    const int k = min(kNeigh, n - 1);
    double pd = -1.0;
    int pj = -1;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double N = (double)n;
    const double *ai = A + 4 * i;
    for (int round = 0; round < k; ++round) {
        double bd = INFINITY;
        int bj = 0x7fffffff;
        for (int j = lane; j < n; j += 64) {
            if (j == i) continue;
            const double d0 = xi0 - x[2 * j], d1 = xi1 - x[2 * j + 1];
            const double d2 = d0 * d0 + d1 * d1;
            const bool after = d2 > pd || (d2 == pd && j > pj);
            if (after && (d2 < bd || (d2 == bd && j < bj))) {
                bd = d2;
                bj = j;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double od = __shfl_xor(bd, o);
            const int oj = __shfl_xor(bj, o);
            if (od < bd || (od == bd && oj < bj)) {
                bd = od;
                bj = oj;
            }
        }
        pd = bd;
        pj = bj;
        if (lane == 0) nb[(size_t)i * kNeigh + round] = bj;
        // accumulate the neighbour's terms (every lane holds the same values)
        const int j = bj;
        const double dx0 = x[2 * j] - xi0, dx1 = x[2 * j + 1] - xi1;
        const double *aj = A + 4 * j;
        s[0] += dx0;
        s[1] += dx1;
        s[2] += aj[0];
        s[3] += aj[1];
        s[4] += aj[3];
        s[5] += N * v[j];
        s[6] += N * (dx0 * (ai[0] * dx0 + ai[1] * dx1) + dx1 * (ai[1] * dx0 + ai[3] * dx1));
        s[7] += N * (dx0 * (aj[0] * dx0 + aj[1] * dx1) + dx1 * (aj[1] * dx0 + aj[3] * dx1));
    }
    if (lane != 0) return;
    const double area = (hi0 - lo0) * (hi1 - lo1);
    const double sc = sqrt(N / area);
    double f[kFeat];
    f[0] = xi0;
    f[1] = xi1;
    f[2] = ai[0];
    f[3] = ai[1];
    f[4] = ai[3];
    f[5] = N * v[i];
    for (int q = 6; q < 14; ++q) f[q] = 0.0;
    if (k > 0) {
        const double c = (double)k, rn = sqrt(N);
        f[6] = rn * s[0] / c;
        f[7] = rn * s[1] / c;
        for (int q = 2; q < 8; ++q) f[6 + q] = s[q] / c;
    }
    f[14] = sc * fmin(xi0 - lo0, hi0 - xi0);
    f[15] = sc * fmin(xi1 - lo1, hi1 - xi1);
    for (int q = 0; q < 16; ++q) F[(size_t)i * kFeat + q] = (float)f[q];
}

// d_i = N grad_i (the deficit at W = 0) into feature 16 and out.
__global__ __launch_bounds__(256) void kw_deficit(int n, const double *grad, double *out, float *F) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double d = (double)n * grad[i];
    out[i] = d;
    F[(size_t)i * kFeat + 16] = (float)d;
}

// out_i = mean of in over the 16 nearest seeds of i (in neighbour order),
// into feature col and out; zero for a lone seed.
__global__ __launch_bounds__(256) void kw_pool(int n, const int *nb, const double *in, double *out,
                                               float *F, int col) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int k = min(kNeigh, n - 1);
    double s = 0.0;
    for (int r = 0; r < k; ++r) s += in[nb[(size_t)i * kNeigh + r]];
    const double m = k > 0 ? s / (double)k : 0.0;
    out[i] = m;
    F[(size_t)i * kFeat + col] = (float)m;
}

// ------------------------------------------------------------------ GEMM

// C[m][n] = sum_k opA(m, k) opB(k, n) with opA(m, k) = TA ? A[k lda + m] :
// A[m lda + k] and opB(k, n) = TB ? B[n ldb + k] : B[k ldb + n], then the
// epilogue: 0 none, 1 + bias[n], 2 relu(. + bias[n]), 3 times (mask[m][n] > 0).
// 64 x 64 output tile per block, K in slices of 16 through LDS, each thread
// a 4 x 4 block of outputs (FP32 vector ALU; the network is small).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void kw_gemm(int M, int N, int K, const float *__restrict__ A,
                                               int lda, const float *__restrict__ B, int ldb,
                                               float *__restrict__ C, int ldc,
                                               const float *__restrict__ bias,
                                               const float *__restrict__ mask, int ldm) {
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = tid; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int m = m0 + mm, k = k0 + kk;
            float a = 0.0f;
            if (m < M && k < K) a = TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
            As[kk][mm] = a;
            const int n = n0 + mm;
            float b = 0.0f;
            if (n < N && k < K) b = TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
            Bs[kk][mm] = b;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = m0 + ty * 4 + r;
        if (m >= M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = n0 + tx * 4 + c;
            if (n >= N) continue;
            float val = acc[r][c];
            if (EPI == 1 || EPI == 2) val += bias[n];
            if (EPI == 2) val = fmaxf(val, 0.0f);
            if (EPI == 3) val = mask[(size_t)m * ldm + n] > 0.0f ? val : 0.0f;
            C[(size_t)m * ldc + n] = val;
        }
    }
}

// Weight (and bias) gradients of one layer, split over the samples: block
// (n tile, m tile, split) sums its slice of the samples of A^T B for a
// 64 x 64 tile into part[split][M][N] (A [K][lda] read transposed, B
// [K][ldb]); with BIAS the blocks of the first m tile also sum B's columns
// over the slice into bpart[split][N].  kw_reduce_parts then adds the
// splits in order, so the gradients are deterministic.  (One block per
// output tile left four blocks looping over every sample.)
template <bool BIAS>
__global__ __launch_bounds__(256) void kw_gemm_tn_part(int M, int N, int K, int kslice,
                                                       const float *__restrict__ A, int lda,
                                                       const float *__restrict__ B, int ldb,
                                                       float *__restrict__ part,
                                                       float *__restrict__ bpart) {
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int ka = blockIdx.z * kslice, kb = min(K, ka + kslice);
    const bool colsum = BIAS && blockIdx.y == 0;
    float acc[4][4] = {};
    float bsum = 0.0f;
    for (int k0 = ka; k0 < kb; k0 += 16) {
        for (int e = tid; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int m = m0 + mm, k = k0 + kk;
            As[kk][mm] = (m < M && k < kb) ? A[(size_t)k * lda + m] : 0.0f;
            const int n = n0 + mm;
            Bs[kk][mm] = (n < N && k < kb) ? B[(size_t)k * ldb + n] : 0.0f;
        }
        __syncthreads();
        if (colsum && tid < 64)
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) bsum += Bs[kk][tid];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = m0 + ty * 4 + r;
        if (m >= M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = n0 + tx * 4 + c;
            if (n < N) out[(size_t)m * N + n] = acc[r][c];
        }
    }
    if (colsum && tid < 64 && n0 + tid < N) bpart[(size_t)blockIdx.z * N + n0 + tid] = bsum;
}

// out[i] = sum over s < nsplit of part[s count + i], in order of s
__global__ __launch_bounds__(256) void kw_reduce_parts(int count, int nsplit, const float *part,
                                                       float *out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    float v = 0.0f;
    for (int q = 0; q < nsplit; ++q) v += part[(size_t)q * count + i];
    out[i] = v;
}

// r = y - t, loss = mean r^2 (double, fixed order), dy = 2 r / S
__global__ __launch_bounds__(1024) void kw_loss(int S, const float *y, const float *t, float *dy,
                                                double *loss) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int m = threadIdx.x; m < S; m += 1024) {
        const float r = y[m] - t[m];
        s += (double)r * (double)r;
        dy[m] = 2.0f * r / (float)S;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)S;
}

// Adam with bias correction
__global__ __launch_bounds__(256) void kw_adam(int64_t P, float *p, const float *g, float *m,
                                               float *v, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// w_i = (y_i - mean y) / N in double (one block, fixed order)
__global__ __launch_bounds__(1024) void kw_center(int n, const float *y, double *w) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += (double)y[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double mean = red[0] / (double)n;
    for (int i = threadIdx.x; i < n; i += 1024) w[i] = ((double)y[i] - mean) / (double)n;
}

// t_i = N (w_i - mean w) in float (one block, fixed order)
__global__ __launch_bounds__(1024) void kw_targets(int n, const double *w, float *t) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double mean = red[0] / (double)n;
    for (int i = threadIdx.x; i < n; i += 1024) t[i] = (float)((double)n * (w[i] - mean));
}

// ------------------------------------------------------- BF16 inference

// Inference in BF16 on the matrix cores with FP32 accumulation
// (v_mfma_f32_32x32x16_bf16): the weights are kept as transposed BF16 copies
// (layer 1 padded from 20 to 32 inputs), activations are rounded to BF16
// between layers, biases and the ReLU are applied in FP32.
constexpr int kK1 = 32;                                  // layer-1 inputs, padded
constexpr int64_t kBfW1 = 0;                             // [128][32]
constexpr int64_t kBfW2 = kBfW1 + (int64_t)kHid * kK1;   // [128][128]
constexpr int64_t kBfW3 = kBfW2 + (int64_t)kHid * kHid;  // [128][128]
constexpr int64_t kBfW4 = kBfW3 + (int64_t)kHid * kHid;  // [128]
constexpr int64_t kBfCount = kBfW4 + kHid;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef unsigned short ushort8_t __attribute__((ext_vector_type(8)));

// round to nearest even (the values are finite)
__device__ inline unsigned short to_bf16(float v) {
    const unsigned u = __float_as_uint(v);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__global__ __launch_bounds__(256) void kw_to_bf16(const float *P, unsigned short *Wb) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= kBfCount) return;
    float v;
    if (e < kBfW2) {
        const int o = (int)(e / kK1), k = (int)(e % kK1);
        v = k < kFeat ? P[oW1 + (int64_t)k * kHid + o] : 0.0f;
    } else if (e < kBfW4) {
        const int64_t base = e < kBfW3 ? kBfW2 : kBfW3;
        const int64_t src = e < kBfW3 ? oW2 : oW3;
        const int o = (int)((e - base) / kHid), k = (int)((e - base) % kHid);
        v = P[src + (int64_t)k * kHid + o];
    } else {
        v = P[oW4 + (e - kBfW4)];
    }
    Wb[e] = to_bf16(v);
}

// One wave per 32 samples (its activations in its own LDS rows, so no block
// barriers); y[s] for s < S.
__global__ __launch_bounds__(256) void kw_infer_bf16(const float *P, const unsigned short *Wb,
                                                     const float *X, int S, float *y) {
    constexpr int kRow = kHid + 8;  // padded LDS row
    __shared__ unsigned short act[4][32 * kRow];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int half = lane >> 5, col = lane & 31;
    const int s0 = (blockIdx.x * 4 + wave) * 32;
    if (s0 >= S) return;  // whole waves leave together
    unsigned short *A = act[wave];
    for (int e = lane; e < 32 * kK1; e += 64) {
        const int r = e / kK1, k = e % kK1;
        const float v = (s0 + r < S && k < kFeat) ? X[(int64_t)(s0 + r) * kFeat + k] : 0.0f;
        A[r * kRow + k] = to_bf16(v);
    }
    auto sync_wave = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    sync_wave();
    auto layer = [&](int kin, const unsigned short *Wt, const float *bias) {
        floatx16_t acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = floatx16_t{};
        for (int k0 = 0; k0 < kin; k0 += 16) {
            const bf16x8_t a = __builtin_bit_cast(
                bf16x8_t, *reinterpret_cast<const ushort8_t *>(A + col * kRow + k0 + 8 * half));
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const bf16x8_t b = __builtin_bit_cast(
                    bf16x8_t, *reinterpret_cast<const ushort8_t *>(Wt + (int64_t)(cb * 32 + col) * kin + k0 + 8 * half));
                acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[cb], 0, 0, 0);
            }
        }
        sync_wave();  // every read of the inputs precedes the writes below
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int o = cb * 32 + col;
            const float bo = bias[o];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r / 4) + 4 * half + (r % 4);
                A[row * kRow + o] = to_bf16(fmaxf(acc[cb][r] + bo, 0.0f));
            }
        }
        sync_wave();
    };
    layer(kK1, Wb + kBfW1, P + ob1);
    layer(kHid, Wb + kBfW2, P + ob2);
    layer(kHid, Wb + kBfW3, P + ob3);
    // output layer: y = b4 + sum_o h3[o] w4[o] (BF16 operands, FP32 sums)
    const int row = col;
    float part = 0.0f;
    for (int o = 64 * half; o < 64 * half + 64; ++o)
        part = fmaf(from_bf16(A[row * kRow + o]), from_bf16(Wb[kBfW4 + o]), part);
    part += __shfl_xor(part, 32);
    if (half == 0 && s0 + row < S) y[s0 + row] = part + P[ob4];
}

template <bool TA, bool TB, int EPI>
hipError_t gemm(hipStream_t s, int M, int N, int K, const float *A, int lda, const float *B, int ldb,
                float *C, int ldc, const float *bias = nullptr, const float *mask = nullptr, int ldm = 0) {
    (void)hipGetLastError();
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    kw_gemm<TA, TB, EPI><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, mask, ldm);
    return hipGetLastError();
}

// Splits of the samples for the weight gradients (at most kSplitMax).
int grad_splits(int K) { return std::max(1, std::min(kSplitMax, (K + 127) / 128)); }

// dW[M][N] = A^T B over K samples and, if db, db[N] = column sums of B
// (part: kSplitMax (M N + N) floats of scratch).
hipError_t weight_grad(hipStream_t s, int M, int N, int K, const float *A, int lda, const float *B,
                       int ldb, float *dW, float *db, float *part) {
    const int ns = grad_splits(K);
    const int kslice = ((K + ns - 1) / ns + 15) & ~15;
    float *bpart = part + (size_t)ns * M * N;
    dim3 grid((N + 63) / 64, (M + 63) / 64, ns);
    if (db) kw_gemm_tn_part<true><<<grid, 256, 0, s>>>(M, N, K, kslice, A, lda, B, ldb, part, bpart);
    else kw_gemm_tn_part<false><<<grid, 256, 0, s>>>(M, N, K, kslice, A, lda, B, ldb, part, bpart);
    kw_reduce_parts<<<(M * N + 255) / 256, 256, 0, s>>>(M * N, ns, part, dW);
    if (db) kw_reduce_parts<<<(N + 255) / 256, 256, 0, s>>>(N, ns, bpart, db);
    return hipGetLastError();
}

}  // namespace

// Forward pass of S samples: H1, H2, H3 [S][128] and y [S].
hipError_t forward(hipStream_t s, const float *P, const float *X, int S, float *H1, float *H2,
                   float *H3, float *y) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    hipError_t e;
    if ((e = gemm<false, false, 2>(s, S, kHid, kFeat, X, kFeat, P + oW1, kHid, H1, kHid, P + ob1)) != hipSuccess) return e;
    if ((e = gemm<false, false, 2>(s, S, kHid, kHid, H1, kHid, P + oW2, kHid, H2, kHid, P + ob2)) != hipSuccess) return e;
    if ((e = gemm<false, false, 2>(s, S, kHid, kHid, H2, kHid, P + oW3, kHid, H3, kHid, P + ob3)) != hipSuccess) return e;
    return gemm<false, false, 1>(s, S, 1, kHid, H3, kHid, P + oW4, 1, y, 1, P + ob4);
}

const int64_t kBf16Count = kBfCount;

hipError_t to_bf16_weights(hipStream_t s, const float *P, unsigned short *Wb) {
    (void)hipGetLastError();
    kw_to_bf16<<<(unsigned)((kBfCount + 255) / 256), 256, 0, s>>>(P, Wb);
    return hipGetLastError();
}

hipError_t infer_bf16(hipStream_t s, const float *P, const unsigned short *Wb, const float *X, int S,
                      float *y) {
    (void)hipGetLastError();
    kw_infer_bf16<<<(unsigned)((S + 127) / 128), 256, 0, s>>>(P, Wb, X, S, y);
    return hipGetLastError();
}

// Loss and gradient of the loss with respect to the flat parameters (into G).
hipError_t backward(hipStream_t s, const float *P, const float *X, const float *t, int S, float *H1,
                    float *H2, float *H3, float *y, float *dy, float *dA, float *dB, float *G,
                    double *loss, float *part) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    hipError_t e;
    if ((e = forward(s, P, X, S, H1, H2, H3, y)) != hipSuccess) return e;
    kw_loss<<<1, 1024, 0, s>>>(S, y, t, dy, loss);
    // layer 4: dW4 = H3^T dy, db4 = sum dy, dH3 = dy W4^T * (H3 > 0)
    if ((e = weight_grad(s, kHid, 1, S, H3, kHid, dy, 1, G + oW4, G + ob4, part)) != hipSuccess) return e;
    if ((e = gemm<false, true, 3>(s, S, kHid, 1, dy, 1, P + oW4, 1, dA, kHid, nullptr, H3, kHid)) != hipSuccess) return e;
    // layer 3
    if ((e = weight_grad(s, kHid, kHid, S, H2, kHid, dA, kHid, G + oW3, G + ob3, part)) != hipSuccess) return e;
    if ((e = gemm<false, true, 3>(s, S, kHid, kHid, dA, kHid, P + oW3, kHid, dB, kHid, nullptr, H2, kHid)) != hipSuccess) return e;
    // layer 2
    if ((e = weight_grad(s, kHid, kHid, S, H1, kHid, dB, kHid, G + oW2, G + ob2, part)) != hipSuccess) return e;
    if ((e = gemm<false, true, 3>(s, S, kHid, kHid, dB, kHid, P + oW2, kHid, dA, kHid, nullptr, H1, kHid)) != hipSuccess) return e;
    // layer 1
    if ((e = weight_grad(s, kFeat, kHid, S, X, kFeat, dA, kHid, G + oW1, G + ob1, part)) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t features(hipStream_t s, int n, const double *x, const double *A, const double *v,
                    const double *lo, const double *hi, const double *grad0, int *nb, double *tmp,
                    float *F) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    kw_features<<<(n + 3) / 4, 256, 0, s>>>(n, x, A, v, lo[0], lo[1], hi[0], hi[1], F, nb);
    const unsigned nb1 = (unsigned)((n + 255) / 256);
    kw_deficit<<<nb1, 256, 0, s>>>(n, grad0, tmp, F);
    for (int h = 0; h < kPoolHops; ++h) {
        const double *in = tmp + (size_t)(h & 1) * n;
        double *out = tmp + (size_t)((h + 1) & 1) * n;
        kw_pool<<<nb1, 256, 0, s>>>(n, nb, in, out, F, 17 + h);
    }
    return hipGetLastError();
}

hipError_t adam(hipStream_t s, float *P, const float *G, float *M, float *V, float lr, int64_t step) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    kw_adam<<<(unsigned)((kParams + 255) / 256), 256, 0, s>>>(kParams, P, G, M, V, lr, c1, c2);
    return hipGetLastError();
}

hipError_t targets(hipStream_t s, int n, const double *w, float *t) {
    (void)hipGetLastError();
    kw_targets<<<1, 1024, 0, s>>>(n, w, t);
    return hipGetLastError();
}

hipError_t center(hipStream_t s, int n, const float *y, double *w) {
    (void)hipGetLastError();  // clear a stale error left by an earlier call
    kw_center<<<1, 1024, 0, s>>>(n, y, w);
    return hipGetLastError();
}

}  // namespace ws
}  // namespace apd
