// apd_internal.h -- shared declarations of the libapd device code and its
// host driver.  Not installed; the public interface is include/apd.h.
#pragma once

#include <stddef.h>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apd {

constexpr int kThreads = 256;  // 4 waves of 64
constexpr int kWaves = 4;
constexpr int kChunk = 256;    // seeds staged in LDS at a time
constexpr int kP = 4;          // pixels per lane along axis 0

// Tile of the vector and bf16 kernels with p pixels per lane along axis 0.
// 2D: a wave is 4 x 16 lanes (lane l at lane row l / 16, column l % 16),
// so it covers 4p x 16 pixels, and the block's 4 waves form a 2 x 2 square
// of waves: the tile is 8p x 32 pixels.  3D: a wave is 8 x 8 lanes on axes
// 1 and 2; the 4 waves are stacked along axis 0: the tile is 4p x 8 x 8.
// Square-ish wave boxes keep the candidate lists short: the upper bound a
// candidate must beat comes from the box's far corners.
constexpr int kHybRows3 = 16;  // rows along axis 0 of the hybrid tile: 3D (8 symmetric pairs per lane)
constexpr int kHybRows2 = 32;  // 2D (4 pairs per lane, 4 waves)
constexpr int tile_ext(int dim, int p, int axis) {
    return dim == 2 ? (axis == 0 ? 8 * p : axis == 1 ? 32 : 1) : (axis == 0 ? kWaves * p : 8);
}
constexpr int wave_ext(int dim, int p, int axis) {
    return dim == 2 ? (axis == 0 ? 4 * p : axis == 1 ? 16 : 1) : (axis == 0 ? p : 8);
}

// Problem geometry passed by value to every kernel.
struct Geo {
    int dim;
    int n;
    int grid[3];
    double lo[3];
    double s[3];      // pixel side (hi - lo) / M, rounded once on the host
    double pixvol;    // |P| = prod s
    const uint8_t *mass = nullptr;  // [J] pixel weights q_j (measure q_j/255 |P|) or null
    double munit = 0.0;             // measure of one unit of the moments' count
    int vec_p = 0;                  // pixels per lane of the vector kernel (0: by grid size)
    int power = 2;                  // cost |y - x|_A^power - w (2: the APD cost)
};

// Seed data (device pointers, caller-owned, row-major).
struct Seeds {
    const double *x;  // [n][dim]
    const double *A;  // [n][dim][dim], upper triangle read
    const double *w;  // [n]
    const double *v;  // [n] or nullptr
};

// Per-pass device scalars.
struct Scalars {
    double wmax;      // max_i w_i (the gauge shift of the single-precision tier)
    double vsum;      // sum_i v_i
    double g;         // objective of eq. (2.7)
    double maxrel;    // max_i |v_i - m_i|P|| / v_i
    // pixels queued for the double re-check and the queue's segments (with
    // candidate lists): one 8-byte pair, taken together by one atomic
    unsigned qcount;
    unsigned segcount;
    float lam;        // upper bound of max_i lambda_max(A_i) (Gershgorin)
    float kap;        // upper bound of max_i lambda_G(A_i) / lambda_min(A_i)
    int bad;          // validation bits
    unsigned long long qtotal;  // sum of the pixel weights (validation)
    unsigned seq;     // host copy only: the finalize's count of published passes
    unsigned credited;  // tiles credited whole (boundary-aware refinement)
    double gpix;        // sum_j q_j C_{H_j j} (costs other than the squared norm)
};

static_assert(offsetof(Scalars, qcount) % 8 == 0 && offsetof(Scalars, segcount) == offsetof(Scalars, qcount) + 4,
              "the queue counters form one aligned 8-byte pair");

enum : int { kBadW = 1, kBadX = 2, kBadA = 4, kBadSPD = 8, kBadV = 16 };

// Per-block partial results of the multi-block prep and finalize kernels;
// the last block to finish (ticket) combines them in block order, so the
// sums do not depend on scheduling.  ticket is zero between launches.
constexpr int kMaxParts = 256;
struct BlockParts {
    double a[kMaxParts];   // prep: max w;  finalize: objective terms
    double b[kMaxParts];   // prep: sum v;  finalize: max relative error
    float l[kMaxParts];    // prep: Gershgorin bound
    float k[kMaxParts];    // prep: condition bound
    int bad[kMaxParts];    // prep: validation bits
    unsigned ticket;
    unsigned published;    // passes whose scalars the finalize wrote to host memory
};

// moments per cell: count, first and second moments of the odd pixel
// coordinates o_d = 2 k_d + 1 (exact unsigned integers)
constexpr int moments_per_cell(int dim) { return dim == 2 ? 6 : 10; }

constexpr int kCullCapDefault = 2048;  // = kCullCap, the tile lists' default capacity

// A block's share of the re-check queue: queue[start, start + count) are
// pixels of tile `tile` (of instance `tag` in the batched form).
struct QSeg {
    uint32_t start;
    uint32_t count;
    int32_t tile;
    int32_t tag;
};

// Per-pass constants of the single-precision certificates: lam bounds the
// Gershgorin bound lambda_G = max_r sum_c |a_rc| of every A_i (so every
// eigenvalue), kap bounds every lambda_G(A_i) / lambda_min(A_i).
struct Cert {
    float lam;
    float kap;
};

// Upper bound of lambda_G(A) / lambda_min(A) for a symmetric positive
// definite A with Gershgorin bound lg and determinant det > 0: the product
// of the eigenvalues is det and none exceeds lg, so lambda_min >= det /
// lg^(D-1); doubled for the rounding of det.
__host__ __device__ inline double cond_bound(int dim, double lg, double det) {
    const double p = dim == 2 ? lg * lg : lg * lg * lg;
    return 2.0 * p / det;
}

struct PassOut {
    int32_t *labels;     // [J] or nullptr
    uint64_t *mom;       // [n][K] or nullptr
    unsigned *queue;     // [J] re-check queue (single-precision tier)
    uint64_t *queue64 = nullptr;  // batched form: (tag << 32 | pixel) entries
    uint32_t tag = 0;             // batched form: instance index
    // candidate lists of the culled vector kernel, kept for the re-check:
    // tile t's seeds in tile_lists[t * list_cap ...], their number in
    // tile_count[t] (above list_cap: every seed); tiles of tp pixels per lane
    int *tile_lists = nullptr;
    int *tile_count = nullptr;
    int list_cap = kCullCapDefault;  // entries kept per tile list
    int tp = 0;
    int ntile[3] = {0, 0, 0};
    // super-tiles of sf[0] x sf[1] x sf[2] tiles (nst[] of them per axis):
    // their candidate seeds, from which the tiles pick theirs
    const int *super_list = nullptr;   // [super-tiles][super_cap]
    const int *super_count = nullptr;  // above super_cap: every seed
    int super_cap = kCullCapDefault;
    int sf[3] = {1, 1, 1};
    int nst[3] = {1, 1, 1};
    // segments of the queue (one per block that queued pixels), so that the
    // re-check can take a tile's pixels together; null: not recorded.  With
    // segments the queue counter is the first of an 8-byte aligned pair
    // (pixels, segments) advanced by one 64-bit atomic.
    QSeg *segs = nullptr;
    int tile_id = 0;  // this tile's index in the tile lists' layout
    // per-pixel lower bound of the relative top-two gap (apd_assign) or
    // null; with candidate lists the tiles also keep, in tile_U, the bound
    // below which no seed outside their list can cost (the re-check needs
    // it for the runner-up)
    float *rel_gap = nullptr;
    double *tile_U = nullptr;
    // the hybrid kernel's seed order (k_seed_order): position q of its scan
    // holds seed seed_order[q]; null: the identity
    const int *seed_order = nullptr;
    // boundary-aware refinement: a tile whose candidate list holds a single
    // seed is that seed's cell at every pixel, and is credited whole
    // (closed-form moments) instead of pixel by pixel
    bool adaptive = false;
    unsigned *credited = nullptr;  // counts the tiles credited whole, or null
    // costs other than the squared norm (FP64 tier): per-block sums of the
    // pixels' least costs, q_j C_{H_j j}, summed into Scalars::gpix
    double *cost_part = nullptr;
};

constexpr int kMfmaLds = kChunk * 16;  // floats of LDS staging of the matrix-core tile
constexpr int kCullCap = 2048;         // candidate seeds kept per tile
constexpr int kSuperCap = 2048;        // candidate seeds kept per super-tile

struct FinalOut {
    double *grad;        // [n] or nullptr
    int64_t *counts;     // [n] or nullptr
    double *centroids;   // [n][dim] or nullptr
    // pinned host copy of the scalars, written at the end; its seq field is
    // written last, after every other host write of the pass is visible
    Scalars *host_sc = nullptr;
};

// Pixels per lane of the vector kernel on this grid, with or without
// candidate lists (its tiles are kWaves * that many pixels long along axis 0).
int vec_pixels_per_lane(const Geo &g, bool cull);
// Pixel rows per lane of the bf16 kernel on this grid (its tiles are kWaves
// * that many pixels long along axis 0, with the vector kernel's other axes).
int bf16_pixels_per_lane(const Geo &g);
// With w_src (pinned host memory) the prep kernel first copies w_src into
// sd.w (then a device buffer of the library's), one copy fewer per pass.
hipError_t launch_prep(const Geo &g, const Seeds &sd, Scalars *sc, uint64_t *mom, double *eig,
                       BlockParts *bp, hipStream_t st, const double *w_src = nullptr);
// Candidate lists of the super-tiles described by out (sf, nst), written to
// list / count.
hipError_t launch_super_cull(const Geo &g, const Seeds &sd, const Scalars *sc, const double *eig,
                             const PassOut &out, int *list, int *count, hipStream_t st);
hipError_t launch_assign_cull(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                              const PassOut &out, hipStream_t st);
hipError_t launch_assign_fp64(const Geo &g, const Seeds &sd, Scalars *sc,
                              const PassOut &out, hipStream_t st);
// Blocks of the FP64 assignment kernel (the entries of PassOut::cost_part).
int64_t fp64_blocks(const Geo &g);
hipError_t launch_assign_fp32(const Geo &g, const Seeds &sd, Scalars *sc,
                              const PassOut &out, hipStream_t st);
hipError_t launch_assign_mfma(const Geo &g, const Seeds &sd, Scalars *sc,
                              const PassOut &out, hipStream_t st);
// The pass over every seed with the matrix cores forming each position's
// quadratic in u0 and the vector ALU evaluating it (16 x 16 x 8 tiles in 3D,
// 32 x 32 in 2D).
hipError_t launch_assign_hyb(const Geo &g, const Seeds &sd, Scalars *sc,
                             const PassOut &out, hipStream_t st);
// The seeds in the order of a space-filling curve over the box (ord [n]),
// for the hybrid kernel's super-blocks.
hipError_t launch_seed_order(const Geo &g, const Seeds &sd, int *ord, hipStream_t st);
// The bf16 pass over every seed (eig null) or over the tiles' candidate
// lists (eig from the prep kernel, tile geometry of bf16_pixels_per_lane).
hipError_t launch_assign_bf16(const Geo &g, const Seeds &sd, Scalars *sc, const double *eig,
                              const PassOut &out, hipStream_t st);
hipError_t launch_recheck(const Geo &g, const Seeds &sd, const Scalars *sc,
                          const PassOut &out, hipStream_t st);
// Zeroes `bytes` (a multiple of 4) at device address p with a kernel.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// Adds sum_j mass[j] to sc->qtotal (which the prep kernel zeroes).
hipError_t launch_mass_total(const Geo &g, Scalars *sc, hipStream_t st);
hipError_t launch_finalize(const Geo &g, const Seeds &sd, const uint64_t *mom, Scalars *sc,
                           const FinalOut &out, BlockParts *bp, hipStream_t st);

namespace ws {
extern const int64_t kParamCount;
hipError_t features(hipStream_t s, int n, const double *x, const double *A, const double *v,
                    const double *lo, const double *hi, const double *grad0, int *nb, double *tmp,
                    float *F);
hipError_t forward(hipStream_t s, const float *P, const float *X, int S, float *H1, float *H2,
                   float *H3, float *y);
// part: kSplitMax * (128 * 128 + 128) floats of scratch (split weight gradients)
constexpr int kSplitMax = 32;
hipError_t backward(hipStream_t s, const float *P, const float *X, const float *t, int S, float *H1,
                    float *H2, float *H3, float *y, float *dy, float *dA, float *dB, float *G,
                    double *loss, float *part);
hipError_t adam(hipStream_t s, float *P, const float *G, float *M, float *V, float lr, int64_t step);
// BF16 inference: transposed BF16 weight copies (kBf16Count values) and the
// matrix-core forward pass.
extern const int64_t kBf16Count;
hipError_t to_bf16_weights(hipStream_t s, const float *P, unsigned short *Wb);
hipError_t infer_bf16(hipStream_t s, const float *P, const unsigned short *Wb, const float *X, int S,
                      float *y);
hipError_t center(hipStream_t s, int n, const float *y, double *w);
hipError_t targets(hipStream_t s, int n, const double *w, float *t);
}  // namespace ws

}  // namespace apd
