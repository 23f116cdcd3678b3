// apd_batch.h -- device-side structures of the batched solver (libapd
// internal).
#pragma once

#include "apd_internal.h"

namespace apd {

// One instance of a batch: geometry, the caller's seed arrays, and the
// solver's vectors inside the batch scratch.
struct BInst {
    Geo g;
    const double *x;
    const double *A;
    const double *v;
    double *w;        // [n] accepted iterate
    double *g_acc;    // [n] projected grad f at w
    double *d;        // [n] search direction
    double *wt;       // [n] trial point (what the pass evaluates)
    double *gt;       // [n] grad f at the trial point
    double *S;        // [10][n] curvature pairs (circular)
    double *Y;        // [10][n]
    double *rho;      // [10]
    uint64_t *mom;    // [n][K]
    double *eig;      // [n][2] eigenvalue range of every A_i
    int tiles1;       // tiles along axis 1
    int tiles2;       // tiles along axis 2 (3D)
    int tiles0;       // tiles along axis 0
    int *tile_lists;  // [tiles][kBatchListCap] candidate lists (vector kernel with lists) or null
    int *tile_count;  // [tiles]
    int *super_lists; // [super-tiles][kBatchSuperCap] (vector kernel with lists) or null
    int *super_count; // [super-tiles]
    int sf[3];        // tiles per super-tile along each axis
    int nst[3];       // super-tiles along each axis
    int tp;           // pixels per lane of the vector kernel's tiles
};

constexpr int kBatchListCap = 256;   // candidate seeds kept per tile for the batched re-check
constexpr int kBatchSuperCap = 512;  // candidate seeds kept per super-tile

// Scalar solver state of one instance.
struct BState {
    double f, gd, alpha, crit;
    double ftrial, crit_trial;
    double vsum, wmax, gamma0;
    float lam;        // Gershgorin bound of every A_i (Cert::lam)
    float kap;        // condition bound of every A_i (Cert::kap)
    int phase;        // 0: first evaluation pending, 1: line search
    int npairs, head, t;
    int iters, evals;
    int status, active, bad;
};

// Batch-wide control block.
struct BCtl {
    // re-check queue length and its segments (one per tile that queued
    // pixels): an 8-byte pair advanced by one atomic
    unsigned qcount;
    unsigned segcount;
    unsigned next;    // work-item counter of kb_assign
    int active;       // instances still running
    int max_iter, max_evals;
    double eps;
    double gamma0;
};

static_assert(offsetof(BCtl, qcount) % 8 == 0 && offsetof(BCtl, segcount) == offsetof(BCtl, qcount) + 4,
              "the queue counters form one aligned 8-byte pair");

hipError_t launch_batch_setup(int dim, BInst *inst, BState *st, int B, hipStream_t s);
// super0: prefix sums of the instances' super-tile counts (used with lists)
// segs: room for one queue segment per tile of the batch
hipError_t launch_batch_step(int dim, BInst *inst, BState *st, const int64_t *tile0, int B,
                             BCtl *ctl, uint64_t *queue, QSeg *segs, int grid_assign, int variant,
                             int recheck_blocks, const int64_t *super0, int64_t nsuper, hipStream_t s);
hipError_t launch_batch_init(BInst *inst, double *const *src, int B, bool warm, hipStream_t s);
hipError_t launch_batch_scatter(BInst *inst, double *const *dst, int B, hipStream_t s);

}  // namespace apd
