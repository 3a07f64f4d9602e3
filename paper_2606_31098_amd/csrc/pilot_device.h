// pilot_device.h -- device-side layout shared by the host runtime and the
// gfx950 kernels of libpilot (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pilot {

constexpr int kMaxLevels = 4;
constexpr int kBlock = 256;      // threads per pass block (4 wave64)
// Per-hypothesis partial record (floats): 21 H, 6 g, count, then the cost as
// an FP64 bit pattern in two slots, 1 pad.
constexpr int kNV = 32;
constexpr int kNSum = 28;        // float sums: 21 H + 6 g + visible count
constexpr int kCostSlot = 28;    // FP64 cost occupies slots 28, 29

// One pyramid level of one frame, as the pass kernel reads it.
struct LevelDev {
    const void *feat;
    const float *qconf;
    const float *x, *y, *z;
    const void *ref;
    const float *ref_w;
    double fx, fy, cx, cy;
    int H, W, C, N;
    int iters, loss_kind;
    double loss_b;
    int dtype;
    // the level's tile for this frame: anchors per lane group (a work item
    // covers kBlock / G * ppg anchors) and the packed-tile threshold of
    // use_packed (INT_MAX: never packed); frames with different values share
    // a launch when their kernel instantiation is the same
    int ppg, pack_min, pad;
    // pass kernel variants 3 to 10: per-cell Gram matrices of the bilinear
    // coefficients of cell (x0, y0) at index y0 W + x0, 10 doubles per cell
    // (variants 3 to 8) or 12 floats (variants 9 and 10: 10 entries, 2 pads)
    const double *gram;
    // anchors in spatial order: when perm is set, x, y, z, ref and ref_w point
    // at the library's copies in Morton order of the anchors' ground position
    // (perm[j] = caller index of anchor j) and in_* at the caller's arrays
    const float *in_x, *in_y, *in_z, *in_w;
    const void *in_ref;
    int *perm;
};

// Anchor sets of up to this many anchors are sorted into spatial order
// (larger ones are taken in the caller's order).
constexpr int kSortMaxN = 16384;

// One frame (solve) or one serving slot.
struct FrameDev {
    LevelDev lv[kMaxLevels];
    int n_levels, M, hyp_base, slot;
    // gravity prior
    int use_g, grav_kind;
    double grav_b, lam_imu;
    double g_imu[3], g_world[3];
    // range prior; q = d_range * unit ray of the range pixel (camera frame)
    int use_r, range_kind;
    double range_b, lam_range;
    double q[3];
    const float *dsm;
    int Hd, Wd;
    double dsm_x0, dsm_y0, dsm_gsd;
    // LM control
    double tau, up, down, lmin_rel, lmax_rel, tol_t, tol_r;
    double z_min;
    int min_valid, adaptive;
    double alpha_ratio, grav_gate, range_gate, cost_tol;
    const double *poses_in;
    const double *prior_poses;   // device hypothesis generation (hyp_offsets non-NULL)
    const int *prior_best;
    const double *hyp_offsets;
    // outputs
    double *poses_out, *cost_out, *alpha_out;
    int *iters_out, *status_out, *best_out;
    // diagnostic outputs (pilot_linearize)
    double *diag_H, *diag_g, *diag_cost;
    int *diag_n;
    int *done_flag;   // serving: set to 1 by the finalize step
    int keep_top, prune_level;
};

// A tile of G hypotheses x P anchors of one frame at one level.
struct WorkItem {
    int frame;       // index into the FrameDev table
    int hbase;       // global index of the tile's first hypothesis (frame base + tile * G)
    int ptile;       // anchor tile (P anchors)
    int nh;          // hypotheses in the tile (G, fewer in a frame's last tile)
};

// A hypothesis tile of one frame and the run of work items holding its partials.
struct TileItem {
    int frame;
    int htile;
    int first_item;  // item index of anchor tile 0
    int n_ptiles;
    int hbase;       // global index of the tile's first hypothesis
    int nh;          // hypotheses in the tile
};

// LM state of one hypothesis (FP64 master pose and damped system).
struct HypState {
    double T[12];    // accepted pose
    double Tc[12];   // candidate under evaluation
    double dxi[6];   // step that produced Tc
    double H[21];    // system at T (upper triangle, row by row)
    double g[6];
    double cost, lam, lmin, lmax;
    double alpha[2]; // prior scales (gravity, range) of the current level
    int level, phase, it_level, it_total, status, nvalid;
    int home;        // the hypothesis' own (global) index: packed copies of the state carry it
    int pad1;
};

enum { PHASE_START = 0, PHASE_CAND = 1 };
enum { ST_CONVERGED = 0, ST_MAX_ITERS = 1, ST_STALLED = 2, ST_DEGENERATE = 3, ST_PRUNED = 4 };
constexpr int HLEV_DONE = -1;       // finished
constexpr int HLEV_WAIT = -2;       // finished the pruning level, waiting for the ranking
enum { MODE_LM = 0, MODE_DIAG = 1 };

// Pose a hypothesis is evaluated at in the next pass: R row-major (9), t (3),
// 4 pad -> 128 bytes.
struct PoseEval {
    double v[16];
};

struct PassArgs {
    const FrameDev *frames;
    const WorkItem *items;
    int n_items;
    int level;
    const PoseEval *pose;
    const int *hlev;             // level whose evaluation is pending; -1 finished
    float *partials;             // [item][G][kNV]
    const int *run_flag;         // NULL, or 0 when no hypothesis is at this level (the launch has nothing to do)
    // Packed hypothesis tiles (pass variants 3 to 10), or NULL: the tile whose
    // first hypothesis index is hb holds, instead of hypotheses hb .. hb + G - 1,
    // the packed entries hb .. hb + G - 1 of the hypotheses still at the level
    // (pcount[frame] of them from the frame's hyp_base on; their poses under
    // evaluation are ppose[hb + hh]); tiles past that count have nothing to do.
    // Block 0 clears pcount_clear[0 .. n_frames) (the counts the pass's
    // epilogue appends to).
    const PoseEval *ppose;
    const int *pcount;
    int *pcount_clear;
    int n_frames;
};

struct EpilogueArgs {
    const FrameDev *frames;
    const TileItem *tiles;
    int n_tiles;
    int level;
    int G;
    int mode;                    // MODE_LM or MODE_DIAG
    const float *partials;
    PoseEval *pose;
    int *hlev;
    HypState *hs;
    unsigned long long *pairs;   // evaluated anchor x hypothesis pairs of this launch's class
    int *next_flag;              // NULL, or set to 1 when a hypothesis stays at this level
    int mask_first;              // test the tile mask before fetching the partial sums (launches
                                 // where most tiles are at other levels), else after
    // packed hypothesis tiles (as in PassArgs), or NULL: slot hh of the tile
    // is packed entry hb + hh, whose LM state and pose are phs / ppose[hb + hh]
    // (the state's `home` is the hypothesis' own index, where its state and
    // pose are also written back); the hypotheses that stay at the level are
    // appended (tiles in order of arrival, a tile's in slot order) to
    // phs_next / ppose_next, counted in pcount_next, for the next pass
    const HypState *phs;
    const PoseEval *ppose;
    const int *pcount;
    HypState *phs_next;
    PoseEval *ppose_next;
    int *pcount_next;
};

// Packed or contiguous hypothesis tiles for one frame in one pass: packed when
// the tiles a contiguous walk may find active (at most one per hypothesis
// still at the level, at most every tile) hold more than pack_min work items,
// i.e. when packing saves rounds of blocks; below that the contiguous tiles
// fit in one round and packing would only put more distinct cells into fewer
// items.  The pass kernel and its epilogue take the decision from the same
// count, and sums do not depend on the tiling: results are the same either way.
__host__ __device__ inline bool use_packed(int count, int M, int G, int npt, int pack_min)
{
    const int tiles = (M + G - 1) / G;
    return (long long)(count < tiles ? count : tiles) * npt > pack_min;
}

}  // namespace pilot
