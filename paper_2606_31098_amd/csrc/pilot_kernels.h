// pilot_kernels.h -- launch entry points of the gfx950 kernels (internal).
#pragma once

#include "pilot_device.h"

namespace pilot {

struct TileConfig {
    int G = 4;          // lanes per anchor = hypotheses per tile (1 to 16)
    int PPG = 1;        // anchors per lane group per work item
    int grid = 0;       // blocks per CU of a persistent grid (0: one block per item); launch: blocks
    int variant = 1;    // pass kernel: 1 batch-then-compute loop, 2 software-pipelined loop,
                        // 3-8 per-cell Gram tables (see pilot_pass3.inc), 9-10 the same with
                        // FP32 arithmetic on the per-pair path for bf16 maps (pilot_pass4.inc)
    int pack = 0;       // variants 3-10: hypothesis tiles 0 contiguous, 1 packed when that saves
                        // rounds of blocks (use_packed), 2 packed whenever hypotheses remain
};

// True if a pass kernel exists for (C, dtype, G).
bool pass_supported(int C, int dtype, int G);

// One pass over `n_items` work items at `level`, every item a tile of
// G hypotheses x (kBlock / G * PPG) anchors of frames with C channels:
// writes the per-item partial sums.
hipError_t launch_pass(int C, int dtype, const TileConfig &tc, const PassArgs &a, hipStream_t s);

// Per hypothesis tile: FP64 reduction of the partials in item order and the
// LM step (or, in MODE_DIAG, the diagnostic outputs).
hipError_t launch_epilogue(const EpilogueArgs &e, hipStream_t s);

// Initialise hypothesis state of frames[0..n_frames) from their poses_in
// (mode LM) or from `diag_poses` at `diag_level` (mode DIAG, one frame), and,
// when `flags` is given, the solve's pass flags (see EpilogueArgs::next_flag):
// n_flags flags, flag_stride per level.
hipError_t launch_init(const FrameDev *frames, int n_frames, int max_M, HypState *hs,
                       PoseEval *pose, int *hlev, int mode, const double *diag_poses,
                       int diag_level, hipStream_t s, int *flags = nullptr, int n_flags = 0,
                       int flag_stride = 1);

// Per-cell Gram matrices of the bilinear coefficients of the feature map of
// level `level` of frames[frame] (pass kernel variants 3 to 10), cells
// y0 W + x0, written to that level's `gram`: fmt 0, 10 doubles per cell
// (variants 3 to 8); fmt 1, 12 floats per cell, the 10 entries and two zero
// pads (variants 9 and 10).  The kernel reads the map, its shape and the
// table pointer from the device descriptor; H, W, C and dtype (the host's
// copy of them) size the grid and pick the instantiation.
hipError_t launch_gram(const FrameDev *frames, int frame, int level, int H, int W, int C, int dtype, int fmt,
                       hipStream_t s);

// Geo-anchor lift and reference-descriptor sampling (see pilot_lift).
hipError_t launch_lift(const float *dsm, int Hd, int Wd, double x0, double y0, double gsd, const float *uv, int N,
                       const void *ref_map, int Hr, int Wr, int C, int dtype, double scale, float *x, float *y,
                       float *z, void *ref_out, hipStream_t s);

// Top-K pruning of frames whose hypotheses all finished their pruning level.
hipError_t launch_prune(const FrameDev *frames, int n_frames, HypState *hs, PoseEval *pose, int *hlev,
                        hipStream_t s);

// Per frame: the LM states and poses under evaluation of the hypotheses whose
// pending level is `level`, in index order, to phs / ppose[hyp_base ..), their
// number to pcount[frame], and the frame's counts in pclear0 / pclear1 set to
// zero (the packed hypothesis tiles of a level's first pass; see
// PassArgs::ppose and EpilogueArgs::phs).
hipError_t launch_pack(const FrameDev *frames, int n_frames, int max_M, const int *hlev, int level,
                       const HypState *hs, const PoseEval *pose, HypState *phs, PoseEval *ppose, int *pcount,
                       int *pclear0, int *pclear1, hipStream_t s);

// Spatial order of the anchors of every level with a permutation buffer
// (LevelDev::perm non-NULL and N <= kSortMaxN): the permutation, then the
// copies x, y, z, ref, ref_w of the caller's in_* arrays in that order.
// Grid: max_levels x n_frames sort blocks, then the copy; max_N bounds N.
hipError_t launch_anchor_sort(const FrameDev *frames, int n_frames, int max_levels, int max_N, hipStream_t s);

// Write results of every frame whose hypotheses have all finished and that
// has not been finalised yet (done_flag == 0), including the argmin.
hipError_t launch_finalize(const FrameDev *frames, int n_frames, const HypState *hs,
                           const int *hlev, hipStream_t s);

}  // namespace pilot

namespace pilot {

// The fixed device scratch of pilot_solve_static (pilot_static.hip):
// its size in bytes, the per-device set-up that takes the array's device
// address (call with `device` current), and that address (NULL before the
// set-up on that device).
size_t static_scratch_bytes();
hipError_t static_scratch_init(int device);
void *static_scratch(int device);

// Zero n_words 32-bit words on stream s with a fill kernel.
hipError_t launch_zero_words(void *p, int n_words, hipStream_t s);

}  // namespace pilot
