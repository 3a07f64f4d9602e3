/*
 * pilot.h -- C ABI of the MI355X (gfx950) sensor-prior featuremetric pose
 * solver: the multi-hypothesis, coarse-to-fine Levenberg-Marquardt
 * refinement of PiLoT v2 (arXiv 2606.31098), Method "Cross-View Learning",
 * "Multi-Sensor Prior Fusion" and "Multi-Sensor Optimization" (Eqs. (1)-(9)),
 * supplement "Multi-Hypothesis Refinement" and "Sensor-Prior Fusion in LM".
 *
 * Plain C: device pointers and sizes only, no framework types.  Every
 * function returns PILOT_OK (0) or a negative error code; nothing throws
 * across the ABI and nothing aborts the process.  On error,
 * pilot_last_error() names the offending field or the HIP failure.
 * Validation happens on the host before any launch: an EINVAL call launches
 * nothing.  Numerical trouble of one hypothesis (too few visible anchors,
 * non-finite values) is reported as its status, not as an error.
 *
 * Conventions
 *   pose       world->camera, double[12]: R row-major (9) then t (3),
 *              X_cam = R X_world + t (camera x right, y down, z forward).
 *   update     T <- Exp(dxi) T, dxi = (rho; omega), translation first
 *              (Eq. (9), applied as a left perturbation in the camera frame).
 *   pixels     integer coordinates are pixel centres; anchor j is visible
 *              at a level iff Z > z_min and 0 <= u <= W-1, 0 <= v <= H-1.
 *   features   channels-last H x W x C (f32, or bf16 bit patterns), already
 *              L2-normalised by the caller; reference descriptors N x C in the
 *              same dtype; both rounded to bf16 once by the caller if bf16.
 *   DSM        Hd x Wd f32 heights; sample (i, j) at (x0 + j gsd, y0 + i gsd),
 *              bilinear with clamp-to-edge (Eq. (6)).
 *   objective  per level l: sum_j rho_l(s_j) with s_j = w_j |r_j|^2
 *              (Eqs. (1)-(2)), w_j = ref_w[j] * qconf(u, v); anchors outside
 *              the view add rho_l(2 ref_w[j]); plus lambda_imu rho_g(|r_imu|^2)
 *              (Eq. (3)) and lambda_range rho_r(r_range^2) (Eqs. (4)-(6)),
 *              Eq. (7).  Normal equations use IRLS weights rho'(s)
 *              (Gauss-Newton), so g = J^T W r = 1/2 grad(cost).
 *   LM         per level: lambda = tau max diag H at the level's first
 *              linearisation; a step that lowers the total cost is accepted
 *              (lambda /= down, floor lambda_min_rel max diag H), otherwise
 *              rejected (lambda *= up; reaching lambda_max_rel max diag H
 *              stops the level, STALLED); an accepted step with
 *              |d rho| < step_tol_t and |d omega| < step_tol_r, or a
 *              candidate whose cost is within cost_tol * cost of the current
 *              one, ends the level (CONVERGED); every iteration, accepted or
 *              not, counts.  The prior scales are lambda_imu, lambda_range, or
 *              (adaptive_priors) set at each level's start and held for it.
 *   selection  best = lowest final cost among hypotheses that are neither
 *              degenerate nor pruned, ties to the lowest index, -1 if none.
 *
 * Threading: a pilot_ctx is used by one host thread at a time; several
 * contexts may share a device.  All work is enqueued on the context's stream
 * and is asynchronous: outputs are valid once the caller has synchronised
 * that stream.  The caller keeps every input alive until then.
 */
#ifndef PILOT_H
#define PILOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PILOT_MAX_LEVELS 4
#define PILOT_ABI_VERSION 1

enum {
    PILOT_OK = 0,
    PILOT_EINVAL = -1,        /* bad argument; message names the field      */
    PILOT_ENOMEM = -2,        /* workspace would exceed the HBM budget       */
    PILOT_EDEVICE = -3,       /* HIP runtime failure; message carries it     */
    PILOT_EAGAIN = -4,        /* serving: no slot or budget free right now   */
    PILOT_EUNSUPPORTED = -5   /* valid request the library does not handle   */
};

enum { PILOT_F32 = 0, PILOT_BF16 = 1 };
enum { PILOT_LOSS_CAUCHY = 0, PILOT_LOSS_HUBER = 1, PILOT_LOSS_L2 = 2 };
enum { PILOT_CONVERGED = 0, PILOT_MAX_ITERS = 1, PILOT_STALLED = 2, PILOT_DEGENERATE = 3, PILOT_PRUNED = 4 };

/* pilot_config.flags */
enum {
    PILOT_FLAG_NO_GRAPH = 1,  /* launch kernels directly instead of replaying a hipGraph */
    PILOT_FLAG_AUTOTUNE = 2,  /* time tile candidates on first use of a shape class     */
    PILOT_FLAG_PROFILE = 4,   /* time every pass launch with hipEvents (implies NO_GRAPH) */
    PILOT_FLAG_KEEP_ORDER = 8,/* walk anchors in the caller's order (no spatial sort)     */
    PILOT_FLAG_SORT_ANCHORS = 16 /* sort every level's anchors (2..16384 of them)          */
};

typedef struct pilot_ctx pilot_ctx;

typedef struct {
    int32_t device;             /* HIP device ordinal                                   */
    int32_t flags;              /* PILOT_FLAG_*                                         */
    void *stream;               /* hipStream_t for all work; NULL = null stream         */
    size_t hbm_budget_bytes;    /* pilot_solve: cap on workspace; serving: cap on the  */
                                /* summed pilot_admit_cost of admitted frames; 0 = none */
    const char *tune_cache;     /* autotune cache file (read at create, appended); NULL */
    int32_t max_slots;          /* serving slots; 0 = 64                                */
    int32_t reserved;
} pilot_config;

/* One pyramid level (Eq. (1) at level l, scaled intrinsics K_l).  The kernels
 * address each level's arrays with 32-bit byte offsets: the map (H*W*C
 * elements), the descriptors (N*C elements) and the per-cell table the library
 * builds (80*H*W bytes) must each be under 4 GiB, else PILOT_EINVAL.
 *
 * Anchor order: the sums of Eq. (1) run over the anchors in an order the
 * library picks, so the caller may list them in any order.  A level with
 * 2 <= N <= 16384 anchors and N * M >= 2^23 anchor-hypothesis pairs per pass
 * is walked in Morton order of the anchors' ground position (x, y on a
 * 256 x 256 grid over their bounding box; anchors of one cell in the
 * caller's order), from copies of x, y, z, ref and ref_w that the library
 * makes in its workspace at the start of every solve (pilot_solve,
 * pilot_solve_static, pilot_linearize) and at pilot_admit; the caller's
 * arrays are only read.  Neighbouring anchors then project to neighbouring
 * cells under one pose and share cache lines.  Results change only in the
 * rounding of the sums.  Below 2^23 pairs the sort costs more than it saves
 * and the caller's order is kept; PILOT_FLAG_SORT_ANCHORS sorts every level
 * of 2..16384 anchors, PILOT_FLAG_KEEP_ORDER none (it wins over the other). */
typedef struct {
    int32_t H, W, C;            /* C in {16, 32, 64, 128, 256}; H, W >= 2             */
    int32_t dtype;              /* PILOT_F32 or PILOT_BF16, for feat and ref         */
    const void *feat;           /* device, H*W*C, channels-last                      */
    const float *qconf;         /* device, H*W query confidence, or NULL (= 1)       */
    double K[4];                /* fx, fy, cx, cy of this level                      */
    int32_t N;                  /* anchors (>= 0)                                    */
    const float *x, *y, *z;     /* device, N each: world points (may be shared)      */
    const void *ref;            /* device, N*C reference descriptors                 */
    const float *ref_w;         /* device, N per-anchor weight >= 0, or NULL (= 1)   */
    int32_t iters;              /* LM iterations at this level (0..1000)             */
    int32_t loss_kind;          /* PILOT_LOSS_*                                      */
    double loss_scale;          /* b > 0                                              */
} pilot_level;

typedef struct {
    int32_t n_levels;           /* 1..PILOT_MAX_LEVELS, coarse -> fine                */
    pilot_level level[PILOT_MAX_LEVELS];
    int32_t M;                  /* hypotheses (1..65536)                              */
    const double *poses_in;     /* device, M*12                                       */
    /* gravity prior, Eq. (3) */
    int32_t use_gravity;
    int32_t gravity_loss_kind;
    double g_imu[3];            /* measured gravity direction, camera frame           */
    double g_world[3];          /* gravity direction, world frame (e.g. 0,0,-1)       */
    double lambda_imu;          /* >= 0                                               */
    double gravity_loss_scale;
    /* laser range prior, Eqs. (4)-(6) */
    int32_t use_range;
    int32_t range_loss_kind;
    double d_range;             /* metres, > 0                                        */
    double pc[2];               /* range pixel on the finest level                    */
    double lambda_range;        /* >= 0                                               */
    double range_loss_scale;
    const float *dsm;           /* device, Hd*Wd (required when use_range)            */
    int32_t Hd, Wd;
    double dsm_x0, dsm_y0, dsm_gsd;
    /* Levenberg-Marquardt control */
    double tau, lambda_up, lambda_down, lambda_min_rel, lambda_max_rel;
    double step_tol_t, step_tol_r, z_min;
    int32_t min_valid;          /* fewer visible anchors at a level start: DEGENERATE */
    int32_t adaptive_priors;    /* 0: fixed scales lambda_imu, lambda_range; else see below */
    /* Optional hypothesis generation on the device (supplement "Multi-Hypothesis
     * Refinement": hypotheses around the propagated prior in (x, y, yaw)).
     * When hyp_offsets is non-NULL, poses_in is ignored and hypothesis m is the
     * prior pose shifted by (dx, dy) metres in world x, y and rotated by dyaw
     * about the world z axis through its camera centre.  The prior is row
     * prior_best[0] of prior_poses (row 0 if prior_best is NULL or holds -1),
     * so a frame can start from the previous frame's result without a host
     * round trip. */
    const double *prior_poses;  /* device, rows of 12                              */
    const int32_t *prior_best;  /* device, 1 index, or NULL                         */
    const double *hyp_offsets;  /* device, M*3: dx, dy, dyaw                        */
    /* Top-K pruning (supplement, Multi-Hypothesis Refinement): once every
     * hypothesis has finished level prune_level, only the keep_top lowest
     * costs (ties to the lower index; degenerate ones excluded) continue to
     * the finer levels; the others end with status PILOT_PRUNED and keep
     * their pose and cost of that level.  keep_top = 0: no pruning.
     * Requires 0 <= prune_level < n_levels - 1 and M <= 8192. */
    int32_t keep_top;
    int32_t prune_level;
    /* Adaptive prior scales (supplement, Sensor-Prior Fusion in LM: the scales
     * of the gravity and range terms follow the relative gradient magnitudes
     * and residual-dependent gates).  With adaptive_priors != 0 each
     * hypothesis sets, at the start of every level (its pose there), for each
     * enabled prior s with base scale lambda_s, unit-scale gradient
     * g_s = J_s^T rho_s' r_s and residual norm |r_s|:
     *   alpha_s = lambda_s * min(1, alpha_ratio |g_vis| / (lambda_s |g_s|))
     *                      * min(1, (gate_s / |r_s|)^2)
     * (g_vis: gradient of the visual term; a factor is 1 when its parameter is
     * <= 0) and keeps it for the rest of the level, so the level's objective
     * is fixed.  All three must be finite and >= 0. */
    double alpha_ratio;
    double gravity_gate;        /* on |R g_world - g_imu|                           */
    double range_gate;          /* metres, on the range residual                      */
    /* Function tolerance of the LM control: a candidate whose total cost
     * differs from the current one by at most cost_tol * cost ends the level
     * as CONVERGED (the candidate is accepted if its cost is lower).  0 turns
     * the rule off; finite and >= 0. */
    double cost_tol;
} pilot_frame;

/* Caller-owned device buffers. */
typedef struct {
    double *poses_out;          /* M*12 final poses                                   */
    double *cost;               /* M final total cost (finest level)                  */
    int32_t *iterations;        /* M iterations executed, all levels                  */
    int32_t *status;            /* M PILOT_CONVERGED .. PILOT_PRUNED                  */
    int32_t *best;              /* 1 index (or -1)                                    */
    double *alpha;              /* M*2 or NULL: gravity and range scales each
                                   hypothesis used at the last level it started  */
} pilot_result;

typedef struct {
    uint64_t pairs[PILOT_MAX_LEVELS];      /* anchor x hypothesis evaluations, per level  */
    uint64_t pair_bytes[PILOT_MAX_LEVELS]; /* algorithmic gathered bytes (4 C s_f/pair)   */
    uint64_t launches[PILOT_MAX_LEVELS];   /* pass launches per level                     */
    double pass_ms[PILOT_MAX_LEVELS];      /* summed pass durations (PILOT_FLAG_PROFILE)  */
    uint64_t timed_launches[PILOT_MAX_LEVELS];
    uint64_t graph_replays, graph_captures;
} pilot_stats;

/* Create a context on cfg->device using cfg->stream.  *out is NULL on error;
 * the message is then available from pilot_last_error(NULL) (per thread). */
int pilot_create(pilot_ctx **out, const pilot_config *cfg);

/* Release the context and its workspace (synchronises its stream first). */
void pilot_destroy(pilot_ctx *ctx);

/* Message of the last failed call on ctx (or of this thread when ctx is
 * NULL); "" if none.  Valid until the next call on ctx. */
const char *pilot_last_error(const pilot_ctx *ctx);

/* Refine frames[0..n_frames) (each with its own hypotheses) coarse to fine
 * and select the best hypothesis of each frame (multi-hypothesis LM of the
 * Method's "Multi-Sensor Optimization").  results[i] receives frame i.
 * Enqueued on the context stream; no host synchronisation inside.  When a
 * pass has launches for frames of different tiles, they are forked through
 * events onto three streams the context owns and joined back before the
 * next pass, so the whole solve stays ordered after earlier and before
 * later work on the context stream. */
int pilot_solve(pilot_ctx *ctx, const pilot_frame *frames, int n_frames,
                const pilot_result *results);

/* pilot_solve for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, hosts that forbid hipMalloc): the
 * same schedule and kernels, with every piece of workspace (descriptors,
 * Gram tables, spatially ordered anchor copies, LM states, partial sums,
 * pass flags) carved from one fixed
 * device array of PILOT_STATIC_SCRATCH_BYTES per GPU that the library holds
 * from the first pilot_create on that GPU until the process ends.  Calls no
 * hipMalloc, hipFree, pinned-memory allocation or graph instantiation: the
 * descriptors are copied from host memory the context keeps.  Tiles come
 * from the context's tile database or the built-in heuristic (no autotuning,
 * whatever the flags), so with the same tiles the results equal pilot_solve's
 * bit for bit.  Frames whose workspace exceeds the scratch are refused with
 * PILOT_ENOMEM before anything is enqueued (the message gives the bytes
 * needed).  Every call on one GPU, from any context, uses that GPU's single
 * array and leaves its contents behind: calls whose work can overlap on one GPU
 * (contexts on different streams without an ordering between them) race and
 * give undefined results; calls ordered on one stream are safe. */
#define PILOT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int pilot_solve_static(pilot_ctx *ctx, const pilot_frame *frames, int n_frames,
                       const pilot_result *results);

/* Diagnostic: the damped system's terms at given poses, without an LM step.
 * For level `level` of `frame` and poses (device, frame->M*12): H21 (device,
 * M*21, upper triangle of the 6x6 row by row), g6 (M*6), cost (M), nvalid
 * (M visible anchors).  Total objective of Eq. (7) and its J^T W J,
 * J^T W r of Eq. (8).  frame->poses_in is ignored. */
int pilot_linearize(pilot_ctx *ctx, const pilot_frame *frame, int level,
                    const double *poses, double *H21, double *g6, double *cost,
                    int32_t *nvalid);

/* Geo-anchor lift on the device (supplement, Geo-anchor Construction; the
 * step before the optimisation): anchor j given at DSM-crop sample
 * coordinates uv[2j], uv[2j+1] (u along columns, v along rows) becomes
 *   x = x0 + u gsd,  y = y0 + v gsd,  z = D(u, v)  (bilinear, clamp-to-edge),
 * and its reference descriptor is the bilinear sample (clamp-to-edge) of the
 * Hr x Wr x C reference feature map ref_map (channels-last, dtype f32 or bf16)
 * at (scale (u + 1/2) - 1/2, scale (v + 1/2) - 1/2), i.e. a map with `scale`
 * pixels per DSM sample and aligned pixel centres.  Values are computed in
 * FP64 and rounded once to the output dtype (bf16: round-to-nearest-even).
 * All arrays are device memory; x, y, z may be NULL (e.g. a second pyramid
 * level reusing the same anchors); ref_out is N x C in the map's dtype.
 * C in {16, 32, 64, 128, 256}.  Enqueued on the context stream. */
int pilot_lift(pilot_ctx *ctx, const float *dsm, int32_t Hd, int32_t Wd, double x0, double y0,
               double gsd, const float *uv, int32_t N, const void *ref_map, int32_t Hr, int32_t Wr,
               int32_t C, int32_t dtype, double scale, float *x, float *y, float *z, void *ref_out);

/* ---------------------------------------------------------------------
 * Serving (continuous batching).  A frame is admitted into a slot when a
 * slot and HBM budget are free; pilot_step advances every active slot by
 * one LM pass (each slot at its own level and iteration); pilot_poll
 * reports completion and frees the slot.  Results are written to the
 * result buffers given at admission.  Admission accounts the frame's input
 * bytes (as declared by its sizes) plus its workspace against the budget.
 * ------------------------------------------------------------------- */

/* Bytes a frame would hold against the budget (inputs + workspace). */
int pilot_admit_cost(pilot_ctx *ctx, const pilot_frame *frame, size_t *bytes);

/* Admit a frame.  PILOT_EAGAIN (nothing enqueued) when no slot is free or
 * the budget would be exceeded.  Hypotheses (poses_in, or generated from the
 * prior) are read on the stream at admission; the frame's other inputs must
 * stay valid until pilot_poll reports the slot finished.  A context with
 * active slots accepts no pilot_solve / pilot_linearize. */
int pilot_admit(pilot_ctx *ctx, const pilot_frame *frame, const pilot_result *result,
                int *slot);

/* One LM pass for every active slot (enqueued on the stream), followed by
 * the result write-out of slots that finished.  At most two steps are in
 * flight: a third call first waits for the oldest. */
int pilot_step(pilot_ctx *ctx);

/* 1 if a completed step has seen the slot's frame finish (its results are
 * then written and the slot is free for reuse), 0 if not yet, negative on
 * error.  Does not block. */
int pilot_poll(pilot_ctx *ctx, int slot);

/* Block until every enqueued step has completed. */
int pilot_sync(pilot_ctx *ctx);

/* Number of active slots and budget bytes in use. */
int pilot_serving_state(pilot_ctx *ctx, int *active_slots, size_t *bytes_in_use);

/* Counters since creation (or the last reset). */
int pilot_get_stats(pilot_ctx *ctx, pilot_stats *out, int reset);

/* Autotune the pass kernel for the level shapes of `frame` now: every
 * candidate tile (kernel variant, lane-group width, anchors per lane group,
 * grid) is timed by eager solves of `frame` with hipEvents around each pass,
 * and each level shape (C, dtype, log2 N, log2 M, log2 H*W) keeps the
 * candidate with the lowest summed pass time; the choice is cached in the
 * context and appended to the tune cache file.  Synchronises the stream;
 * leaves the counters of pilot_get_stats as they were.  Shapes already
 * tuned are skipped. */
int pilot_autotune(pilot_ctx *ctx, const pilot_frame *frame);

/* "G=8 PPG=8 BPC=2 V=3 tuned=1" style description of the tile choice for a
 * level shape (C channels, dtype, N anchors, M hypotheses, HW = H*W map
 * pixels). */
int pilot_tile_choice(pilot_ctx *ctx, int C, int dtype, int N, int M, int64_t HW, char *buf, int buflen);

int pilot_abi_version(void);

/* sizeof of an ABI struct by name ("pilot_frame", "pilot_level",
 * "pilot_result", "pilot_config", "pilot_stats"); 0 if unknown.  Lets a
 * binding check its struct layout against the library's. */
size_t pilot_sizeof(const char *name);

#ifdef __cplusplus
}
#endif
#endif /* PILOT_H */
