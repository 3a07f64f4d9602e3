// pilot_runtime.cpp -- host runtime and C ABI of libpilot.
//
// A solve is planned on the host (validation, tile choice, work lists),
// its descriptors are copied to the device once, and the whole
// coarse-to-fine LM schedule -- init, then per level (1 + iters) x
// [pass kernel -> epilogue kernel], then finalize -- is enqueued on the
// context stream, replayed from a cached hipGraph when a solve with the same
// plan shape was seen before.  No device->host traffic inside a solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pilot.h"
#include "pilot_kernels.h"

using namespace pilot;

namespace {

thread_local std::string g_thread_err;

constexpr int kStatClasses = 64;

int class_index(int level, int C, int dtype)
{
    int ci = C == 16 ? 0 : C == 32 ? 1 : C == 64 ? 2 : C == 128 ? 3 : 4;
    return level * 10 + ci * 2 + dtype;
}

int elem_size(int dtype) { return dtype == PILOT_BF16 ? 2 : 4; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct LaunchGroup {
    int level = 0, C = 0, dtype = 0;
    TileConfig tc{};
    int item_off = 0, n_items = 0;
    int tile_off = 0, n_tiles = 0;
    int passes = 0;
    int stat_class = 0;
    size_t partial_off = 0;   // its partial records in the partials buffer (floats)
};

// Side streams of a context: the launch groups of one pass run concurrently
// on the context's stream and up to kSideStreams more, forked and joined
// through events around every pass (captured into the solve's graph).
constexpr int kSideStreams = 3;

struct Plan {
    std::vector<FrameDev> frames;
    std::vector<WorkItem> items;
    std::vector<TileItem> tiles;
    std::vector<LaunchGroup> groups;
    int total_hyps = 0, max_M = 0, max_levels = 0;
    size_t partial_floats = 0;
    std::string key;
    // Gram tables of the (frame, level) pairs whose tiles use a Gram pass variant (3 to 10)
    struct GramJob {
        int frame = 0, level = 0;
        size_t offset = 0;
        int fmt = 0;
    };
    std::vector<GramJob> gram_jobs;
    size_t gram_bytes = 0;
    // the (frame, level) pairs whose anchors are walked in spatial order, with
    // the offset of their copies in the anchor buffer
    struct AnchorJob {
        int frame = 0, level = 0;
        size_t offset = 0;
    };
    std::vector<AnchorJob> anchor_jobs;
    size_t anchor_bytes = 0;
    int anchor_max_N = 0;
    int flag_stride = 1;         // pass flags per level (most passes of a level's groups + 1)
};

struct TimedLaunch {
    hipEvent_t a = nullptr, b = nullptr;
    int level = 0, cls = 0;
};

struct ServingSlot {
    bool active = false;
    int M = 0;
    int hyp_base = 0;
    size_t bytes = 0;
    uint64_t admit_step = 0;
    pilot_frame frame{};
    FrameDev dev{};      // host copy of the slot's device descriptor
    DevBuf gram;         // Gram tables of the slot's Gram-variant levels (kept for reuse)
    DevBuf anch;         // the slot's anchors in spatial order (kept for reuse)
};

constexpr int kFlagRing = 4;

}  // namespace

struct pilot_ctx {
    int device = 0;
    int flags = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSideStreams] = {};
    size_t budget = 0;
    std::string tune_cache;
    int max_slots = 64;
    int ncu = 256;
    std::string err;

    // workspace
    DevBuf desc, hs, pose, hlev, partials, pairs, gram, anch, passflag, phs, ppose, pcount;
    size_t ws_bytes = 0;
    unsigned generation = 0;
    // the bytes of the last descriptor upload and the workspace generation
    // it was made in: a solve whose descriptors are the same skips the copy
    std::vector<char> desc_img, desc_next;
    unsigned desc_gen = ~0u;
    // host image of the descriptors of the last pilot_solve_static call
    std::vector<char> static_img;

    // pinned staging ring
    struct Stage {
        void *p = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    } stage[2];
    int stage_next = 0;

    std::unordered_map<std::string, hipGraphExec_t> graphs;
    std::map<std::string, TileConfig> tuned;

    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    double pass_ms[kStatClasses] = {0};
    uint64_t timed_launches[kStatClasses] = {0};
    uint64_t launches[kStatClasses] = {0};
    uint64_t graph_replays = 0, graph_captures = 0;

    // serving
    std::vector<ServingSlot> slots;
    DevBuf s_frames, s_desc, s_done;
    int arena_cap = 0;                          // hypotheses in the slot arena
    std::vector<std::pair<int, int>> arena_free;   // (offset, length), sorted
    size_t serv_bytes = 0;
    bool serv_dirty = true;
    Plan serv_plan;                             // work lists over the active slots
    uint64_t steps_enqueued = 0;
    struct FlagBuf {
        int *host = nullptr;
        hipEvent_t ev = nullptr;
        uint64_t step = 0;
        bool used = false;
    } flagbuf[kFlagRing];
    int n_active() const
    {
        int n = 0;
        for (const ServingSlot &x : slots) n += x.active ? 1 : 0;
        return n;
    }
};

namespace {

int fail(pilot_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_thread_err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), PILOT_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                                    \
    } while (0)

bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------- validation
int validate_frame(pilot_ctx *ctx, const pilot_frame *f, int fi, bool need_poses)
{
    if (!f) return fail(ctx, PILOT_EINVAL, "frames[%d]: NULL", fi);
    if (f->n_levels < 1 || f->n_levels > PILOT_MAX_LEVELS)
        return fail(ctx, PILOT_EINVAL, "frames[%d].n_levels: must be 1..%d (got %d)", fi, PILOT_MAX_LEVELS, f->n_levels);
    if (f->M < 1 || f->M > 65536) return fail(ctx, PILOT_EINVAL, "frames[%d].M: must be 1..65536 (got %d)", fi, f->M);
    if (need_poses && !f->poses_in && !(f->hyp_offsets && f->prior_poses))
        return fail(ctx, PILOT_EINVAL, "frames[%d].poses_in: NULL (and no prior_poses + hyp_offsets)", fi);
    for (int l = 0; l < f->n_levels; ++l) {
        const pilot_level &L = f->level[l];
        if (L.H < 2 || L.W < 2)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].H/W: must be >= 2 (got %dx%d)", fi, l, L.H, L.W);
        if (L.dtype != PILOT_F32 && L.dtype != PILOT_BF16)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].dtype: must be PILOT_F32 or PILOT_BF16", fi, l);
        if (L.C != 16 && L.C != 32 && L.C != 64 && L.C != 128 && L.C != 256) {
            if (L.C > 0 && L.C % 8 == 0 && L.C <= 512)
                return fail(ctx, PILOT_EUNSUPPORTED, "frames[%d].level[%d].C: %d channels has no kernel (16, 32, 64, 128, 256)", fi, l, L.C);
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].C: must be 16, 32, 64, 128 or 256 (got %d)", fi, l, L.C);
        }
        // the kernels address maps, descriptors and per-cell tables with 32-bit byte offsets
        if ((double)L.H * L.W * L.C * elem_size(L.dtype) >= 4294967296.0 || (double)L.H * L.W * 80.0 >= 4294967296.0)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d]: the map (H*W*C elements) must be under 4 GiB", fi, l);
        if (!L.feat) return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].feat: NULL", fi, l);
        if (!aligned16(L.feat)) return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].feat: must be 16-byte aligned", fi, l);
        if (!finite_all(L.K, 4) || !(L.K[0] > 0) || !(L.K[1] > 0))
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].K: fx, fy must be > 0 and all finite", fi, l);
        if (L.N < 0 || (double)L.N * L.C * elem_size(L.dtype) >= 4294967296.0)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].N: must be >= 0 with N*C elements under 4 GiB (got %d)",
                        fi, l, L.N);
        if (L.N > 0) {
            if (!L.x || !L.y || !L.z) return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].x/y/z: NULL", fi, l);
            if (!L.ref) return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].ref: NULL", fi, l);
            if (!aligned16(L.ref)) return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].ref: must be 16-byte aligned", fi, l);
        }
        if (L.iters < 0 || L.iters > 1000)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].iters: must be 0..1000 (got %d)", fi, l, L.iters);
        if (L.loss_kind < 0 || L.loss_kind > 2)
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].loss_kind: must be PILOT_LOSS_*", fi, l);
        if (!(L.loss_scale > 0) || !std::isfinite(L.loss_scale))
            return fail(ctx, PILOT_EINVAL, "frames[%d].level[%d].loss_scale: must be finite and > 0", fi, l);
    }
    if (f->use_gravity) {
        if (!finite_all(f->g_imu, 3) || !finite_all(f->g_world, 3))
            return fail(ctx, PILOT_EINVAL, "frames[%d].g_imu/g_world: must be finite", fi);
        if (!(f->lambda_imu >= 0) || !std::isfinite(f->lambda_imu))
            return fail(ctx, PILOT_EINVAL, "frames[%d].lambda_imu: must be finite and >= 0", fi);
        if (f->gravity_loss_kind < 0 || f->gravity_loss_kind > 2 || !(f->gravity_loss_scale > 0) ||
            !std::isfinite(f->gravity_loss_scale))
            return fail(ctx, PILOT_EINVAL, "frames[%d].gravity_loss_kind/scale: invalid", fi);
    }
    if (f->use_range) {
        if (!f->dsm) return fail(ctx, PILOT_EINVAL, "frames[%d].dsm: NULL with use_range", fi);
        if (f->Hd < 2 || f->Wd < 2) return fail(ctx, PILOT_EINVAL, "frames[%d].Hd/Wd: must be >= 2", fi);
        if (!(f->dsm_gsd > 0) || !std::isfinite(f->dsm_gsd) || !std::isfinite(f->dsm_x0) || !std::isfinite(f->dsm_y0))
            return fail(ctx, PILOT_EINVAL, "frames[%d].dsm_x0/y0/gsd: invalid", fi);
        if (!(f->d_range > 0) || !std::isfinite(f->d_range))
            return fail(ctx, PILOT_EINVAL, "frames[%d].d_range: must be finite and > 0", fi);
        if (!finite_all(f->pc, 2)) return fail(ctx, PILOT_EINVAL, "frames[%d].pc: must be finite", fi);
        if (!(f->lambda_range >= 0) || !std::isfinite(f->lambda_range))
            return fail(ctx, PILOT_EINVAL, "frames[%d].lambda_range: must be finite and >= 0", fi);
        if (f->range_loss_kind < 0 || f->range_loss_kind > 2 || !(f->range_loss_scale > 0) ||
            !std::isfinite(f->range_loss_scale))
            return fail(ctx, PILOT_EINVAL, "frames[%d].range_loss_kind/scale: invalid", fi);
    }
    if (!(f->tau > 0) || !std::isfinite(f->tau)) return fail(ctx, PILOT_EINVAL, "frames[%d].tau: must be finite and > 0", fi);
    if (!(f->lambda_up > 1) || !std::isfinite(f->lambda_up)) return fail(ctx, PILOT_EINVAL, "frames[%d].lambda_up: must be > 1", fi);
    if (!(f->lambda_down >= 1) || !std::isfinite(f->lambda_down)) return fail(ctx, PILOT_EINVAL, "frames[%d].lambda_down: must be >= 1", fi);
    if (!(f->lambda_min_rel >= 0) || !(f->lambda_max_rel > f->lambda_min_rel) || !std::isfinite(f->lambda_max_rel))
        return fail(ctx, PILOT_EINVAL, "frames[%d].lambda_min_rel/lambda_max_rel: need 0 <= min < max < inf", fi);
    if (!(f->step_tol_t >= 0) || !(f->step_tol_r >= 0) || !std::isfinite(f->step_tol_t) || !std::isfinite(f->step_tol_r))
        return fail(ctx, PILOT_EINVAL, "frames[%d].step_tol_t/r: must be finite and >= 0", fi);
    if (!(f->z_min >= 0) || !std::isfinite(f->z_min)) return fail(ctx, PILOT_EINVAL, "frames[%d].z_min: must be finite and >= 0", fi);
    if (f->min_valid < 0) return fail(ctx, PILOT_EINVAL, "frames[%d].min_valid: must be >= 0", fi);
    if (f->keep_top < 0) return fail(ctx, PILOT_EINVAL, "frames[%d].keep_top: must be >= 0", fi);
    if (!std::isfinite(f->cost_tol) || f->cost_tol < 0.0)
        return fail(ctx, PILOT_EINVAL, "frames[%d].cost_tol: must be finite and >= 0", fi);
    if (f->adaptive_priors) {
        const double v[3] = {f->alpha_ratio, f->gravity_gate, f->range_gate};
        const char *nm[3] = {"alpha_ratio", "gravity_gate", "range_gate"};
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(v[i]) || v[i] < 0.0)
                return fail(ctx, PILOT_EINVAL, "frames[%d].%s: must be finite and >= 0", fi, nm[i]);
    }
    if (f->keep_top > 0) {
        if (f->prune_level < 0 || f->prune_level >= f->n_levels - 1)
            return fail(ctx, PILOT_EINVAL, "frames[%d].prune_level: must be 0..n_levels-2 with keep_top > 0", fi);
        if (f->M > 8192) return fail(ctx, PILOT_EUNSUPPORTED, "frames[%d].keep_top: pruning supports M <= 8192", fi);
    }
    return PILOT_OK;
}

// ---------------------------------------------------------------- workspace
// Grow a workspace buffer.  Solve workspace is charged against the HBM
// budget; serving buffers (check_budget = false) are covered by the
// per-frame admission costs instead.
int ensure(pilot_ctx *ctx, DevBuf &b, size_t bytes, bool zero = false, bool check_budget = true)
{
    if (bytes <= b.cap) return PILOT_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 4095) & ~(size_t)4095;
    size_t total = ctx->ws_bytes - b.cap + want;
    if (check_budget && ctx->budget && total > ctx->budget) {
        want = bytes;
        total = ctx->ws_bytes - b.cap + want;
        if (total > ctx->budget)
            return fail(ctx, PILOT_ENOMEM, "workspace of %zu bytes exceeds the HBM budget of %zu bytes", total, ctx->budget);
    }
    if (b.p) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        HIPCHK(ctx, hipFree(b.p));
        b.p = nullptr;
    }
    HIPCHK(ctx, hipMalloc(&b.p, want));
    if (zero) HIPCHK(ctx, hipMemset(b.p, 0, want));
    ctx->ws_bytes = total;
    b.cap = want;
    ctx->generation++;
    return PILOT_OK;
}

void *stage_acquire(pilot_ctx *ctx, size_t bytes, int *which, int *rc)
{
    *rc = PILOT_OK;
    pilot_ctx::Stage &s = ctx->stage[ctx->stage_next];
    *which = ctx->stage_next;
    ctx->stage_next ^= 1;
    if (s.pending) {
        hipError_t e = hipEventSynchronize(s.ev);
        if (e != hipSuccess) {
            *rc = fail(ctx, PILOT_EDEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
            return nullptr;
        }
        s.pending = false;
    }
    if (bytes > s.cap) {
        if (s.p) hipHostFree(s.p);
        s.p = nullptr;
        size_t want = std::max(bytes, (size_t)1 << 16);
        hipError_t e = hipHostMalloc(&s.p, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            s.cap = 0;
            *rc = fail(ctx, PILOT_EDEVICE, "hipHostMalloc: %s", hipGetErrorString(e));
            return nullptr;
        }
        s.cap = want;
    }
    return s.p;
}

// ---------------------------------------------------------------- tiles
// pass variants 3 to 10 read per-cell Gram tables: 10 doubles per cell
// (format 0) or, for variants 9 and 10 on bf16 maps, 12 floats (format 1;
// on f32 maps those variants run variants 3 and 4)
bool uses_gram(const TileConfig &tc) { return tc.variant >= 3 && tc.variant <= 10; }
int gram_format(const TileConfig &tc, int dtype) { return (tc.variant >= 9 && dtype == PILOT_BF16) ? 1 : 0; }

int log2_bucket(int n)
{
    int b = 0;
    while ((1 << (b + 1)) <= std::max(n, 1)) ++b;
    return b;
}

// Tile-database key of a level shape: channels, dtype and log2 buckets of
// the anchors, hypotheses and map pixels.
std::string tune_key(int C, int dtype, int N, int M, long HW)
{
    std::ostringstream o;
    o << "C" << C << "_d" << dtype << "_N" << log2_bucket(N) << "_M" << log2_bucket(M) << "_P"
      << log2_bucket((int)std::min<long>(HW, 1L << 30)) << "_v3";
    return o.str();
}

TileConfig heuristic_tile(const pilot_ctx *ctx, int C, int dtype, int N, int M, long HW)
{
    TileConfig tc{};
    tc.G = (C >= 128) ? 8 : 4;      // measured: G = 4 up to C = 64, G = 8 at C = 128
    const int NG = kBlock / tc.G;
    const long ht = (M + tc.G - 1) / tc.G;
    tc.PPG = 1;
    for (int ppg : {16, 8, 4, 2, 1}) {
        const long items = ht * std::max(1, (N + NG * ppg - 1) / (NG * ppg));
        tc.PPG = ppg;
        if (items >= 4L * ctx->ncu) break;
    }
    tc.grid = 0;   // one block per item
    return tc;
}

// Lane groups of 4, 8 or 16 lanes exist for every variant; variants 9 and 10
// on bf16 maps also take 1 lane (C <= 32) and 2 lanes (C <= 64).
bool tile_ok(const TileConfig &tc, int C, int dtype)
{
    if (tc.G == 4 || tc.G == 8 || tc.G == 16) return true;
    if (dtype != PILOT_BF16 || tc.variant < 9) return false;
    return (tc.G == 1 && C <= 32) || (tc.G == 2 && C <= 64);
}

TileConfig choose_tile(const pilot_ctx *ctx, int C, int dtype, int N, int M, long HW)
{
    auto it = ctx->tuned.find(tune_key(C, dtype, N, M, HW));
    if (it != ctx->tuned.end() && tile_ok(it->second, C, dtype)) return it->second;
    return heuristic_tile(ctx, C, dtype, N, M, HW);
}

// Serving slots use the same tiles as solves (a slot's Gram tables are built
// when its frame is admitted).
TileConfig serving_tile(const pilot_ctx *ctx, int C, int dtype, int N, int M, long HW)
{
    return choose_tile(ctx, C, dtype, N, M, HW);
}

size_t gram_table_bytes(const pilot_level &L, int fmt)
{
    const size_t per_cell = fmt == 1 ? 12 * sizeof(float) : 10 * sizeof(double);
    return ((size_t)L.H * L.W * per_cell + 255) & ~(size_t)255;
}

int n_ptiles_of(const TileConfig &tc, int N)
{
    const int P = (kBlock / tc.G) * tc.PPG;
    return std::max(1, (N + P - 1) / P);
}

int grid_of(const pilot_ctx *ctx, const TileConfig &tc, int n_items)
{
    if (tc.grid <= 0) return std::max(1, n_items);
    return std::max(1, std::min(n_items, tc.grid * ctx->ncu));
}

void fill_frame_dev(FrameDev &d, const pilot_frame &f, const pilot_result *r, int hyp_base)
{
    memset(&d, 0, sizeof d);
    for (int l = 0; l < f.n_levels; ++l) {
        const pilot_level &L = f.level[l];
        LevelDev &o = d.lv[l];
        o.feat = L.feat;
        o.qconf = L.qconf;
        o.x = L.x;
        o.y = L.y;
        o.z = L.z;
        o.ref = L.ref;
        o.ref_w = L.ref_w;
        o.fx = L.K[0];
        o.fy = L.K[1];
        o.cx = L.K[2];
        o.cy = L.K[3];
        o.H = L.H;
        o.W = L.W;
        o.C = L.C;
        o.N = L.N;
        o.iters = L.iters;
        o.loss_kind = L.loss_kind;
        o.loss_b = L.loss_scale;
        o.dtype = L.dtype;
    }
    d.n_levels = f.n_levels;
    d.M = f.M;
    d.hyp_base = hyp_base;
    d.use_g = f.use_gravity ? 1 : 0;
    d.grav_kind = f.gravity_loss_kind;
    d.grav_b = f.gravity_loss_scale;
    d.lam_imu = f.lambda_imu;
    for (int i = 0; i < 3; ++i) {
        d.g_imu[i] = f.g_imu[i];
        d.g_world[i] = f.g_world[i];
    }
    d.use_r = f.use_range ? 1 : 0;
    d.range_kind = f.range_loss_kind;
    d.range_b = f.range_loss_scale;
    d.lam_range = f.lambda_range;
    {
        // unit ray of the range pixel through the finest level's intrinsics (Eq. (4))
        const pilot_level &Lf = f.level[f.n_levels - 1];
        double ray[3] = {(f.pc[0] - Lf.K[2]) / Lf.K[0], (f.pc[1] - Lf.K[3]) / Lf.K[1], 1.0};
        const double n = std::sqrt(ray[0] * ray[0] + ray[1] * ray[1] + ray[2] * ray[2]);
        for (int i = 0; i < 3; ++i) d.q[i] = f.use_range ? f.d_range * ray[i] / n : 0.0;
    }
    d.dsm = f.dsm;
    d.Hd = f.Hd;
    d.Wd = f.Wd;
    d.dsm_x0 = f.dsm_x0;
    d.dsm_y0 = f.dsm_y0;
    d.dsm_gsd = f.dsm_gsd;
    d.tau = f.tau;
    d.up = f.lambda_up;
    d.down = f.lambda_down;
    d.lmin_rel = f.lambda_min_rel;
    d.lmax_rel = f.lambda_max_rel;
    d.tol_t = f.step_tol_t;
    d.tol_r = f.step_tol_r;
    d.keep_top = f.keep_top;
    d.prune_level = f.prune_level;
    d.z_min = f.z_min;
    d.min_valid = f.min_valid;
    d.adaptive = f.adaptive_priors ? 1 : 0;
    d.alpha_ratio = f.alpha_ratio;
    d.grav_gate = f.gravity_gate;
    d.range_gate = f.range_gate;
    d.cost_tol = f.cost_tol;
    d.poses_in = f.poses_in;
    d.prior_poses = f.prior_poses;
    d.prior_best = f.prior_best;
    d.hyp_offsets = f.hyp_offsets;
    if (r) {
        d.poses_out = r->poses_out;
        d.cost_out = r->cost;
        d.iters_out = r->iterations;
        d.status_out = r->status;
        d.best_out = r->best;
        d.alpha_out = r->alpha;
    }
}

// Anchors in spatial order (the sort and copy kernels): levels of 2 to
// kSortMaxN anchors with at least kSortMinPairs anchor-hypothesis pairs per
// pass, or all of them under PILOT_FLAG_SORT_ANCHORS; none under
// PILOT_FLAG_KEEP_ORDER.  Measured on MI355X: a 16384-anchor sort costs about
// 60 us and a 8192-anchor one 35 us; 1024 hypotheses over 16384 anchors
// solve 1.3 % faster sorted than in raster order (6.5 % than shuffled),
// 256 over 8192 2 % slower.
constexpr long kSortMinPairs = 1L << 23;

bool sorts_anchors(const pilot_ctx *ctx, const pilot_level &L, int M)
{
    if ((ctx->flags & PILOT_FLAG_KEEP_ORDER) || L.N < 2 || L.N > kSortMaxN) return false;
    return (ctx->flags & PILOT_FLAG_SORT_ANCHORS) || (long)L.N * M >= kSortMinPairs;
}

// Bytes of a level's spatially ordered copy: x, y, z, the permutation, ref_w
// when given, then the reference rows, each 256-byte aligned.
size_t anchor_copy_bytes(const pilot_level &L)
{
    const size_t n4 = align256((size_t)L.N * 4);
    return 4 * n4 + (L.ref_w ? n4 : 0) + align256((size_t)L.N * L.C * elem_size(L.dtype));
}

// Point a level at its copy at device address p (anchor_copy_bytes(L) bytes),
// keeping the caller's arrays as the sort's input.
void place_anchor_copy(LevelDev &o, char *p)
{
    const size_t n4 = align256((size_t)o.N * 4);
    o.in_x = o.x;
    o.in_y = o.y;
    o.in_z = o.z;
    o.in_w = o.ref_w;
    o.in_ref = o.ref;
    o.x = (const float *)p;
    o.y = (const float *)(p + n4);
    o.z = (const float *)(p + 2 * n4);
    o.perm = (int *)(p + 3 * n4);
    size_t off = 4 * n4;
    if (o.in_w) {
        o.ref_w = (const float *)(p + off);
        off += n4;
    }
    o.ref = p + off;
}

// The packed-tile threshold of a tile (use_packed): mode 0 never packs, mode
// 1 packs when the tiles that may be active hold more work items than four
// per CU, mode 2 always.
int pack_min_of(const pilot_ctx *ctx, const TileConfig &tc)
{
    if (!uses_gram(tc) || tc.pack == 0) return INT_MAX;
    return tc.pack == 2 ? 0 : 4 * ctx->ncu;
}

// Build the schedule: per level, frames grouped by (C, dtype), each group a
// list of (hypothesis tile x anchor tile) work items.
void build_plan(const pilot_ctx *ctx, const pilot_frame *frames, int n, const pilot_result *results,
                int only_level, Plan &plan)
{
    plan.frames.resize(n);
    int base = 0;
    for (int i = 0; i < n; ++i) {
        fill_frame_dev(plan.frames[i], frames[i], results ? &results[i] : nullptr, base);
        base += frames[i].M;
        plan.max_M = std::max(plan.max_M, frames[i].M);
        plan.max_levels = std::max(plan.max_levels, frames[i].n_levels);
    }
    plan.total_hyps = base;
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < frames[i].n_levels; ++l) {
            const pilot_level &L = frames[i].level[l];
            if ((only_level >= 0 && l != only_level) || !sorts_anchors(ctx, L, frames[i].M)) continue;
            plan.anchor_jobs.push_back(Plan::AnchorJob{i, l, plan.anchor_bytes});
            plan.anchor_bytes += anchor_copy_bytes(L);
            plan.anchor_max_N = std::max(plan.anchor_max_N, L.N);
        }
    std::ostringstream key;
    // a captured graph bakes in the grids of the anchor sort and copy
    key << "n" << n << "_h" << base << "_m" << plan.max_M << "_a" << plan.anchor_max_N << "." << plan.anchor_jobs.size();
    for (int l = 0; l < plan.max_levels; ++l) {
        if (only_level >= 0 && l != only_level) continue;
        // each frame's tile depends on its own shape only, so its sums (and
        // results) are the same alone or batched with any other frames;
        // frames whose tiles share a kernel instantiation (C, dtype, G,
        // variant) share a launch, each walked with its own anchors per lane
        // group and packing rule (LevelDev::ppg, pack_min)
        std::map<std::array<int, 4>, std::vector<int>> by_class;
        std::vector<TileConfig> tci(n);
        size_t level_partials = 0;
        for (int i = 0; i < n; ++i)
            if (l < frames[i].n_levels) {
                const pilot_level &L = frames[i].level[l];
                tci[i] = choose_tile(ctx, L.C, L.dtype, L.N, frames[i].M, (long)L.H * L.W);
                LevelDev &o = plan.frames[i].lv[l];
                o.ppg = tci[i].PPG;
                o.pack_min = pack_min_of(ctx, tci[i]);
                by_class[{L.C, L.dtype, tci[i].G, tci[i].variant}].push_back(i);
            }
        for (auto &kv : by_class) {
            LaunchGroup g{};
            g.level = l;
            g.C = kv.first[0];
            g.dtype = kv.first[1];
            int iters = 0, pack = 0;
            for (int i : kv.second) {
                iters = std::max(iters, frames[i].level[l].iters);
                pack = std::max(pack, tci[i].pack);
            }
            g.item_off = (int)plan.items.size();
            g.tile_off = (int)plan.tiles.size();
            int most = -1, most_items = -1;    // the launch takes the grid rule of the frame with most items
            for (int i : kv.second) {
                const TileConfig &t = tci[i];
                const int nht = (frames[i].M + t.G - 1) / t.G;
                const int npt = n_ptiles_of(t, frames[i].level[l].N);
                if (nht * npt > most_items) most = i, most_items = nht * npt;
                for (int ht = 0; ht < nht; ++ht) {
                    const int h0 = ht * t.G, nh = std::min(t.G, frames[i].M - h0);
                    plan.tiles.push_back(
                        TileItem{i, ht, (int)plan.items.size() - g.item_off, npt, plan.frames[i].hyp_base + h0, nh});
                    for (int pt = 0; pt < npt; ++pt)
                        plan.items.push_back(WorkItem{i, plan.frames[i].hyp_base + h0, pt, nh});
                }
            }
            g.tc = tci[most];
            g.tc.pack = pack;                   // packed lists when any frame of the launch packs
            g.n_items = (int)plan.items.size() - g.item_off;
            g.n_tiles = (int)plan.tiles.size() - g.tile_off;
            g.passes = (only_level >= 0) ? 1 : 1 + iters;
            plan.flag_stride = std::max(plan.flag_stride, g.passes + 1);
            g.stat_class = class_index(l, g.C, g.dtype);
            g.tc.grid = grid_of(ctx, g.tc, g.n_items);
            if (uses_gram(g.tc))
                for (int i : kv.second) {
                    const pilot_level &Li = frames[i].level[l];
                    const int fmt = gram_format(g.tc, Li.dtype);
                    plan.gram_jobs.push_back(Plan::GramJob{i, l, plan.gram_bytes, fmt});
                    plan.gram_bytes += gram_table_bytes(Li, fmt);
                    // a captured graph bakes in each Gram launch's grid and instantiation
                    key << "|g" << i << "." << l << ":" << Li.H << "x" << Li.W << "x" << Li.C << "d" << Li.dtype
                        << "f" << fmt;
                }
            // the groups of a level run concurrently: disjoint partial records
            g.partial_off = level_partials;
            level_partials += (size_t)g.n_items * g.tc.G * kNV;
            plan.partial_floats = std::max(plan.partial_floats, level_partials);
            plan.groups.push_back(g);
            key << "|l" << l << "c" << g.C << "d" << g.dtype << "G" << g.tc.G << "g" << g.tc.grid << "v"
                << g.tc.variant << "k" << (g.tc.pack != 0) << "i" << g.n_items << "t" << g.n_tiles << "s" << g.passes;
        }
    }
    plan.key = key.str();
}

hipEvent_t pool_event(pilot_ctx *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct DevPtrs {
    FrameDev *frames = nullptr;
    WorkItem *items = nullptr;
    TileItem *tiles = nullptr;
};

// Device workspace a schedule runs on: the context's buffers, or the fixed
// scratch of pilot_solve_static.
struct Ws {
    HypState *hs = nullptr;
    PoseEval *pose = nullptr;
    int *hlev = nullptr;
    float *partials = nullptr;
    unsigned long long *pairs = nullptr;
    int *passflag = nullptr;
    // packed hypothesis tiles, three rotating buffers (pass k of a level reads
    // buffer k % 3, its epilogue appends to (k + 1) % 3, and the pass clears the
    // counts of (k + 2) % 3): per frame the LM states of the hypotheses still at
    // the level, their poses under evaluation and their number
    HypState *phs = nullptr;     // 3 x hyps
    PoseEval *ppose = nullptr;   // 3 x hyps
    int *pcount = nullptr;       // 3 x frames
    int hyps = 0, frames = 0;    // buffer strides
};

Ws ws_of(const pilot_ctx *ctx)
{
    Ws w;
    w.hs = (HypState *)ctx->hs.p;
    w.pose = (PoseEval *)ctx->pose.p;
    w.hlev = (int *)ctx->hlev.p;
    w.partials = (float *)ctx->partials.p;
    w.pairs = (unsigned long long *)ctx->pairs.p;
    w.passflag = (int *)ctx->passflag.p;
    w.phs = (HypState *)ctx->phs.p;
    w.ppose = (PoseEval *)ctx->ppose.p;
    w.pcount = (int *)ctx->pcount.p;
    return w;
}

// Copy the plan's descriptors to the device (pinned staging, async).  The
// kernels only read them, so when they are byte for byte those of the last
// upload into the same buffer the copy is skipped: a repeated solve of the
// same frames then enqueues its graph alone, with no host-to-device copy (and
// its cross-engine wait) between two solves.
int upload_plan(pilot_ctx *ctx, const Plan &plan, DevPtrs &dp)
{
    const size_t fb = align256(plan.frames.size() * sizeof(FrameDev));
    const size_t ib = align256(std::max<size_t>(1, plan.items.size()) * sizeof(WorkItem));
    const size_t tb = align256(std::max<size_t>(1, plan.tiles.size()) * sizeof(TileItem));
    int rc = ensure(ctx, ctx->desc, fb + ib + tb);
    if (rc) return rc;
    char *d = (char *)ctx->desc.p;
    dp.frames = (FrameDev *)d;
    dp.items = (WorkItem *)(d + fb);
    dp.tiles = (TileItem *)(d + fb + ib);
    std::vector<char> &img = ctx->desc_next;
    img.assign(fb + ib + tb, 0);
    memcpy(img.data(), plan.frames.data(), plan.frames.size() * sizeof(FrameDev));
    if (!plan.items.empty()) memcpy(img.data() + fb, plan.items.data(), plan.items.size() * sizeof(WorkItem));
    if (!plan.tiles.empty()) memcpy(img.data() + fb + ib, plan.tiles.data(), plan.tiles.size() * sizeof(TileItem));
    if (ctx->desc_gen == ctx->generation && img == ctx->desc_img) return PILOT_OK;
    int which;
    char *h = (char *)stage_acquire(ctx, img.size(), &which, &rc);
    if (!h) return rc;
    memcpy(h, img.data(), img.size());
    ctx->desc_gen = ~0u;   // until the copy is enqueued
    HIPCHK(ctx, hipMemcpyAsync(ctx->desc.p, h, img.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->stage[which].ev, ctx->stream));
    ctx->stage[which].pending = true;
    ctx->desc_img.swap(img);
    ctx->desc_gen = ctx->generation;
    return PILOT_OK;
}

// Workspace for a plan; points the plan's levels at their Gram tables.
int ensure_state(pilot_ctx *ctx, Plan &plan)
{
    int rc;
    if (plan.anchor_bytes) {
        if ((rc = ensure(ctx, ctx->anch, plan.anchor_bytes))) return rc;
        for (const Plan::AnchorJob &j : plan.anchor_jobs)
            place_anchor_copy(plan.frames[j.frame].lv[j.level], (char *)ctx->anch.p + j.offset);
    }
    if (plan.gram_bytes) {
        if ((rc = ensure(ctx, ctx->gram, plan.gram_bytes))) return rc;
        for (const Plan::GramJob &j : plan.gram_jobs)
            plan.frames[j.frame].lv[j.level].gram = (const double *)((const char *)ctx->gram.p + j.offset);
    }
    const size_t H = std::max(1, plan.total_hyps);
    if ((rc = ensure(ctx, ctx->hs, H * sizeof(HypState)))) return rc;
    if ((rc = ensure(ctx, ctx->pose, H * sizeof(PoseEval)))) return rc;
    if ((rc = ensure(ctx, ctx->hlev, H * sizeof(int)))) return rc;
    if ((rc = ensure(ctx, ctx->partials, std::max<size_t>(1, plan.partial_floats) * sizeof(float)))) return rc;
    if ((rc = ensure(ctx, ctx->pairs, kStatClasses * sizeof(unsigned long long), true))) return rc;
    if ((rc = ensure(ctx, ctx->passflag, (size_t)PILOT_MAX_LEVELS * plan.flag_stride * sizeof(int)))) return rc;
    if ((rc = ensure(ctx, ctx->phs, 3 * H * sizeof(HypState)))) return rc;
    if ((rc = ensure(ctx, ctx->ppose, 3 * H * sizeof(PoseEval)))) return rc;
    if ((rc = ensure(ctx, ctx->pcount, 3 * std::max<size_t>(1, plan.frames.size()) * sizeof(int)))) return rc;
    return PILOT_OK;
}

// Enqueue one pass (pass kernel + epilogue) of a launch group.
// packed: the Gram-table variants (3 to 10) walk packed hypothesis tiles,
// built by the pack kernel right before the pass.
int enqueue_pass(pilot_ctx *ctx, const Plan &plan, const DevPtrs &dp, const Ws &ws, const LaunchGroup &g, int mode,
                 hipStream_t s, bool timed, const int *run_flag = nullptr, int *next_flag = nullptr,
                 bool mask_first = false, bool packed = false, int pass_index = 0)
{
    packed = packed && uses_gram(g.tc) && g.tc.pack != 0;
    const int b0 = pass_index % 3, b1 = (pass_index + 1) % 3, b2 = (pass_index + 2) % 3;
    if (uses_gram(g.tc))                       // every frame of the group needs its Gram table
        for (int t = g.tile_off; t < g.tile_off + g.n_tiles; ++t)
            if (!plan.frames[plan.tiles[t].frame].lv[g.level].gram)
                return fail(ctx, PILOT_EDEVICE, "internal: Gram pass variant without a Gram table (level %d)", g.level);
    PassArgs a{};
    a.frames = dp.frames;
    a.items = dp.items + g.item_off;
    a.n_items = g.n_items;
    a.level = g.level;
    a.pose = ws.pose;
    a.hlev = ws.hlev;
    a.partials = ws.partials + g.partial_off;
    a.run_flag = run_flag;
    if (packed) {
        a.ppose = ws.ppose + (size_t)b0 * ws.hyps;
        a.pcount = ws.pcount + (size_t)b0 * ws.frames;
        a.pcount_clear = ws.pcount + (size_t)b2 * ws.frames;
        a.n_frames = ws.frames;
    }
    TimedLaunch tl{};
    if (timed) {
        tl.a = pool_event(ctx);
        tl.b = pool_event(ctx);
        tl.level = g.level;
        tl.cls = g.stat_class;
        if (!tl.a || !tl.b) return fail(ctx, PILOT_EDEVICE, "hipEventCreate failed");
        HIPCHK(ctx, hipEventRecord(tl.a, s));
    }
    HIPCHK(ctx, launch_pass(g.C, g.dtype, g.tc, a, s));
    if (timed) {
        HIPCHK(ctx, hipEventRecord(tl.b, s));
        ctx->timed.push_back(tl);
    }
    EpilogueArgs e{};
    e.frames = dp.frames;
    e.tiles = dp.tiles + g.tile_off;
    e.n_tiles = g.n_tiles;
    e.level = g.level;
    e.G = g.tc.G;
    e.mode = mode;
    e.partials = ws.partials + g.partial_off;
    e.pose = ws.pose;
    e.hlev = ws.hlev;
    e.hs = ws.hs;
    e.pairs = ws.pairs + g.stat_class;
    e.next_flag = next_flag;
    e.mask_first = mask_first ? 1 : 0;
    if (packed) {
        e.phs = ws.phs + (size_t)b0 * ws.hyps;
        e.ppose = ws.ppose + (size_t)b0 * ws.hyps;
        e.pcount = ws.pcount + (size_t)b0 * ws.frames;
        e.phs_next = ws.phs + (size_t)b1 * ws.hyps;
        e.ppose_next = ws.ppose + (size_t)b1 * ws.hyps;
        e.pcount_next = ws.pcount + (size_t)b1 * ws.frames;
    }
    HIPCHK(ctx, launch_epilogue(e, s));
    ctx->launches[g.stat_class]++;
    return PILOT_OK;
}

// Gram tables of the plan's Gram-variant levels (they depend on the feature
// maps only, and are rebuilt with every solve since a replay may see new maps:
// the kernel reads each map's address from the device descriptors).
// The per-frame preparation: anchors into spatial order, then Gram tables.
int enqueue_gram(pilot_ctx *ctx, const Plan &plan, const DevPtrs &dp, hipStream_t s)
{
    if (!plan.anchor_jobs.empty())
        HIPCHK(ctx, launch_anchor_sort(dp.frames, (int)plan.frames.size(), plan.max_levels, plan.anchor_max_N, s));
    for (const Plan::GramJob &j : plan.gram_jobs) {
        const LevelDev &L = plan.frames[j.frame].lv[j.level];
        HIPCHK(ctx, launch_gram(dp.frames, j.frame, j.level, L.H, L.W, L.C, L.dtype, j.fmt, s));
    }
    return PILOT_OK;
}

// The full LM schedule of a plan on stream s.
int enqueue_schedule(pilot_ctx *ctx, const Plan &plan, const DevPtrs &dp, const Ws &ws, hipStream_t s, bool timed)
{
    if (int rc = enqueue_gram(ctx, plan, dp, s)) return rc;
    HIPCHK(ctx, launch_init(dp.frames, (int)plan.frames.size(), plan.max_M, ws.hs, ws.pose, ws.hlev, MODE_LM,
                            nullptr, 0, s, ws.passflag, PILOT_MAX_LEVELS * plan.flag_stride, plan.flag_stride));
    // packed hypothesis tiles: the Gram-variant passes walk, G at a time, the
    // list of each frame's hypotheses still at the level (listed in index order
    // at the level's start, then by each epilogue, which appends the ones that
    // stay), so a pass costs what its live hypotheses need rather than every
    // tile that still holds one.  Sums do not depend on a hypothesis' tile or
    // slot, so results are those of contiguous tiles, bit for bit.
    const int nf = (int)plan.frames.size();
    bool pack = false;
    for (const LaunchGroup &g : plan.groups) pack = pack || (uses_gram(g.tc) && g.tc.pack != 0);
    Ws wp = ws;
    wp.hyps = std::max(1, plan.total_hyps);
    wp.frames = std::max(1, nf);
    // a level's first pass reads buffer 0, filled here; its epilogue appends
    // to buffer 1, and the next pass clears buffer 2
    auto pack_level = [&](int level) -> hipError_t {
        return launch_pack(dp.frames, nf, plan.max_M, wp.hlev, level, wp.hs, wp.pose, wp.phs, wp.ppose, wp.pcount,
                           wp.pcount + wp.frames, wp.pcount + 2 * (size_t)wp.frames, s);
    };
    if (pack) HIPCHK(ctx, pack_level(0));
    for (int l = 0; l < plan.max_levels; ++l) {
        int maxp = 0;
        for (const LaunchGroup &g : plan.groups)
            if (g.level == l) maxp = std::max(maxp, g.passes);
        bool prunes = false;
        for (const FrameDev &f : plan.frames) prunes = prunes || (f.keep_top > 0 && f.prune_level == l);
        for (int k = 0; k < maxp; ++k) {
            // the pass's launch groups (disjoint frames, disjoint partial
            // records) run concurrently: the largest first, each on the least
            // loaded of the context's stream and its side streams
            std::vector<const LaunchGroup *> gs;
            for (const LaunchGroup &g : plan.groups)
                if (g.level == l && k < g.passes) gs.push_back(&g);
            std::stable_sort(gs.begin(), gs.end(),
                             [](const LaunchGroup *a, const LaunchGroup *b) { return a->n_items > b->n_items; });
            const int nside = std::min<int>(kSideStreams, (int)gs.size() - 1);
            if (nside > 0) {
                HIPCHK(ctx, hipEventRecord(ctx->fork_ev, s));
                for (int i = 0; i < nside; ++i) HIPCHK(ctx, hipStreamWaitEvent(ctx->side[i], ctx->fork_ev, 0));
            }
            long load[1 + kSideStreams] = {0};
            for (const LaunchGroup *g : gs) {
                int q = 0;
                for (int i = 1; i <= nside; ++i)
                    if (load[i] < load[q]) q = i;
                load[q] += g->n_items;
                // pass k of level l runs only if pass k - 1 left a hypothesis at level l
                int *flags = ws.passflag + (size_t)l * plan.flag_stride;
                int rc = enqueue_pass(ctx, plan, dp, wp, *g, MODE_LM, q ? ctx->side[q - 1] : s, timed, flags + k,
                                      flags + k + 1, false, pack, k);
                if (rc) return rc;
            }
            for (int i = 0; i < nside; ++i) {
                HIPCHK(ctx, hipEventRecord(ctx->join_ev[i], ctx->side[i]));
                HIPCHK(ctx, hipStreamWaitEvent(s, ctx->join_ev[i], 0));
            }
        }
        if (prunes) HIPCHK(ctx, launch_prune(dp.frames, nf, ws.hs, ws.pose, ws.hlev, s));
        if (pack && l + 1 < plan.max_levels) HIPCHK(ctx, pack_level(l + 1));
    }
    HIPCHK(ctx, launch_finalize(dp.frames, (int)plan.frames.size(), ws.hs, ws.hlev, s));
    return PILOT_OK;
}

void load_tune_cache(pilot_ctx *ctx)
{
    if (ctx->tune_cache.empty()) return;
    std::ifstream in(ctx->tune_cache);
    std::string line;
    // "key G PPG grid variant [pack]" per line (pack 0 when absent)
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        TileConfig tc{};
        if (!(ls >> key >> tc.G >> tc.PPG >> tc.grid >> tc.variant)) continue;
        if (!(ls >> tc.pack)) tc.pack = 0;
        if ((tc.G == 1 || tc.G == 2 || tc.G == 4 || tc.G == 8 || tc.G == 16) && tc.PPG >= 1 && tc.PPG <= 64 &&
            tc.variant >= 1 && tc.variant <= 10 && tc.pack >= 0 && tc.pack <= 2)
            ctx->tuned[key] = tc;
    }
}

int collect_timings(pilot_ctx *ctx)
{
    if (ctx->timed.empty()) return PILOT_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (TimedLaunch &t : ctx->timed) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->pass_ms[t.cls] += ms;
        ctx->timed_launches[t.cls]++;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return PILOT_OK;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

int pilot_abi_version(void) { return PILOT_ABI_VERSION; }

size_t pilot_sizeof(const char *name)
{
    if (!name) return 0;
    if (!strcmp(name, "pilot_frame")) return sizeof(pilot_frame);
    if (!strcmp(name, "pilot_level")) return sizeof(pilot_level);
    if (!strcmp(name, "pilot_result")) return sizeof(pilot_result);
    if (!strcmp(name, "pilot_config")) return sizeof(pilot_config);
    if (!strcmp(name, "pilot_stats")) return sizeof(pilot_stats);
    return 0;
}

const char *pilot_last_error(const pilot_ctx *ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

int pilot_create(pilot_ctx **out, const pilot_config *cfg)
{
    if (!out) return fail(nullptr, PILOT_EINVAL, "out: NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, PILOT_EINVAL, "cfg: NULL");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return fail(nullptr, PILOT_EDEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (cfg->device < 0 || cfg->device >= ndev)
        return fail(nullptr, PILOT_EINVAL, "cfg.device: %d is not one of the %d visible devices", cfg->device, ndev);
    if (cfg->max_slots < 0 || cfg->max_slots > 4096) return fail(nullptr, PILOT_EINVAL, "cfg.max_slots: must be 0..4096");
    e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return fail(nullptr, PILOT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, cfg->device);
    if (e != hipSuccess) return fail(nullptr, PILOT_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, PILOT_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", cfg->device, prop.gcnArchName);
    pilot_ctx *ctx = new pilot_ctx();
    ctx->device = cfg->device;
    ctx->flags = cfg->flags;
    if (ctx->flags & PILOT_FLAG_PROFILE) ctx->flags |= PILOT_FLAG_NO_GRAPH;
    ctx->stream = (hipStream_t)cfg->stream;
    ctx->budget = cfg->hbm_budget_bytes;
    ctx->tune_cache = cfg->tune_cache ? cfg->tune_cache : "";
    ctx->max_slots = cfg->max_slots ? cfg->max_slots : 64;
    ctx->ncu = prop.multiProcessorCount;
    e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->stage[0].ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->stage[1].ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        int rc = fail(nullptr, PILOT_EDEVICE, "stream/event creation: %s", hipGetErrorString(e));
        pilot_destroy(ctx);
        return rc;
    }
    // the fixed scratch of pilot_solve_static: its address on this device
    e = static_scratch_init(cfg->device);
    if (e != hipSuccess) {
        int rc = fail(nullptr, PILOT_EDEVICE, "hipGetSymbolAddress(static scratch): %s", hipGetErrorString(e));
        pilot_destroy(ctx);
        return rc;
    }
    load_tune_cache(ctx);
    *out = ctx;
    return PILOT_OK;
}

void pilot_destroy(pilot_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    for (auto &t : ctx->timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ctx->event_pool) hipEventDestroy(e);
    for (auto &s : ctx->stage) {
        if (s.ev) hipEventSynchronize(s.ev), hipEventDestroy(s.ev);
        if (s.p) hipHostFree(s.p);
    }
    for (DevBuf *b : {&ctx->desc, &ctx->hs, &ctx->pose, &ctx->hlev, &ctx->partials, &ctx->pairs, &ctx->gram,
                      &ctx->anch, &ctx->passflag, &ctx->phs, &ctx->ppose, &ctx->pcount,
                      &ctx->s_frames, &ctx->s_desc, &ctx->s_done})
        if (b->p) hipFree(b->p);
    for (auto &fb : ctx->flagbuf) {
        if (fb.ev) hipEventDestroy(fb.ev);
        if (fb.host) hipHostFree(fb.host);
    }
    for (ServingSlot &sl : ctx->slots) {
        if (sl.gram.p) hipFree(sl.gram.p);
        if (sl.anch.p) hipFree(sl.anch.p);
    }
    for (int i = 0; i < kSideStreams; ++i) {
        if (ctx->side[i]) hipStreamSynchronize(ctx->side[i]), hipStreamDestroy(ctx->side[i]);
        if (ctx->join_ev[i]) hipEventDestroy(ctx->join_ev[i]);
    }
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

}  // extern "C"

namespace {

// Argument checks shared by pilot_solve and pilot_solve_static.
int validate_solve(pilot_ctx *ctx, const pilot_frame *frames, int n_frames, const pilot_result *results)
{
    if (!frames) return fail(ctx, PILOT_EINVAL, "frames: NULL");
    if (n_frames < 1) return fail(ctx, PILOT_EINVAL, "n_frames: must be >= 1 (got %d)", n_frames);
    if (!results) return fail(ctx, PILOT_EINVAL, "results: NULL");
    long total = 0;
    for (int i = 0; i < n_frames; ++i) {
        int rc = validate_frame(ctx, &frames[i], i, true);
        if (rc) return rc;
        const pilot_result &r = results[i];
        if (!r.poses_out || !r.cost || !r.iterations || !r.status || !r.best)
            return fail(ctx, PILOT_EINVAL, "results[%d]: every output buffer must be non-NULL", i);
        total += frames[i].M;
    }
    if (total > (1L << 24)) return fail(ctx, PILOT_EINVAL, "total hypotheses %ld exceed 2^24", total);
    if (ctx->n_active() > 0) return fail(ctx, PILOT_EINVAL, "context has active serving slots");
    return PILOT_OK;
}

}  // namespace

extern "C" {

int pilot_solve(pilot_ctx *ctx, const pilot_frame *frames, int n_frames, const pilot_result *results)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    if (int rc = validate_solve(ctx, frames, n_frames, results)) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));

    if (ctx->flags & PILOT_FLAG_AUTOTUNE) {
        for (int i = 0; i < n_frames; ++i) {
            bool need = false;
            for (int l = 0; l < frames[i].n_levels; ++l) {
                const pilot_level &L = frames[i].level[l];
                if (!ctx->tuned.count(tune_key(L.C, L.dtype, L.N, frames[i].M, (long)L.H * L.W))) need = true;
            }
            if (need) {
                int rc = pilot_autotune(ctx, &frames[i]);
                if (rc) return rc;
            }
        }
    }

    Plan plan;
    build_plan(ctx, frames, n_frames, results, -1, plan);
    int rc = ensure_state(ctx, plan);
    if (rc) return rc;
    DevPtrs dp;
    if ((rc = upload_plan(ctx, plan, dp))) return rc;

    if (ctx->flags & PILOT_FLAG_NO_GRAPH)
        return enqueue_schedule(ctx, plan, dp, ws_of(ctx), ctx->stream, (ctx->flags & PILOT_FLAG_PROFILE) != 0);

    std::string key = plan.key + "#" + std::to_string(ctx->generation) + "#" + std::to_string((uintptr_t)dp.frames);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_schedule(ctx, plan, dp, ws_of(ctx), ctx->cap_stream, false);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (rc) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(ctx, PILOT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(ctx, PILOT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        if (ctx->graphs.size() >= 64) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            for (auto &kv : ctx->graphs) hipGraphExecDestroy(kv.second);
            ctx->graphs.clear();
        }
        it = ctx->graphs.emplace(key, exec).first;
        ctx->graph_captures++;
    }
    HIPCHK(ctx, hipGraphLaunch(it->second, ctx->stream));
    ctx->graph_replays++;
    return PILOT_OK;
}

int pilot_solve_static(pilot_ctx *ctx, const pilot_frame *frames, int n_frames, const pilot_result *results)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    if (int rc = validate_solve(ctx, frames, n_frames, results)) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    char *base = (char *)static_scratch(ctx->device);
    if (!base) return fail(ctx, PILOT_EDEVICE, "internal: no static scratch address for device %d", ctx->device);

    // tiles from the context's tile database or the heuristic (no tuning here)
    Plan plan;
    build_plan(ctx, frames, n_frames, results, -1, plan);
    const size_t fb = align256(plan.frames.size() * sizeof(FrameDev));
    const size_t ib = align256(std::max<size_t>(1, plan.items.size()) * sizeof(WorkItem));
    const size_t tb = align256(std::max<size_t>(1, plan.tiles.size()) * sizeof(TileItem));
    const size_t H = std::max(1, plan.total_hyps);
    size_t off = fb + ib + tb;
    const size_t o_gram = off;
    off += align256(plan.gram_bytes);
    const size_t o_anch = off;
    off += align256(plan.anchor_bytes);
    const size_t o_hs = off;
    off += align256(H * sizeof(HypState));
    const size_t o_pose = off;
    off += align256(H * sizeof(PoseEval));
    const size_t o_hlev = off;
    off += align256(H * sizeof(int));
    const size_t o_part = off;
    off += align256(std::max<size_t>(1, plan.partial_floats) * sizeof(float));
    const size_t o_pairs = off;
    off += align256(kStatClasses * sizeof(unsigned long long));
    const size_t o_flag = off;
    off += align256((size_t)PILOT_MAX_LEVELS * plan.flag_stride * sizeof(int));
    const size_t o_phs = off;
    off += align256(3 * H * sizeof(HypState));
    const size_t o_ppose = off;
    off += align256(3 * H * sizeof(PoseEval));
    const size_t o_pcount = off;
    off += align256(3 * std::max<size_t>(1, plan.frames.size()) * sizeof(int));
    if (off > static_scratch_bytes())
        return fail(ctx, PILOT_ENOMEM,
                    "pilot_solve_static: these frames need %zu bytes of device scratch; the fixed scratch holds %zu "
                    "(use pilot_solve)", off, static_scratch_bytes());

    for (const Plan::GramJob &j : plan.gram_jobs)
        plan.frames[j.frame].lv[j.level].gram = (const double *)(base + o_gram + j.offset);
    for (const Plan::AnchorJob &j : plan.anchor_jobs)
        place_anchor_copy(plan.frames[j.frame].lv[j.level], base + o_anch + j.offset);
    DevPtrs dp;
    dp.frames = (FrameDev *)base;
    dp.items = (WorkItem *)(base + fb);
    dp.tiles = (TileItem *)(base + fb + ib);
    Ws ws;
    ws.hs = (HypState *)(base + o_hs);
    ws.pose = (PoseEval *)(base + o_pose);
    ws.hlev = (int *)(base + o_hlev);
    ws.partials = (float *)(base + o_part);
    ws.pairs = (unsigned long long *)(base + o_pairs);
    ws.passflag = (int *)(base + o_flag);
    ws.phs = (HypState *)(base + o_phs);
    ws.ppose = (PoseEval *)(base + o_ppose);
    ws.pcount = (int *)(base + o_pcount);

    // descriptors: from a host image the context keeps (pageable; the copy
    // has consumed it when hipMemcpyAsync returns)
    std::vector<char> &img = ctx->static_img;
    img.assign(fb + ib + tb, 0);
    memcpy(img.data(), plan.frames.data(), plan.frames.size() * sizeof(FrameDev));
    if (!plan.items.empty()) memcpy(img.data() + fb, plan.items.data(), plan.items.size() * sizeof(WorkItem));
    if (!plan.tiles.empty()) memcpy(img.data() + fb + ib, plan.tiles.data(), plan.tiles.size() * sizeof(TileItem));
    HIPCHK(ctx, hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, ctx->stream));
    // the pair counters start at zero (a fill kernel, not a memset node)
    HIPCHK(ctx, launch_zero_words(ws.pairs, (int)(kStatClasses * sizeof(unsigned long long) / 4), ctx->stream));
    return enqueue_schedule(ctx, plan, dp, ws, ctx->stream, false);
}

int pilot_linearize(pilot_ctx *ctx, const pilot_frame *frame, int level, const double *poses, double *H21,
                    double *g6, double *cost, int32_t *nvalid)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    int rc = validate_frame(ctx, frame, 0, false);
    if (rc) return rc;
    if (level < 0 || level >= frame->n_levels)
        return fail(ctx, PILOT_EINVAL, "level: must be 0..%d (got %d)", frame->n_levels - 1, level);
    if (!poses) return fail(ctx, PILOT_EINVAL, "poses: NULL");
    if (!H21 || !g6 || !cost || !nvalid) return fail(ctx, PILOT_EINVAL, "H21/g6/cost/nvalid: NULL");
    if (ctx->n_active() > 0) return fail(ctx, PILOT_EINVAL, "context has active serving slots");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Plan plan;
    build_plan(ctx, frame, 1, nullptr, level, plan);
    FrameDev &d = plan.frames[0];
    d.diag_H = H21;
    d.diag_g = g6;
    d.diag_cost = cost;
    d.diag_n = nvalid;
    if ((rc = ensure_state(ctx, plan))) return rc;
    DevPtrs dp;
    if ((rc = upload_plan(ctx, plan, dp))) return rc;
    if ((rc = enqueue_gram(ctx, plan, dp, ctx->stream))) return rc;
    const Ws ws = ws_of(ctx);
    HIPCHK(ctx, launch_init(dp.frames, 1, plan.max_M, ws.hs, ws.pose, ws.hlev, MODE_DIAG, poses, level, ctx->stream));
    for (const LaunchGroup &g : plan.groups)
        if ((rc = enqueue_pass(ctx, plan, dp, ws, g, MODE_DIAG, ctx->stream, (ctx->flags & PILOT_FLAG_PROFILE) != 0)))
            return rc;
    return PILOT_OK;
}

int pilot_lift(pilot_ctx *ctx, const float *dsm, int32_t Hd, int32_t Wd, double x0, double y0, double gsd,
               const float *uv, int32_t N, const void *ref_map, int32_t Hr, int32_t Wr, int32_t C, int32_t dtype,
               double scale, float *x, float *y, float *z, void *ref_out)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    if (N < 0) return fail(ctx, PILOT_EINVAL, "N: must be >= 0");
    if (N == 0) return PILOT_OK;
    if (!dsm || Hd < 2 || Wd < 2) return fail(ctx, PILOT_EINVAL, "dsm/Hd/Wd: need a device raster of at least 2x2");
    if (!(gsd > 0) || !std::isfinite(gsd) || !std::isfinite(x0) || !std::isfinite(y0))
        return fail(ctx, PILOT_EINVAL, "x0/y0/gsd: invalid");
    if (!uv) return fail(ctx, PILOT_EINVAL, "uv: NULL");
    if (!ref_map || Hr < 2 || Wr < 2) return fail(ctx, PILOT_EINVAL, "ref_map/Hr/Wr: need a device map of at least 2x2");
    if (C != 16 && C != 32 && C != 64 && C != 128 && C != 256)
        return fail(ctx, PILOT_EINVAL, "C: must be 16, 32, 64, 128 or 256 (got %d)", C);
    if (dtype != PILOT_F32 && dtype != PILOT_BF16) return fail(ctx, PILOT_EINVAL, "dtype: must be PILOT_F32 or PILOT_BF16");
    if (!(scale > 0) || !std::isfinite(scale)) return fail(ctx, PILOT_EINVAL, "scale: must be finite and > 0");
    if (!ref_out) return fail(ctx, PILOT_EINVAL, "ref_out: NULL");
    if ((double)Hr * Wr * C >= 2147483647.0 || (double)N * C >= 2147483647.0)
        return fail(ctx, PILOT_EINVAL, "Hr*Wr*C and N*C must be < 2^31");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_lift(dsm, Hd, Wd, x0, y0, gsd, uv, N, ref_map, Hr, Wr, C, dtype, scale, x, y, z, ref_out,
                            ctx->stream));
    return PILOT_OK;
}

// One eager solve of `frame` with per-pass events; summed pass-kernel ms per
// level into ms[].  The context's counters are left as they were.
static int timed_solve(pilot_ctx *ctx, const pilot_frame *frame, const pilot_result *res, double ms[PILOT_MAX_LEVELS])
{
    Plan plan;
    build_plan(ctx, frame, 1, res, -1, plan);
    int rc = ensure_state(ctx, plan);
    if (rc) return rc;
    DevPtrs dp;
    if ((rc = upload_plan(ctx, plan, dp))) return rc;
    uint64_t launches[kStatClasses];
    memcpy(launches, ctx->launches, sizeof launches);
    rc = enqueue_schedule(ctx, plan, dp, ws_of(ctx), ctx->stream, true);
    memcpy(ctx->launches, launches, sizeof launches);
    if (rc) return rc;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int l = 0; l < PILOT_MAX_LEVELS; ++l) ms[l] = 0.0;
    for (TimedLaunch &t : ctx->timed) {
        float x = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&x, t.a, t.b));
        ms[t.level] += x;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return PILOT_OK;
}

// Tiles are chosen by what they cost inside a solve of the caller's frame:
// hypotheses finish at different iterations, and a tile is paid for as
// long as any of its hypotheses is active, so timing a pass with every
// hypothesis active favours tiles that are slower in practice.
int pilot_autotune(pilot_ctx *ctx, const pilot_frame *frame)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    int rc = validate_frame(ctx, frame, 0, true);
    if (rc) return rc;
    if (ctx->n_active() > 0) return fail(ctx, PILOT_EINVAL, "context has active serving slots");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    std::vector<std::string> keys(frame->n_levels);
    std::vector<std::string> todo;
    std::vector<int> todo_C, todo_dt;
    for (int l = 0; l < frame->n_levels; ++l) {
        const pilot_level &L = frame->level[l];
        keys[l] = tune_key(L.C, L.dtype, L.N, frame->M, (long)L.H * L.W);
        if (!ctx->tuned.count(keys[l]) && std::find(todo.begin(), todo.end(), keys[l]) == todo.end()) {
            todo.push_back(keys[l]);
            todo_C.push_back(L.C);
            todo_dt.push_back(L.dtype);
        }
    }
    if (todo.empty()) return PILOT_OK;
    if ((rc = collect_timings(ctx))) return rc;           // earlier profiled launches go to the counters

    std::vector<TileConfig> cand;
    // variants 5, 6, 8, 9 and 10 differ from 3, 4, 7, 3 and 4 for bf16 maps only
    bool bf16 = false;
    for (int l = 0; l < frame->n_levels; ++l) bf16 = bf16 || frame->level[l].dtype == PILOT_BF16;
    for (int variant : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10}) {
        if ((variant == 5 || variant == 6 || variant >= 8) && !bf16) continue;
        for (int G : {1, 2, 4, 8, 16}) {
            if (G < 4 && variant < 9) continue;          // narrow lane groups: variants 9 and 10 only
            for (int ppg : {2, 4, 8, 16})
                for (int bpc : {0, 2, 4}) cand.push_back(TileConfig{G, ppg, bpc, variant});
        }
    }

    // scratch outputs of the timed solves
    const int M = frame->M;
    void *buf = nullptr;
    const size_t bytes = (size_t)M * (12 + 1) * sizeof(double) + (size_t)M * 2 * sizeof(int32_t) + 64;
    HIPCHK(ctx, hipMalloc(&buf, bytes));
    pilot_result res{};                 // every pointer not set below stays NULL (optional outputs off)
    res.poses_out = (double *)buf;
    res.cost = res.poses_out + (size_t)M * 12;
    res.iterations = (int32_t *)(res.cost + M);
    res.status = res.iterations + M;
    res.best = res.status + M;
    unsigned long long pairs_saved[kStatClasses] = {0};

    auto apply = [&](const TileConfig &tc) {
        for (const std::string &k : todo) ctx->tuned[k] = tc;
    };
    // score[c][k]: lowest summed pass ms of candidate c on key k
    std::vector<std::vector<double>> score(cand.size(), std::vector<double>(todo.size(), 1e300));
    auto run = [&](size_t c) -> int {
        apply(cand[c]);
        double ms[PILOT_MAX_LEVELS];
        int r = timed_solve(ctx, frame, &res, ms);
        if (r) return r;
        std::vector<double> per(todo.size(), 0.0);
        for (int l = 0; l < frame->n_levels; ++l) {
            const auto it = std::find(todo.begin(), todo.end(), keys[l]);
            if (it != todo.end()) per[it - todo.begin()] += ms[l];
        }
        for (size_t k = 0; k < todo.size(); ++k)
            if (tile_ok(cand[c], todo_C[k], todo_dt[k])) score[c][k] = std::min(score[c][k], per[k]);
        return PILOT_OK;
    };

    rc = PILOT_OK;
    do {
        if (ctx->pairs.p) {
            if (hipMemcpy(pairs_saved, ctx->pairs.p, sizeof pairs_saved, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(ctx, PILOT_EDEVICE, "hipMemcpy of counters failed");
                break;
            }
        }
        // bring the clocks up (an idle GPU runs the first tens of ms slower)
        apply(heuristic_tile(ctx, frame->level[0].C, frame->level[0].dtype, frame->level[0].N, M,
                             (long)frame->level[0].H * frame->level[0].W));
        double warm = 0.0;
        for (int k = 0; k < 50 && warm < 40.0 && rc == PILOT_OK; ++k) {
            double ms[PILOT_MAX_LEVELS];
            rc = timed_solve(ctx, frame, &res, ms);
            for (int l = 0; l < frame->n_levels; ++l) warm += ms[l];
        }
        if (rc) break;
        for (size_t c = 0; c < cand.size() && rc == PILOT_OK; ++c) rc = run(c);
        if (rc) break;
        // second round for the 8 best of each key, and the same tiles with packed
        // hypothesis tiles (Gram variants; packing pays where stragglers are many)
        const size_t n1 = cand.size();
        std::vector<char> again(n1, 0);
        for (size_t k = 0; k < todo.size(); ++k) {
            std::vector<size_t> order(n1);
            for (size_t c = 0; c < n1; ++c) order[c] = c;
            std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return score[a][k] < score[b][k]; });
            for (size_t i = 0; i < 8 && i < order.size(); ++i) again[order[i]] = 1;
        }
        for (size_t c = 0; c < n1; ++c)
            if (again[c] && uses_gram(cand[c]))
                for (int pk : {1, 2}) {
                    TileConfig t = cand[c];
                    t.pack = pk;
                    cand.push_back(t);
                    score.push_back(std::vector<double>(todo.size(), 1e300));
                    again.push_back(1);
                }
        for (size_t c = 0; c < cand.size() && rc == PILOT_OK; ++c)
            if (again[c]) rc = run(c);
    } while (false);
    // put the counters back as they were (zero if the buffer did not exist yet)
    if (ctx->pairs.p) {
        if (hipMemcpy(ctx->pairs.p, pairs_saved, sizeof pairs_saved, hipMemcpyHostToDevice) != hipSuccess && !rc)
            rc = fail(ctx, PILOT_EDEVICE, "hipMemcpy of counters failed");
    }
    hipFree(buf);
    for (const std::string &k : todo) ctx->tuned.erase(k);
    if (rc) return rc;

    for (size_t k = 0; k < todo.size(); ++k) {
        size_t bi = 0;
        for (size_t c = 1; c < cand.size(); ++c)
            if (score[c][k] < score[bi][k]) bi = c;
        ctx->tuned[todo[k]] = cand[bi];
        if (!ctx->tune_cache.empty()) {
            std::ofstream out(ctx->tune_cache, std::ios::app);
            out << todo[k] << " " << cand[bi].G << " " << cand[bi].PPG << " " << cand[bi].grid << " "
                << cand[bi].variant << " " << cand[bi].pack << "\n";
        }
    }
    return PILOT_OK;
}

int pilot_tile_choice(pilot_ctx *ctx, int C, int dtype, int N, int M, int64_t HW, char *buf, int buflen)
{
    if (!ctx || !buf || buflen < 1) return fail(ctx, PILOT_EINVAL, "ctx/buf: invalid");
    TileConfig tc = choose_tile(ctx, C, dtype, N, M, (long)HW);
    auto it = ctx->tuned.find(tune_key(C, dtype, N, M, (long)HW));
    snprintf(buf, buflen, "G=%d PPG=%d BPC=%d V=%d pack=%d tuned=%d", tc.G, tc.PPG, tc.grid, tc.variant, tc.pack,
             (int)(it != ctx->tuned.end() && tile_ok(it->second, C, dtype)));
    return PILOT_OK;
}

int pilot_get_stats(pilot_ctx *ctx, pilot_stats *out, int reset)
{
    if (!ctx || !out) return fail(ctx, PILOT_EINVAL, "ctx/out: NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int rc = collect_timings(ctx);
    if (rc) return rc;
    memset(out, 0, sizeof *out);
    unsigned long long pairs[kStatClasses] = {0};
    if (ctx->pairs.p) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        HIPCHK(ctx, hipMemcpy(pairs, ctx->pairs.p, sizeof pairs, hipMemcpyDeviceToHost));
    }
    static const int Cs[5] = {16, 32, 64, 128, 256};
    for (int l = 0; l < PILOT_MAX_LEVELS; ++l)
        for (int ci = 0; ci < 5; ++ci)
            for (int dt = 0; dt < 2; ++dt) {
                const int k = l * 10 + ci * 2 + dt;
                out->pairs[l] += pairs[k];
                out->pair_bytes[l] += pairs[k] * 4ull * Cs[ci] * elem_size(dt);
                out->launches[l] += ctx->launches[k];
                out->pass_ms[l] += ctx->pass_ms[k];
                out->timed_launches[l] += ctx->timed_launches[k];
            }
    out->graph_replays = ctx->graph_replays;
    out->graph_captures = ctx->graph_captures;
    if (reset) {
        if (ctx->pairs.p) HIPCHK(ctx, hipMemset(ctx->pairs.p, 0, kStatClasses * sizeof(unsigned long long)));
        memset(ctx->pass_ms, 0, sizeof ctx->pass_ms);
        memset(ctx->timed_launches, 0, sizeof ctx->timed_launches);
        memset(ctx->launches, 0, sizeof ctx->launches);
        ctx->graph_replays = ctx->graph_captures = 0;
    }
    return PILOT_OK;
}

// ================================================================ serving
}  // extern "C"

namespace {

size_t per_hyp_bytes() { return sizeof(HypState) + sizeof(PoseEval) + sizeof(int); }

// Input bytes a frame declares (maps, anchors, descriptors) plus its
// hypothesis state and the largest partial-sum block of its levels.
size_t frame_cost(const pilot_ctx *ctx, const pilot_frame &f)
{
    size_t in = (size_t)f.M * 12 * sizeof(double);
    size_t part = 0;
    for (int l = 0; l < f.n_levels; ++l) {
        const pilot_level &L = f.level[l];
        const size_t es = elem_size(L.dtype);
        in += (size_t)L.H * L.W * L.C * es + (size_t)L.N * (3 * sizeof(float) + L.C * es);
        if (L.qconf) in += (size_t)L.H * L.W * sizeof(float);
        if (L.ref_w) in += (size_t)L.N * sizeof(float);
        if (sorts_anchors(ctx, L, f.M)) in += anchor_copy_bytes(L);
        const TileConfig tc = choose_tile(ctx, L.C, L.dtype, L.N, f.M, (long)L.H * L.W);
        if (uses_gram(tc)) in += gram_table_bytes(L, gram_format(tc, L.dtype));
        const size_t items = (size_t)((f.M + tc.G - 1) / tc.G) * n_ptiles_of(tc, L.N);
        part = std::max(part, items * tc.G * kNV * sizeof(float));
    }
    if (f.use_range) in += (size_t)f.Hd * f.Wd * sizeof(float);
    return in + (size_t)f.M * per_hyp_bytes() + part;
}

int arena_alloc(pilot_ctx *ctx, int M)
{
    for (size_t i = 0; i < ctx->arena_free.size(); ++i) {
        auto &blk = ctx->arena_free[i];
        if (blk.second >= M) {
            const int off = blk.first;
            blk.first += M;
            blk.second -= M;
            if (blk.second == 0) ctx->arena_free.erase(ctx->arena_free.begin() + i);
            return off;
        }
    }
    return -1;
}

void arena_release(pilot_ctx *ctx, int off, int M)
{
    auto &fl = ctx->arena_free;
    fl.push_back({off, M});
    std::sort(fl.begin(), fl.end());
    std::vector<std::pair<int, int>> merged;
    for (auto &b : fl) {
        if (!merged.empty() && merged.back().first + merged.back().second == b.first)
            merged.back().second += b.second;
        else
            merged.push_back(b);
    }
    fl.swap(merged);
}

int serving_init(pilot_ctx *ctx)
{
    if (!ctx->slots.empty()) return PILOT_OK;
    int rc;
    ctx->arena_cap = std::max(16384, ctx->max_slots * 512);
    const size_t H = ctx->arena_cap;
    if ((rc = ensure(ctx, ctx->hs, H * sizeof(HypState), false, false))) return rc;
    if ((rc = ensure(ctx, ctx->pose, H * sizeof(PoseEval), false, false))) return rc;
    if ((rc = ensure(ctx, ctx->hlev, H * sizeof(int), false, false))) return rc;
    if ((rc = ensure(ctx, ctx->pairs, kStatClasses * sizeof(unsigned long long), true, false))) return rc;
    if ((rc = ensure(ctx, ctx->s_frames, (size_t)ctx->max_slots * sizeof(FrameDev), true, false))) return rc;
    if ((rc = ensure(ctx, ctx->s_done, (size_t)ctx->max_slots * sizeof(int), true, false))) return rc;
    for (auto &fb : ctx->flagbuf) {
        HIPCHK(ctx, hipHostMalloc((void **)&fb.host, (size_t)ctx->max_slots * sizeof(int), hipHostMallocDefault));
        memset(fb.host, 0, (size_t)ctx->max_slots * sizeof(int));
        HIPCHK(ctx, hipEventCreateWithFlags(&fb.ev, hipEventDisableTiming));
    }
    ctx->arena_free.assign(1, {0, ctx->arena_cap});
    ctx->slots.assign(ctx->max_slots, ServingSlot());
    return PILOT_OK;
}

// Work lists over the active slots: per level, slots grouped by (C, dtype).
int serving_rebuild(pilot_ctx *ctx)
{
    Plan &plan = ctx->serv_plan;
    plan = Plan();
    plan.frames.assign(ctx->slots.size(), FrameDev{});     // indexed by slot (host copies, for checks)
    for (int i = 0; i < (int)ctx->slots.size(); ++i)
        if (ctx->slots[i].active) plan.frames[i] = ctx->slots[i].dev;
    std::vector<pilot_frame> frames;
    std::vector<int> slot_of;
    for (int i = 0; i < (int)ctx->slots.size(); ++i)
        if (ctx->slots[i].active) {
            frames.push_back(ctx->slots[i].frame);
            slot_of.push_back(i);
        }
    for (int l = 0; l < PILOT_MAX_LEVELS; ++l) {
        // slots whose tiles share a kernel instantiation share a launch, each
        // with its own anchors per lane group (set in its descriptor at
        // admission); serving steps run their groups one after another
        std::map<std::array<int, 4>, std::vector<int>> by_class;
        std::vector<TileConfig> tck(frames.size());
        for (int k = 0; k < (int)frames.size(); ++k)
            if (l < frames[k].n_levels) {
                const pilot_level &L = frames[k].level[l];
                tck[k] = serving_tile(ctx, L.C, L.dtype, L.N, frames[k].M, (long)L.H * L.W);
                by_class[{L.C, L.dtype, tck[k].G, tck[k].variant}].push_back(k);
            }
        for (auto &kv : by_class) {
            LaunchGroup g{};
            g.level = l;
            g.C = kv.first[0];
            g.dtype = kv.first[1];
            g.item_off = (int)plan.items.size();
            g.tile_off = (int)plan.tiles.size();
            int most = kv.second[0], most_items = -1;
            for (int k : kv.second) {
                const int slot = slot_of[k];
                const TileConfig &t = tck[k];
                const int nht = (frames[k].M + t.G - 1) / t.G;
                const int npt = n_ptiles_of(t, frames[k].level[l].N);
                if (nht * npt > most_items) most = k, most_items = nht * npt;
                for (int ht = 0; ht < nht; ++ht) {
                    const int h0 = ht * t.G, nh = std::min(t.G, frames[k].M - h0);
                    plan.tiles.push_back(TileItem{slot, ht, (int)plan.items.size() - g.item_off, npt,
                                                  ctx->slots[slot].hyp_base + h0, nh});
                    for (int pt = 0; pt < npt; ++pt)
                        plan.items.push_back(WorkItem{slot, ctx->slots[slot].hyp_base + h0, pt, nh});
                }
            }
            g.tc = tck[most];
            g.n_items = (int)plan.items.size() - g.item_off;
            g.n_tiles = (int)plan.tiles.size() - g.tile_off;
            g.passes = 1;
            g.stat_class = class_index(l, g.C, g.dtype);
            g.tc.grid = grid_of(ctx, g.tc, g.n_items);
            plan.partial_floats = std::max(plan.partial_floats, (size_t)g.n_items * g.tc.G * kNV);
            plan.groups.push_back(g);
        }
    }
    int rc = ensure(ctx, ctx->partials, std::max<size_t>(1, plan.partial_floats) * sizeof(float), false, false);
    if (rc) return rc;
    const size_t ib = align256(std::max<size_t>(1, plan.items.size()) * sizeof(WorkItem));
    const size_t tb = align256(std::max<size_t>(1, plan.tiles.size()) * sizeof(TileItem));
    if ((rc = ensure(ctx, ctx->s_desc, ib + tb, false, false))) return rc;
    int which;
    char *h = (char *)stage_acquire(ctx, ib + tb, &which, &rc);
    if (!h) return rc;
    if (!plan.items.empty()) memcpy(h, plan.items.data(), plan.items.size() * sizeof(WorkItem));
    if (!plan.tiles.empty()) memcpy(h + ib, plan.tiles.data(), plan.tiles.size() * sizeof(TileItem));
    HIPCHK(ctx, hipMemcpyAsync(ctx->s_desc.p, h, ib + tb, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->stage[which].ev, ctx->stream));
    ctx->stage[which].pending = true;
    ctx->serv_dirty = false;
    return PILOT_OK;
}

}  // namespace

extern "C" {

int pilot_admit_cost(pilot_ctx *ctx, const pilot_frame *frame, size_t *bytes)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    if (!bytes) return fail(ctx, PILOT_EINVAL, "bytes: NULL");
    int rc = validate_frame(ctx, frame, 0, false);
    if (rc) return rc;
    *bytes = frame_cost(ctx, *frame);
    return PILOT_OK;
}

int pilot_admit(pilot_ctx *ctx, const pilot_frame *frame, const pilot_result *result, int *slot)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    if (!slot) return fail(ctx, PILOT_EINVAL, "slot: NULL");
    *slot = -1;
    int rc = validate_frame(ctx, frame, 0, true);
    if (rc) return rc;
    if (!result || !result->poses_out || !result->cost || !result->iterations || !result->status || !result->best)
        return fail(ctx, PILOT_EINVAL, "result: every output buffer must be non-NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if ((rc = serving_init(ctx))) return rc;
    const size_t cost = frame_cost(ctx, *frame);
    if (ctx->budget && ctx->serv_bytes + cost > ctx->budget)
        return fail(ctx, PILOT_EAGAIN, "HBM budget: %zu bytes in use + %zu needed > %zu", ctx->serv_bytes, cost, ctx->budget);
    int s = -1;
    for (int i = 0; i < (int)ctx->slots.size(); ++i)
        if (!ctx->slots[i].active) {
            s = i;
            break;
        }
    if (s < 0) return fail(ctx, PILOT_EAGAIN, "all %d slots are busy", (int)ctx->slots.size());
    const int base = arena_alloc(ctx, frame->M);
    if (base < 0) return fail(ctx, PILOT_EAGAIN, "hypothesis arena full (%d hypotheses)", ctx->arena_cap);

    FrameDev d{};
    fill_frame_dev(d, *frame, result, base);
    d.slot = s;
    d.done_flag = (int *)ctx->s_done.p + s;
    // Gram tables of the levels whose tiles use a Gram variant, in the slot's own buffer
    ServingSlot &sl = ctx->slots[s];
    size_t gbytes = 0, goff[PILOT_MAX_LEVELS] = {0};
    bool gneed[PILOT_MAX_LEVELS] = {false};
    int gfmt[PILOT_MAX_LEVELS] = {0};
    for (int l = 0; l < frame->n_levels; ++l) {
        const pilot_level &L = frame->level[l];
        const TileConfig tc = serving_tile(ctx, L.C, L.dtype, L.N, frame->M, (long)L.H * L.W);
        d.lv[l].ppg = tc.PPG;
        d.lv[l].pack_min = INT_MAX;          // serving walks contiguous tiles
        if (uses_gram(tc)) {
            gneed[l] = true;
            gfmt[l] = gram_format(tc, L.dtype);
            goff[l] = gbytes;
            gbytes += gram_table_bytes(L, gfmt[l]);
        }
    }
    if (gbytes) {
        if ((rc = ensure(ctx, sl.gram, gbytes, false, false))) {
            arena_release(ctx, base, frame->M);
            return rc;
        }
        for (int l = 0; l < frame->n_levels; ++l)
            if (gneed[l]) d.lv[l].gram = (const double *)((const char *)sl.gram.p + goff[l]);
    }
    // the slot's anchors in spatial order, in its own buffer
    size_t abytes = 0, aoff[PILOT_MAX_LEVELS] = {0};
    bool aneed[PILOT_MAX_LEVELS] = {false};
    int amax = 0;
    for (int l = 0; l < frame->n_levels; ++l)
        if (sorts_anchors(ctx, frame->level[l], frame->M)) {
            aneed[l] = true;
            aoff[l] = abytes;
            abytes += anchor_copy_bytes(frame->level[l]);
            amax = std::max(amax, frame->level[l].N);
        }
    if (abytes) {
        if ((rc = ensure(ctx, sl.anch, abytes, false, false))) {
            arena_release(ctx, base, frame->M);
            return rc;
        }
        for (int l = 0; l < frame->n_levels; ++l)
            if (aneed[l]) place_anchor_copy(d.lv[l], (char *)sl.anch.p + aoff[l]);
    }
    int which;
    char *h = (char *)stage_acquire(ctx, sizeof(FrameDev), &which, &rc);
    if (!h) {
        arena_release(ctx, base, frame->M);
        return rc;
    }
    memcpy(h, &d, sizeof d);
    FrameDev *dst = (FrameDev *)ctx->s_frames.p + s;
    HIPCHK(ctx, hipMemcpyAsync(dst, h, sizeof d, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->stage[which].ev, ctx->stream));
    ctx->stage[which].pending = true;
    HIPCHK(ctx, launch_init(dst, 1, frame->M, (HypState *)ctx->hs.p, (PoseEval *)ctx->pose.p, (int *)ctx->hlev.p,
                            MODE_LM, nullptr, 0, ctx->stream));
    if (abytes) HIPCHK(ctx, launch_anchor_sort(dst, 1, frame->n_levels, amax, ctx->stream));
    for (int l = 0; l < frame->n_levels; ++l)
        if (gneed[l]) {
            const pilot_level &L = frame->level[l];
            HIPCHK(ctx, launch_gram(dst, 0, l, L.H, L.W, L.C, L.dtype, gfmt[l], ctx->stream));
        }
    sl.dev = d;
    sl.active = true;
    sl.M = frame->M;
    sl.hyp_base = base;
    sl.bytes = cost;
    sl.admit_step = ctx->steps_enqueued;
    sl.frame = *frame;
    ctx->serv_bytes += cost;
    ctx->serv_dirty = true;
    *slot = s;
    return PILOT_OK;
}

int pilot_step(pilot_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    ctx->err.clear();
    if (ctx->n_active() == 0) return PILOT_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int rc;
    if (ctx->serv_dirty && (rc = serving_rebuild(ctx))) return rc;
    // at most two steps in flight: step k+1 waits for step k-1
    if (ctx->steps_enqueued >= 1) {
        pilot_ctx::FlagBuf &old = ctx->flagbuf[(ctx->steps_enqueued - 1) % kFlagRing];
        if (old.used && old.step == ctx->steps_enqueued - 1) HIPCHK(ctx, hipEventSynchronize(old.ev));
    }
    const Plan &plan = ctx->serv_plan;
    const size_t ib = align256(std::max<size_t>(1, plan.items.size()) * sizeof(WorkItem));
    DevPtrs dp;
    dp.frames = (FrameDev *)ctx->s_frames.p;
    dp.items = (WorkItem *)ctx->s_desc.p;
    dp.tiles = (TileItem *)((char *)ctx->s_desc.p + ib);
    // a serving step runs every level over every active slot, so most tiles of
    // a launch are at other levels: its epilogues test the tile mask first
    for (int l = 0; l < PILOT_MAX_LEVELS; ++l)
        for (const LaunchGroup &g : plan.groups)
            if (g.level == l && (rc = enqueue_pass(ctx, plan, dp, ws_of(ctx), g, MODE_LM, ctx->stream,
                                                   (ctx->flags & PILOT_FLAG_PROFILE) != 0, nullptr, nullptr, true)))
                return rc;
    bool prunes = false;
    for (const ServingSlot &sl : ctx->slots) prunes = prunes || (sl.active && sl.frame.keep_top > 0);
    if (prunes)
        HIPCHK(ctx, launch_prune(dp.frames, (int)ctx->slots.size(), (HypState *)ctx->hs.p, (PoseEval *)ctx->pose.p,
                                 (int *)ctx->hlev.p, ctx->stream));
    HIPCHK(ctx, launch_finalize(dp.frames, (int)ctx->slots.size(), (const HypState *)ctx->hs.p,
                                (const int *)ctx->hlev.p, ctx->stream));
    ctx->steps_enqueued++;
    pilot_ctx::FlagBuf &fb = ctx->flagbuf[ctx->steps_enqueued % kFlagRing];
    if (fb.used) HIPCHK(ctx, hipEventSynchronize(fb.ev));
    HIPCHK(ctx, hipMemcpyAsync(fb.host, ctx->s_done.p, ctx->slots.size() * sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipEventRecord(fb.ev, ctx->stream));
    fb.step = ctx->steps_enqueued;
    fb.used = true;
    return PILOT_OK;
}

int pilot_poll(pilot_ctx *ctx, int slot)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    if (slot < 0 || slot >= (int)ctx->slots.size() || !ctx->slots[slot].active)
        return fail(ctx, PILOT_EINVAL, "slot %d is not an active serving slot", slot);
    ServingSlot &sl = ctx->slots[slot];
    // newest completed flag copy taken after this slot's admission
    const pilot_ctx::FlagBuf *best = nullptr;
    for (const auto &fb : ctx->flagbuf) {
        if (!fb.used || fb.step <= sl.admit_step) continue;
        if (best && fb.step < best->step) continue;
        const hipError_t q = hipEventQuery(fb.ev);
        if (q == hipSuccess)
            best = &fb;
        else if (q != hipErrorNotReady)
            return fail(ctx, PILOT_EDEVICE, "hipEventQuery: %s", hipGetErrorString(q));
    }
    if (!best || !best->host[slot]) return 0;
    // The slot's device descriptor is cleared (M = 0) behind the steps already
    // enqueued: the prune and finalize kernels of later steps walk every slot,
    // and a stale descriptor would rank or write the hypotheses of whichever
    // frame is given this slot's hypothesis range next.
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipMemsetAsync((FrameDev *)ctx->s_frames.p + slot, 0, sizeof(FrameDev), ctx->stream));
    arena_release(ctx, sl.hyp_base, sl.M);
    ctx->serv_bytes -= sl.bytes;
    DevBuf gram = sl.gram, anch = sl.anch;   // the slot keeps its buffers for the next frame
    sl = ServingSlot();
    sl.gram = gram;
    sl.anch = anch;
    ctx->serv_dirty = true;
    return 1;
}

int pilot_sync(pilot_ctx *ctx)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PILOT_OK;
}

int pilot_serving_state(pilot_ctx *ctx, int *active_slots, size_t *bytes_in_use)
{
    if (!ctx) return fail(nullptr, PILOT_EINVAL, "ctx: NULL");
    if (active_slots) *active_slots = ctx->n_active();
    if (bytes_in_use) *bytes_in_use = ctx->serv_bytes;
    return PILOT_OK;
}

}  // extern "C"
