// pilot_kernels.hip -- hypothesis-state initialisation, result finalisation
// (with the best-hypothesis selection) and the pass-kernel dispatch.
#include "pilot_kernels.h"
#include "pilot_lm.h"

namespace pilot {

hipError_t launch_pass_c16(int, const TileConfig &, const PassArgs &, hipStream_t);
hipError_t launch_pass_c32(int, const TileConfig &, const PassArgs &, hipStream_t);
hipError_t launch_pass_c64(int, const TileConfig &, const PassArgs &, hipStream_t);
hipError_t launch_pass_c128(int, const TileConfig &, const PassArgs &, hipStream_t);
hipError_t launch_pass_c256(int, const TileConfig &, const PassArgs &, hipStream_t);

bool pass_supported(int C, int dtype, int G)
{
    if (dtype != 0 && dtype != 1) return false;
    if (G != 4 && G != 8 && G != 16) return false;
    return C == 16 || C == 32 || C == 64 || C == 128 || C == 256;
}

hipError_t launch_pass(int C, int dtype, const TileConfig &tc, const PassArgs &a, hipStream_t s)
{
    switch (C) {
    case 16: return launch_pass_c16(dtype, tc, a, s);
    case 32: return launch_pass_c32(dtype, tc, a, s);
    case 64: return launch_pass_c64(dtype, tc, a, s);
    case 128: return launch_pass_c128(dtype, tc, a, s);
    case 256: return launch_pass_c256(dtype, tc, a, s);
    default: return hipErrorInvalidValue;
    }
}

constexpr int kMaxG = 16;

// One block per hypothesis tile: kEpiThreads threads sum the tile's per-item
// partials in FP64 in item order (fixed, independent of what else shares the
// launch) while one more wave evaluates the prior terms at each hypothesis'
// pending pose; then one thread per hypothesis adds the priors and advances
// its LM state (or writes the diagnostic system).
constexpr int kEpiThreads = 512;
constexpr int kEpiBlock = kEpiThreads + 64;

__global__ __launch_bounds__(kEpiBlock) void epilogue_kernel(EpilogueArgs e)
{
    __shared__ double s_sum[kMaxG][kNV];
    __shared__ double s_part[4 * kEpiThreads];     // R x G x kNV partial sums
    __shared__ HypState s_hs[kMaxG];
    __shared__ PoseEval s_pe[kMaxG];
    __shared__ PriorTerms s_pri[kMaxG];
    __shared__ FrameDev s_f;
    __shared__ unsigned s_keep;
    __shared__ int s_pos;
    // one block per tile: the tile's own mask (lane hh < nh of each wave reads
    // the level of hypothesis hb + hh) also covers a level with no hypothesis
    // left, so the run flag is not read here.  By default the levels, the LM
    // states, the poses and the partial sums are all fetched in one load round
    // trip: the loads below do not wait for the mask, which is only tested
    // (uniformly over the block) before the first barrier.  With mask_first
    // (launches where most tiles have no hypothesis at the level) an inactive
    // tile exits after the level loads instead.
    const TileItem ti = e.tiles[blockIdx.x];
    const FrameDev *f = e.frames + ti.frame;
    const int G = e.G;
    const int hb = ti.hbase;
    // With packed lists (e.phs) the tiling of this frame in this pass is the
    // pass kernel's (use_packed on the same count): packed, slot hh is packed
    // entry hb + hh, the first nh slots still at the level; otherwise
    // hypothesis hb + hh.  Either way the survivors are appended to the next
    // pass's lists.
    const bool lists = e.phs != nullptr;
    const int cnt = lists ? e.pcount[ti.frame] : 0;
    const bool packed = lists && use_packed(cnt, f->M, G, ti.n_ptiles, f->lv[e.level].pack_min);
    const int nh = packed ? min(ti.nh, cnt - ti.htile * G) : ti.nh;
    if (packed && nh <= 0) return;               // past the hypotheses still at the level
    const HypState *hs_in = (packed ? e.phs : e.hs) + hb;
    const PoseEval *pe_in = (packed ? e.ppose : e.pose) + hb;
    const int lane = threadIdx.x & 63;
    const int lv = lane < nh ? (packed ? e.level : e.hlev[hb + lane]) : -1;
    if (e.mask_first && __builtin_amdgcn_readfirstlane((unsigned)__ballot(lv == e.level)) == 0) return;
    // LM states and poses of the tile's hypotheses and the frame's constants,
    // fetched by the summing threads and staged in LDS (the LM step then reads
    // its parameters there rather than one dependent global load at a time)
    constexpr int kHsW = sizeof(HypState) / sizeof(double), kPeW = sizeof(PoseEval) / sizeof(double);
    constexpr int kFdW = sizeof(FrameDev) / sizeof(unsigned long long);
    static_assert(sizeof(FrameDev) % sizeof(unsigned long long) == 0 && kFdW <= kEpiThreads, "frame staging shape");
    static_assert(sizeof(HypState) % sizeof(double) == 0 && kMaxG * kHsW <= 3 * kEpiThreads &&
                      kMaxG * kPeW <= kEpiThreads, "state prefetch shape");
    const bool lm_mode = e.mode != MODE_DIAG;
    const int nhs = lm_mode ? nh * kHsW : 0, npe = lm_mode ? nh * kPeW : 0;
    const int stride = G * kNV;
    const int Q = stride / 4;
    const int R = kEpiThreads / Q;
    if (threadIdx.x >= kEpiThreads) {
        // the prior wave: lane hh evaluates the prior terms of hypothesis hh at
        // the pose the pass evaluated (the level's start pose, else the
        // candidate); inactive hypotheses are evaluated too (their terms go
        // unused: the DSM lookup clamps to the grid whatever the pose)
        const int hh = threadIdx.x - kEpiThreads;
        if (lm_mode && hh < nh) {
            const HypState &hs = hs_in[hh];
            const bool start = hs.phase == PHASE_START;
            double Tp[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                const double a = hs.T[i], c = hs.Tc[i];
                Tp[i] = start ? a : c;
            }
            PriorTerms p{};
            prior_terms(*f, Tp, p);
            s_pri[hh] = p;
        }
    } else {
        double hsv[3], pev = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int w = threadIdx.x + k * kEpiThreads;
            hsv[k] = w < nhs ? reinterpret_cast<const double *>(hs_in)[w] : 0.0;
        }
        if ((int)threadIdx.x < npe) pev = reinterpret_cast<const double *>(pe_in)[threadIdx.x];
        unsigned long long fdv = 0;
        if (threadIdx.x < kFdW) fdv = reinterpret_cast<const unsigned long long *>(f)[threadIdx.x];
        // The tile's records are read as float4 columns (4 adjacent values; a
        // hypothesis' 32 slots are 8 columns, the last holding the FP64 cost bits).
        // R threads per column: thread (r, q) sums the items r, r + R, r + 2R, ...
        // of column q, issuing the loads of 8 items before adding them in item
        // order; then the R partial sums are added in r order.  The order depends
        // on the tile shape only.
        const int q = threadIdx.x % Q, r = threadIdx.x / Q;
        {
            const bool cost_col = (q % (kNV / 4)) == kCostSlot / 4;
            const float4 *src = reinterpret_cast<const float4 *>(e.partials + (size_t)ti.first_item * stride) + q;
            const int n = ti.n_ptiles;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int it = r;
            for (; it + 7 * R < n; it += 8 * R) {
                float4 x[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) x[k] = src[(size_t)(it + k * R) * Q];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (cost_col) {
                        a0 += __longlong_as_double((long long)((unsigned long long)__float_as_uint(x[k].x) |
                                                               ((unsigned long long)__float_as_uint(x[k].y) << 32)));
                    } else {
                        a0 += (double)x[k].x;
                        a1 += (double)x[k].y;
                        a2 += (double)x[k].z;
                        a3 += (double)x[k].w;
                    }
                }
            }
            for (; it < n; it += R) {
                const float4 x = src[(size_t)it * Q];
                if (cost_col) {
                    a0 += __longlong_as_double((long long)((unsigned long long)__float_as_uint(x.x) |
                                                           ((unsigned long long)__float_as_uint(x.y) << 32)));
                } else {
                    a0 += (double)x.x;
                    a1 += (double)x.y;
                    a2 += (double)x.z;
                    a3 += (double)x.w;
                }
            }
            double *dst = s_part + (size_t)r * stride + 4 * q;
            dst[0] = a0;
            dst[1] = cost_col ? 0.0 : a1;
            dst[2] = cost_col ? 0.0 : a2;
            dst[3] = cost_col ? 0.0 : a3;
        }
        {
            double *hs_lds = reinterpret_cast<double *>(s_hs), *pe_lds = reinterpret_cast<double *>(s_pe);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int w = threadIdx.x + k * kEpiThreads;
                if (w < nhs) hs_lds[w] = hsv[k];
            }
            if ((int)threadIdx.x < npe) pe_lds[threadIdx.x] = pev;
            if (threadIdx.x < kFdW) reinterpret_cast<unsigned long long *>(&s_f)[threadIdx.x] = fdv;
        }
    }
    const unsigned act = __builtin_amdgcn_readfirstlane((unsigned)__ballot(lv == e.level));
    if (act == 0) return;
    __syncthreads();
    for (int tv = threadIdx.x; tv < stride; tv += kEpiThreads) {
        const int hh = tv / kNV, v = tv - hh * kNV;
        double sum = 0.0;
        for (int k = 0; k < R; ++k) sum += s_part[(size_t)k * stride + tv];
        s_sum[hh][v] = sum;
    }
    __syncthreads();
    if (threadIdx.x == kEpiThreads)   // the prior wave: not on an LM thread's path
        atomicAdd(e.pairs, (unsigned long long)__popc(act) * (unsigned long long)s_f.lv[e.level].N);
    const int t = threadIdx.x;
    const int gh = (packed && t < nh) ? s_hs[t].home : hb + t;
    const int m = gh - f->hyp_base;
    const double *S = s_sum[t];
    if (!lm_mode) {
        if (t >= G || !((act >> t) & 1u)) return;
        double Hd[21], gd[6];
        for (int i = 0; i < 21; ++i) Hd[i] = S[i];
        for (int i = 0; i < 6; ++i) gd[i] = S[21 + i];
        double cost = S[kCostSlot];
        add_priors(*f, e.hs[gh].T, f->use_g ? f->lam_imu : 0.0, f->use_r ? f->lam_range : 0.0, Hd, gd, cost);
        for (int i = 0; i < 21; ++i) f->diag_H[(size_t)m * 21 + i] = Hd[i];
        for (int i = 0; i < 6; ++i) f->diag_g[(size_t)m * 6 + i] = gd[i];
        f->diag_cost[m] = cost;
        f->diag_n[m] = (int)S[27];
        e.hlev[gh] = -1;
        return;
    }
    // the LM state lives in LDS while it is updated (a register copy of the
    // whole state would not fit beside the reduction's registers)
    bool stay = false;
    if (t < G && ((act >> t) & 1u)) {
        int hl = e.level;
        lm_advance(s_f, s_hs[t], S, s_pri[t], s_pe[t], hl);
        e.hlev[gh] = hl;
        stay = hl == e.level;
        if (e.next_flag && stay) *e.next_flag = 1;   // the next pass of this level has work
    }
    if (lists) {
        // hypotheses that stay at the level go to the next pass's packed list:
        // one atomic per tile reserves their entries (slot order within the tile)
        const unsigned keep = (unsigned)__ballot(stay);          // t < G <= 16: wave 0 only
        if (threadIdx.x == 0) {
            s_keep = keep;
            s_pos = keep ? atomicAdd(e.pcount_next + ti.frame, __popc(keep)) : 0;
        }
    }
    __syncthreads();
    // write the updated states back with the whole block (active hypotheses only)
    {
        const double *hs_lds = reinterpret_cast<const double *>(s_hs);
        const double *pe_lds = reinterpret_cast<const double *>(s_pe);
        auto home = [&](int hh) -> int { return packed ? s_hs[hh].home : hb + hh; };
        for (int w = threadIdx.x; w < nhs; w += kEpiBlock)
            if ((act >> (w / kHsW)) & 1u) reinterpret_cast<double *>(e.hs + home(w / kHsW))[w % kHsW] = hs_lds[w];
        if ((int)threadIdx.x < npe && ((act >> (threadIdx.x / kPeW)) & 1u))
            reinterpret_cast<double *>(e.pose + home(threadIdx.x / kPeW))[threadIdx.x % kPeW] = pe_lds[threadIdx.x];
        if (lists) {
            // the survivors' states and next poses, to their entries of the next list
            const unsigned keep = s_keep;
            const int dst0 = f->hyp_base + s_pos;
            constexpr int kW = kHsW + kPeW;
            for (int w = threadIdx.x; w < __popc(keep) * kW; w += kEpiBlock) {
                const int r = w / kW, x = w - r * kW;
                int j = 0;
                for (int seen = 0; j < kMaxG; ++j)
                    if (((keep >> j) & 1u) && seen++ == r) break;
                if (x < kHsW) reinterpret_cast<double *>(e.phs_next + dst0 + r)[x] = hs_lds[j * kHsW + x];
                else reinterpret_cast<double *>(e.ppose_next + dst0 + r)[x - kHsW] = pe_lds[j * kPeW + x - kHsW];
            }
        }
    }
}

hipError_t launch_epilogue(const EpilogueArgs &e, hipStream_t s)
{
    if (e.G > kMaxG) return hipErrorInvalidValue;
    if (e.n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(epilogue_kernel, dim3(e.n_tiles), dim3(kEpiBlock), 0, s, e);
    return hipGetLastError();
}

// One thread per hypothesis; blockIdx.y selects the frame.  Block (0, 0) also
// sets the solve's pass flags, if given: flag (l, 0) = 1 (every level's first
// pass runs), the others 0 until an epilogue raises them.
__global__ __launch_bounds__(256) void init_kernel(const FrameDev *frames, HypState *hs, PoseEval *pose,
                                                    int *hlev, int mode, const double *dposes, int dlevel,
                                                    int *flags, int n_flags, int flag_stride)
{
    const FrameDev &f = frames[blockIdx.y];
    if (flags && blockIdx.x == 0 && blockIdx.y == 0)
        for (int i = threadIdx.x; i < n_flags; i += blockDim.x) flags[i] = (i % flag_stride == 0) ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && f.done_flag) *f.done_flag = 0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= f.M) return;
    const int gh = f.hyp_base + m;
    double src[12];
    if (mode == MODE_DIAG) {
        for (int i = 0; i < 12; ++i) src[i] = dposes[(size_t)12 * m + i];
    } else if (f.hyp_offsets) {
        // hypothesis m around the prior: centre += (dx, dy, 0), R_wc <- Rz(dyaw) R_wc
        // (a positive dyaw turns the camera counter-clockwise seen from above),
        // i.e. R <- R Rz(-dyaw), t <- -R C
        const int b = f.prior_best ? max(*f.prior_best, 0) : 0;
        const double *T = f.prior_poses + (size_t)12 * b;
        const double dx = f.hyp_offsets[3 * m], dy = f.hyp_offsets[3 * m + 1], dz = f.hyp_offsets[3 * m + 2];
        double Cw[3];
        for (int i = 0; i < 3; ++i) Cw[i] = -(T[i] * T[9] + T[3 + i] * T[10] + T[6 + i] * T[11]);   // -R^T t
        Cw[0] += dx;
        Cw[1] += dy;
        double sz, cz;
        sincos(dz, &sz, &cz);
        for (int r = 0; r < 3; ++r) {
            const double a0 = T[3 * r], a1 = T[3 * r + 1];
            src[3 * r] = a0 * cz - a1 * sz;           // R Rz(-dyaw): columns 0, 1 rotate
            src[3 * r + 1] = a0 * sz + a1 * cz;
            src[3 * r + 2] = T[3 * r + 2];
        }
        for (int r = 0; r < 3; ++r) src[9 + r] = -(src[3 * r] * Cw[0] + src[3 * r + 1] * Cw[1] + src[3 * r + 2] * Cw[2]);
    } else {
        for (int i = 0; i < 12; ++i) src[i] = f.poses_in[(size_t)12 * m + i];
    }
    HypState s{};
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        s.T[i] = src[i];
        s.Tc[i] = src[i];
        finite = finite && isfinite(src[i]);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        s.dxi[i] = 0.0;
        s.g[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < 21; ++i) s.H[i] = 0.0;
    s.cost = __longlong_as_double(0x7ff8000000000000LL);   // NaN until evaluated
    s.lam = s.lmin = s.lmax = 0.0;
    s.alpha[0] = f.use_g ? f.lam_imu : 0.0;
    s.alpha[1] = f.use_r ? f.lam_range : 0.0;
    s.level = (mode == MODE_DIAG) ? dlevel : 0;
    s.phase = PHASE_START;
    s.it_level = s.it_total = 0;
    s.status = finite ? ST_MAX_ITERS : ST_DEGENERATE;
    s.nvalid = 0;
    s.home = gh;
    s.pad1 = 0;
    hs[gh] = s;
    PoseEval p{};
#pragma unroll
    for (int i = 0; i < 12; ++i) p.v[i] = src[i];
#pragma unroll
    for (int i = 12; i < 16; ++i) p.v[i] = 0.0;
    pose[gh] = p;
    hlev[gh] = finite ? s.level : -1;
}

hipError_t launch_init(const FrameDev *frames, int n_frames, int max_M, HypState *hs, PoseEval *pose,
                       int *hlev, int mode, const double *diag_poses, int diag_level, hipStream_t s, int *flags,
                       int n_flags, int flag_stride)
{
    if (flags && (n_flags < 0 || flag_stride <= 0)) return hipErrorInvalidValue;
    dim3 grid((max_M + 255) / 256, n_frames), block(256);
    hipLaunchKernelGGL(init_kernel, grid, block, 0, s, frames, hs, pose, hlev, mode, diag_poses, diag_level, flags,
                       n_flags, flag_stride);
    return hipGetLastError();
}

// One block per frame.  Writes poses, costs, iterations and statuses and the
// index of the lowest final cost among non-degenerate hypotheses (NaN never
// wins, ties go to the lowest index) once every hypothesis has finished.
__global__ __launch_bounds__(256) void finalize_kernel(const FrameDev *frames, const HypState *hs,
                                                        const int *hlev)
{
    const FrameDev &f = frames[blockIdx.x];
    if (f.M <= 0) return;                          // unused serving slot
    __shared__ double s_cost[256];
    __shared__ int s_idx[256];
    // The done flag, the levels and the states of the first 256 hypotheses are
    // fetched in one load round trip; nothing is written unless the frame is
    // not yet finalised and none of its hypotheses is still running.
    const int done = f.done_flag ? *f.done_flag : 0;
    int pending = 0;
    for (int m = threadIdx.x; m < f.M; m += blockDim.x) pending |= (hlev[f.hyp_base + m] != -1);
    double T0[12], cost0 = 0.0, al0 = 0.0, al1 = 0.0;
    int it0 = 0, st0 = 0;
    const bool has0 = (int)threadIdx.x < f.M;
    if (has0) {
        const HypState &s = hs[f.hyp_base + threadIdx.x];
#pragma unroll
        for (int i = 0; i < 12; ++i) T0[i] = s.T[i];
        cost0 = s.cost;
        it0 = s.it_total;
        st0 = s.status;
        al0 = s.alpha[0];
        al1 = s.alpha[1];
    }
    if (done) return;                              // the same value in every thread
    if (__syncthreads_or(pending)) return;

    double bc = 0.0;
    int bi = -1;
    for (int m = threadIdx.x; m < f.M; m += blockDim.x) {
        double T[12], cost, a0, a1;
        int it, st;
        if (m == (int)threadIdx.x) {
#pragma unroll
            for (int i = 0; i < 12; ++i) T[i] = T0[i];
            cost = cost0, it = it0, st = st0, a0 = al0, a1 = al1;
        } else {
            const HypState &s = hs[f.hyp_base + m];
#pragma unroll
            for (int i = 0; i < 12; ++i) T[i] = s.T[i];
            cost = s.cost, it = s.it_total, st = s.status, a0 = s.alpha[0], a1 = s.alpha[1];
        }
#pragma unroll
        for (int i = 0; i < 12; ++i) f.poses_out[(size_t)12 * m + i] = T[i];
        f.cost_out[m] = cost;
        f.iters_out[m] = it;
        f.status_out[m] = st;
        if (f.alpha_out) {
            f.alpha_out[2 * m] = a0;
            f.alpha_out[2 * m + 1] = a1;
        }
        if (st != ST_DEGENERATE && st != ST_PRUNED && isfinite(cost) && (bi < 0 || cost < bc)) {
            bc = cost;
            bi = m;
        }
    }
    s_cost[threadIdx.x] = bc;
    s_idx[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            const int j = threadIdx.x + w;
            const int ia = s_idx[threadIdx.x], ib = s_idx[j];
            if (ib >= 0 && (ia < 0 || s_cost[j] < s_cost[threadIdx.x] ||
                            (s_cost[j] == s_cost[threadIdx.x] && ib < ia))) {
                s_cost[threadIdx.x] = s_cost[j];
                s_idx[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *f.best_out = s_idx[0];
        if (f.done_flag) {
            __threadfence_system();
            *f.done_flag = 1;
        }
    }
}

// Top-K pruning, one block per frame: once no hypothesis of the frame is
// still at or before its pruning level (all are waiting or finished), rank
// the waiting ones by cost (ties to the lower index) and let the keep_top
// best continue at the next level; the others end as PRUNED.
constexpr int kPruneMaxM = 8192;

__global__ __launch_bounds__(256) void prune_kernel(const FrameDev *frames, HypState *hs, PoseEval *pose,
                                                     int *hlev)
{
    const FrameDev &f = frames[blockIdx.x];
    if (f.M <= 0 || f.keep_top <= 0) return;
    __shared__ double s_cost[kPruneMaxM];
    int waiting = 0, busy = 0;
    for (int m = threadIdx.x; m < f.M; m += blockDim.x) {
        const int h = hlev[f.hyp_base + m];
        waiting |= (h == HLEV_WAIT);
        busy |= (h >= 0 && h <= f.prune_level);
        const double c = hs[f.hyp_base + m].cost;
        s_cost[m] = (h == HLEV_WAIT) ? (isnan(c) ? __longlong_as_double(0x7ff0000000000000LL) : c)
                                     : __longlong_as_double(0x7ff8000000000000LL);   // NaN: not ranked
    }
    if (!__syncthreads_or(waiting) || __syncthreads_or(busy)) return;
    for (int m = threadIdx.x; m < f.M; m += blockDim.x) {
        const double cm = s_cost[m];
        if (isnan(cm)) continue;
        int better = 0;
        for (int j = 0; j < f.M; ++j) {
            const double cj = s_cost[j];
            better += (!isnan(cj) && (cj < cm || (cj == cm && j < m))) ? 1 : 0;
        }
        HypState &s = hs[f.hyp_base + m];
        if (better < f.keep_top) {
            s.level = f.prune_level + 1;
            s.phase = PHASE_START;
            for (int i = 0; i < 12; ++i) pose[f.hyp_base + m].v[i] = s.T[i];
            hlev[f.hyp_base + m] = s.level;
        } else {
            s.status = ST_PRUNED;
            hlev[f.hyp_base + m] = HLEV_DONE;
        }
    }
}

hipError_t launch_prune(const FrameDev *frames, int n_frames, HypState *hs, PoseEval *pose, int *hlev, hipStream_t s)
{
    hipLaunchKernelGGL(prune_kernel, dim3(n_frames), dim3(256), 0, s, frames, hs, pose, hlev);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Gram tables
// Per cell (x0, y0), x0 <= W-2, y0 <= H-2: with the cell's taps in
// the bilinear coefficient basis c = (t00, t10 - t00, t01 - t00,
// t11 - t10 - t01 + t00), K = sum over channels of c c^T, upper triangle row
// by row, in FP64 (products of two f32 or bf16 values are exact in FP64).
template <int DT>
__device__ inline void load4(const void *base, size_t off, double out[4])
{
    if constexpr (DT == 0) {
        const float4 v = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(base) + off);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        const uint2 v = *reinterpret_cast<const uint2 *>(reinterpret_cast<const uint16_t *>(base) + off);
        out[0] = __uint_as_float(v.x << 16);
        out[1] = __uint_as_float(v.x & 0xffff0000u);
        out[2] = __uint_as_float(v.y << 16);
        out[3] = __uint_as_float(v.y & 0xffff0000u);
    }
}

// sum over the 4 lanes of an aligned lane quad (DPP quad permutes)
__device__ __forceinline__ double quad_sum(double v)
{
    auto perm = [](double x, int ctrl) {
        const long long b = __double_as_longlong(x);
        int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
        if (ctrl == 0) {
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
        } else {
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
        }
        return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
    };
    v += perm(v, 0);
    v += perm(v, 1);
    return v;
}

// A lane quad per cell: lane q of the quad takes channels 4q + 16k .. +3, so
// the quad's loads of one tap are one contiguous 64-byte run.  Blocks are
// dealt to the 8 XCDs round-robin; the block index is remapped so that each
// XCD walks one contiguous band of cell rows, and the map row shared by two
// consecutive cell rows is read into one XCD's L2 rather than two.
// The map, its shape and the table are read from the frame descriptor in
// device memory (not passed by value), so a captured graph replayed for a new
// frame of the same shape builds the new frame's tables.
// F32: the record format of pass variants 9 and 10, the ten entries rounded
// to FP32 and two zero pads (48 bytes per cell); otherwise ten FP64 entries.
template <int DT, bool F32>
__global__ __launch_bounds__(256) void gram_kernel(const FrameDev *frames, int fi, int level)
{
    const LevelDev &L = frames[fi].lv[level];
    const void *feat = L.feat;
    const int H = L.H, W = L.W, C = L.C;
    double *gram = const_cast<double *>(L.gram);
    const unsigned nb = gridDim.x, xcd = blockIdx.x % 8u, per = nb / 8u, rem = nb % 8u;
    const unsigned lb = xcd * per + min(xcd, rem) + blockIdx.x / 8u;
    const long cell = ((long)lb * blockDim.x + threadIdx.x) >> 2;
    const int q = threadIdx.x & 3;
    const bool live = cell < (long)H * W;
    const int y0 = live ? (int)(cell / W) : 0, x0 = live ? (int)(cell - (long)y0 * W) : 0;
    const bool work = live && x0 <= W - 2 && y0 <= H - 2;   // no cell starts on the last row or column
    double k[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) k[i] = 0.0;
    if (work) {
        const size_t o = (size_t)cell * C, oW = o + (size_t)W * C;
        for (int c = 4 * q; c < C; c += 16) {
            double t0[4], t1[4], t2[4], t3[4];
            load4<DT>(feat, o + c, t0);
            load4<DT>(feat, o + C + c, t1);
            load4<DT>(feat, oW + c, t2);
            load4<DT>(feat, oW + C + c, t3);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double c0 = t0[e], c1 = t1[e] - t0[e], c2 = t2[e] - t0[e], c3 = (t3[e] - t2[e]) - c1;
                k[0] = fma(c0, c0, k[0]);
                k[1] = fma(c0, c1, k[1]);
                k[2] = fma(c0, c2, k[2]);
                k[3] = fma(c0, c3, k[3]);
                k[4] = fma(c1, c1, k[4]);
                k[5] = fma(c1, c2, k[5]);
                k[6] = fma(c1, c3, k[6]);
                k[7] = fma(c2, c2, k[7]);
                k[8] = fma(c2, c3, k[8]);
                k[9] = fma(c3, c3, k[9]);
            }
        }
    }
    // every lane of the wave takes part in the quad sums (inactive cells add zeros)
#pragma unroll
    for (int i = 0; i < 10; ++i) k[i] = quad_sum(k[i]);
    if (work) {
        if constexpr (F32) {
            float *out = (float *)gram + (size_t)12 * cell;
            for (int i = q; i < 12; i += 4) out[i] = i < 10 ? (float)k[i] : 0.0f;
        } else {
            double *out = gram + (size_t)10 * cell;
            for (int i = q; i < 10; i += 4) out[i] = k[i];
        }
    }
}

hipError_t launch_gram(const FrameDev *frames, int frame, int level, int H, int W, int C, int dtype, int fmt,
                       hipStream_t s)
{
    const long cells = (long)H * W;
    if (cells <= 0 || C % 16) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((4 * cells + 255) / 256)), block(256);
    if (fmt == 1) {
        if (dtype == 0)
            hipLaunchKernelGGL((gram_kernel<0, true>), grid, block, 0, s, frames, frame, level);
        else
            hipLaunchKernelGGL((gram_kernel<1, true>), grid, block, 0, s, frames, frame, level);
    } else {
        if (dtype == 0)
            hipLaunchKernelGGL((gram_kernel<0, false>), grid, block, 0, s, frames, frame, level);
        else
            hipLaunchKernelGGL((gram_kernel<1, false>), grid, block, 0, s, frames, frame, level);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ anchor lift
__device__ inline double bilinear_clamped(const float *F, const uint16_t *Fb, int H, int W, int C, int c,
                                          double u, double v)
{
    u = fmin(fmax(u, 0.0), W - 1.0);
    v = fmin(fmax(v, 0.0), H - 1.0);
    const int x0 = min((int)u, W - 2), y0 = min((int)v, H - 2);
    const double a = u - x0, b = v - y0;
    const size_t o = ((size_t)y0 * W + x0) * C + c;
    auto at = [&](size_t k) -> double {
        return F ? (double)F[k] : (double)__uint_as_float(((uint32_t)Fb[k]) << 16);
    };
    const double f00 = at(o), f10 = at(o + C), f01 = at(o + (size_t)W * C), f11 = at(o + (size_t)W * C + C);
    const double top = f00 + a * (f10 - f00), bot = f01 + a * (f11 - f01);
    return top + b * (bot - top);
}

__device__ inline uint16_t to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN stays NaN
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// One thread per (anchor, channel); channel 0 also writes the lifted point.
__global__ __launch_bounds__(256) void lift_kernel(const float *dsm, int Hd, int Wd, double x0, double y0, double gsd,
                                                    const float *uv, int N, const void *ref_map, int Hr, int Wr, int C,
                                                    int dtype, double scale, float *x, float *y, float *z, void *ref_out)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)N * C) return;
    const int j = (int)(t / C), c = (int)(t - (size_t)j * C);
    const double u = uv[2 * j], v = uv[2 * j + 1];
    if (c == 0) {
        if (x) x[j] = (float)(x0 + u * gsd);
        if (y) y[j] = (float)(y0 + v * gsd);
        if (z) z[j] = (float)bilinear_clamped(dsm, nullptr, Hd, Wd, 1, 0, u, v);
    }
    const double val = bilinear_clamped(dtype == 0 ? (const float *)ref_map : nullptr,
                                        dtype == 0 ? nullptr : (const uint16_t *)ref_map, Hr, Wr, C, c,
                                        scale * (u + 0.5) - 0.5, scale * (v + 0.5) - 0.5);
    if (dtype == 0)
        ((float *)ref_out)[t] = (float)val;
    else
        ((uint16_t *)ref_out)[t] = to_bf16_rne((float)val);
}

hipError_t launch_lift(const float *dsm, int Hd, int Wd, double x0, double y0, double gsd, const float *uv, int N,
                       const void *ref_map, int Hr, int Wr, int C, int dtype, double scale, float *x, float *y,
                       float *z, void *ref_out, hipStream_t s)
{
    const size_t n = (size_t)N * C;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(lift_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dsm, Hd, Wd, x0, y0, gsd, uv, N,
                       ref_map, Hr, Wr, C, dtype, scale, x, y, z, ref_out);
    return hipGetLastError();
}

hipError_t launch_finalize(const FrameDev *frames, int n_frames, const HypState *hs, const int *hlev,
                           hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(n_frames), dim3(256), 0, s, frames, hs, hlev);
    return hipGetLastError();
}

// ------------------------------------------------------------------ packing
// The LM states and poses under evaluation of each frame's hypotheses whose
// pending level is `level`, in index order, to phs / ppose[hyp_base + 0 ..
// count), count to pcount[frame], and the frame's counts in pclear0 and
// pclear1 (the next two passes' append targets) cleared.  Block (c, frame)
// takes hypotheses 16 c .. 16 c + 15: it counts the listed ones before its
// chunk (the hypotheses' level words, a block-wide sum) for the chunk's first
// entry, then copies the chunk's records a word per thread.  Block (0, frame)
// also counts the whole frame.
constexpr int kPackChunk = 16;
constexpr int kPackBlock = 256;

__device__ __forceinline__ int block_count(const int *hlev, int lo, int hi, int level, int *s_red)
{
    int c = 0;
    for (int m = lo + (int)threadIdx.x; m < hi; m += kPackBlock) c += hlev[m] == level;
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = c;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < kPackBlock / 64; ++w) t += s_red[w];
    return t;
}

__global__ __launch_bounds__(kPackBlock) void pack_kernel(const FrameDev *frames, const int *hlev, int level,
                                                          const HypState *hs, const PoseEval *pose, HypState *phs,
                                                          PoseEval *ppose, int *pcount, int *pclear0, int *pclear1)
{
    __shared__ int s_red[kPackBlock / 64];
    __shared__ int s_src[kPackChunk];
    constexpr int kHsW = sizeof(HypState) / sizeof(double), kPeW = sizeof(PoseEval) / sizeof(double);
    constexpr int kW = kHsW + kPeW;
    const FrameDev &f = frames[blockIdx.y];
    const int m0 = blockIdx.x * kPackChunk;
    if (m0 >= f.M) return;
    const int b = f.hyp_base;
    const int before = block_count(hlev, b, b + m0, level, s_red);
    if (blockIdx.x == 0) {
        const int total = block_count(hlev, b, b + f.M, level, s_red);
        if (threadIdx.x == 0) {
            pcount[blockIdx.y] = total;
            pclear0[blockIdx.y] = 0;
            pclear1[blockIdx.y] = 0;
        }
    }
    // the chunk's listed hypotheses, in order (lanes 0..15 of wave 0)
    int n = 0;
    if (threadIdx.x < 64) {
        const int m = m0 + (int)threadIdx.x;
        const bool in = threadIdx.x < kPackChunk && m < f.M && hlev[b + m] == level;
        const unsigned long long bal = __ballot(in);
        if (in) s_src[__popcll(bal & ((1ull << threadIdx.x) - 1ull))] = b + m;
        n = __popcll(bal);
        if (threadIdx.x == 0) s_red[0] = n;
    }
    __syncthreads();
    n = s_red[0];
    const int dst0 = b + before;
    for (int w = threadIdx.x; w < n * kW; w += kPackBlock) {
        const int r = w / kW, x = w - r * kW;
        if (x < kHsW)
            reinterpret_cast<double *>(phs + dst0 + r)[x] = reinterpret_cast<const double *>(hs + s_src[r])[x];
        else
            reinterpret_cast<double *>(ppose + dst0 + r)[x - kHsW] =
                reinterpret_cast<const double *>(pose + s_src[r])[x - kHsW];
    }
}

hipError_t launch_pack(const FrameDev *frames, int n_frames, int max_M, const int *hlev, int level,
                       const HypState *hs, const PoseEval *pose, HypState *phs, PoseEval *ppose, int *pcount,
                       int *pclear0, int *pclear1, hipStream_t s)
{
    if (n_frames <= 0 || max_M <= 0) return hipSuccess;
    const dim3 grid((max_M + kPackChunk - 1) / kPackChunk, n_frames);
    hipLaunchKernelGGL(pack_kernel, grid, dim3(kPackBlock), 0, s, frames, hlev, level, hs, pose, phs, ppose, pcount,
                       pclear0, pclear1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Anchors in spatial order.  The pass kernels walk a level's anchors in array
// order, P at a time per work item, so the locality of their gathers (taps of
// neighbouring anchors under one pose fall in neighbouring cells, sharing
// cache lines in L1 and L2) depends on how the caller listed the anchors.
// The library therefore sorts a level's anchors (the runtime decides which
// levels: enough anchor x hypothesis pairs per pass to repay the sort) by the
// Morton code of their ground position (x, y quantised to 256 x 256 cells
// over the level's bounding box) before the first pass and walks its own
// copies.  The sums over anchors change only in their rounding order; the
// order is a function of the anchor set alone (ties of one cell keep the
// caller's order).

namespace {
constexpr int kSortThreads = 1024;
typedef uint32_t row16 __attribute__((ext_vector_type(4)));   // 16 bytes of a reference row

// The thread index, opaque to the optimiser: element indices derived from it
// are recomputed in each loop instead of being kept live (and spilled)
// across the whole kernel.
__device__ __forceinline__ int fresh_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ uint32_t spread_bits8(uint32_t v)
{
    v &= 0xffu;
    v = (v | (v << 4)) & 0x0f0fu;
    v = (v | (v << 2)) & 0x3333u;
    v = (v | (v << 1)) & 0x5555u;
    return v;
}
}  // namespace

// One block per (level, frame): keys (Morton code << 16 | caller index) in
// LDS, sorted on the 12-bit code by a stable least-significant-digit radix
// sort (three passes of 4 bits), so anchors of one cell keep the caller's
// order; perm[j] = caller index of the j-th anchor in spatial order.
//
// A pass over element i = r kSortThreads + tid (r < kSortPer): the 32
// elements of one half-wave and round form group i / 32 (groups in element
// order).  Each element learns from four ballots the lanes of its group with
// the same digit (its rank among them, and the leader of them writes their
// count to cnt[group][digit]); the waves then scan each digit's counts over
// the groups, and a second sweep moves every element to the start of its
// digit + the count of its digit in the groups before its own + its rank.
// The passes alternate between the keys in LDS and the permutation buffer
// (global memory, N words), so no pass holds its keys in registers.
template <int kSortPer>   // anchors per thread: N <= kSortPer kSortThreads
__global__ __launch_bounds__(kSortThreads) void sort_anchors_kernel(const FrameDev *frames)
{
    constexpr int kCap = kSortPer * kSortThreads;
    __shared__ uint32_t s_key[kCap];
    constexpr int kGroups = kCap / 32, kStride = kGroups + 2;   // padded rows: no bank conflicts
    __shared__ unsigned short s_cnt[16][kStride];   // [digit][group]
    __shared__ uint32_t s_dtot[16], s_dstart[16];
    __shared__ float s_bb[kSortThreads / 64][4];
    const FrameDev &f = frames[blockIdx.y];
    const int l = blockIdx.x;
    if (l >= f.n_levels) return;
    const LevelDev &L = f.lv[l];
    int *perm = L.perm;
    const int N = L.N;
    if (!perm || N <= 0 || N > kCap) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    typedef const __attribute__((address_space(1))) float gfloat;
    gfloat *xs = (gfloat *)L.in_x, *ys = (gfloat *)L.in_y;
    // the thread's anchors tid + r kSortThreads, loaded in one round trip
    // (clamped indices: no branch between the loads), and the bounding box of
    // their ground positions (as -min, max, so every step is a max; repeats
    // of anchor N - 1 change no extreme)
    float xv[kSortPer], yv[kSortPer];
    float b[4] = {-3.4e38f, -3.4e38f, -3.4e38f, -3.4e38f};
    {
        const int tl = fresh_tid();
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int i = min(tl + r * kSortThreads, N - 1);
            xv[r] = xs[i];
            yv[r] = ys[i];
        }
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            b[0] = fmaxf(b[0], -xv[r]);
            b[1] = fmaxf(b[1], xv[r]);
            b[2] = fmaxf(b[2], -yv[r]);
            b[3] = fmaxf(b[3], yv[r]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int sft = 1; sft < 64; sft <<= 1) b[k] = fmaxf(b[k], __shfl_xor(b[k], sft, 64));
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) s_bb[wave][k] = b[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b[k] = s_bb[0][k];
        for (int w = 1; w < kSortThreads / 64; ++w) b[k] = fmaxf(b[k], s_bb[w][k]);
    }
    const float x0 = -b[0], y0 = -b[2];
    const float sx = b[1] + b[0] > 0.0f ? 256.0f / (b[1] + b[0]) : 0.0f;
    const float sy = b[3] + b[2] > 0.0f ? 256.0f / (b[3] + b[2]) : 0.0f;
    const int tk = fresh_tid();
#pragma unroll
    for (int r = 0; r < kSortPer; ++r) {
        const int i = tk + r * kSortThreads;
        if (i < N) {
            const uint32_t qx = (uint32_t)fminf(fmaxf((xv[r] - x0) * sx, 0.0f), 255.0f);
            const uint32_t qy = (uint32_t)fminf(fmaxf((yv[r] - y0) * sy, 0.0f), 255.0f);
            s_key[i] = ((spread_bits8(qx) | (spread_bits8(qy) << 1)) << 16) | (uint32_t)i;
        }
    }
    const int ngroups = (N + 31) >> 5;
    const uint32_t below = (1u << (lane & 31)) - 1u;
    const bool upper = lane >= 32;
    typedef __attribute__((address_space(1))) uint32_t guint;
    guint *gk = (guint *)perm;     // the other buffer of the passes (N words)
    // the keys of the thread's elements in the pass's source, loaded in one
    // round trip (indices beyond N read a valid slot and go unused)
    auto load_keys = [&](bool from_lds, uint32_t (&kv)[kSortPer]) {
        const int t = fresh_tid();
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            const int i = t + r * kSortThreads;
            kv[r] = from_lds ? s_key[min(i, kCap - 1)] : gk[min(i, N - 1)];
        }
    };
    // the lanes of element i's group (its half of the wave) with the same digit d
    auto peers_of = [&](int i, uint32_t d) {
        const unsigned long long v = __ballot(i < N);
        uint32_t peers = upper ? (uint32_t)(v >> 32) : (uint32_t)v;
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            const unsigned long long m = __ballot((d >> bit) & 1u);
            const uint32_t mh = upper ? (uint32_t)(m >> 32) : (uint32_t)m;
            peers &= ((d >> bit) & 1u) ? mh : ~mh;
        }
        return peers;
    };
#pragma unroll 1
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 16 + 4 * pass;
        const bool from_lds = (pass & 1) == 0;    // LDS -> global, then global -> LDS
        for (int e = tid; e < 16 * kStride; e += kSortThreads) (&s_cnt[0][0])[e] = 0;
        __syncthreads();
        {
            uint32_t kv[kSortPer];
            load_keys(from_lds, kv);
            const int ta = fresh_tid();
#pragma unroll
            for (int r = 0; r < kSortPer; ++r) {
                const int i = ta + r * kSortThreads;
                const uint32_t d = (kv[r] >> shift) & 15u;
                const uint32_t peers = peers_of(i, d);
                if (i < N && (peers & below) == 0u) s_cnt[d][i >> 5] = (unsigned short)__popc(peers);
            }
        }
        __syncthreads();
        {
            // wave d: exclusive scan of digit d's counts over the groups, a row
            // of 64 groups at a time
            static_assert(kSortThreads / 64 == 16, "one wave per digit");
            const int d = wave;
            uint32_t carry = 0;
            for (int g0 = 0; g0 < ngroups; g0 += 64) {
                const int g = g0 + lane;
                const uint32_t c = g < ngroups ? s_cnt[d][g] : 0u;
                uint32_t incl = c;
#pragma unroll
                for (int sft = 1; sft < 64; sft <<= 1) {
                    const uint32_t o = __shfl_up(incl, sft, 64);
                    if (lane >= sft) incl += o;
                }
                if (g < ngroups) s_cnt[d][g] = (unsigned short)(carry + incl - c);
                carry += __shfl(incl, 63, 64);
            }
            if (lane == 0) s_dtot[d] = carry;
        }
        __syncthreads();
        if (tid < 16) {
            uint32_t acc = 0;
            for (int d = 0; d < tid; ++d) acc += s_dtot[d];
            s_dstart[tid] = acc;
        }
        __syncthreads();
        {
            uint32_t kv[kSortPer];
            load_keys(from_lds, kv);
            const int tb = fresh_tid();
#pragma unroll
            for (int r = 0; r < kSortPer; ++r) {
                const int i = tb + r * kSortThreads;
                const uint32_t d = (kv[r] >> shift) & 15u;
                const uint32_t peers = peers_of(i, d);
                if (i < N) {
                    const uint32_t dst = s_dstart[d] + s_cnt[d][i >> 5] + (uint32_t)__popc(peers & below);
                    if (from_lds) gk[dst] = kv[r];
                    else s_key[dst] = kv[r];
                }
            }
        }
        __syncthreads();                          // also orders the block's global stores before the next pass
    }
    for (int i = tid; i < N; i += kSortThreads) perm[i] = (int)(s_key[i] & 0xffffu);
}

// Copies of the anchors in perm order: 64 anchors per block, the reference
// rows moved 16 bytes per thread and load.
__global__ __launch_bounds__(256) void gather_anchors_kernel(const FrameDev *frames)
{
    const FrameDev &f = frames[blockIdx.z];
    const int l = blockIdx.y;
    if (l >= f.n_levels) return;
    const LevelDev &L = f.lv[l];
    const int *perm = L.perm;
    const int N = L.N;
    const int a0 = blockIdx.x * 64;
    if (!perm || N > kSortMaxN || a0 >= N) return;
    const int na = min(64, N - a0);
    const int cpr = L.C * (L.dtype == 1 ? 2 : 4) / 16;    // 16-byte chunks per reference row
    const row16 *src = (const row16 *)L.in_ref;
    row16 *dst = (row16 *)const_cast<void *>(L.ref);
    for (int t = threadIdx.x; t < na * cpr; t += 256) {
        const int a = t / cpr, c = t - a * cpr;
        dst[(size_t)(a0 + a) * cpr + c] = src[(size_t)min(max(perm[a0 + a], 0), N - 1) * cpr + c];
    }
    if ((int)threadIdx.x < na) {
        const int a = a0 + threadIdx.x, i = min(max(perm[a], 0), N - 1);
        const_cast<float *>(L.x)[a] = L.in_x[i];
        const_cast<float *>(L.y)[a] = L.in_y[i];
        const_cast<float *>(L.z)[a] = L.in_z[i];
        if (L.in_w) const_cast<float *>(L.ref_w)[a] = L.in_w[i];
    }
}

hipError_t launch_anchor_sort(const FrameDev *frames, int n_frames, int max_levels, int max_N, hipStream_t s)
{
    if (n_frames <= 0 || max_levels <= 0 || max_N <= 0) return hipSuccess;
    if (max_levels > kMaxLevels || max_N > kSortMaxN) return hipErrorInvalidValue;
    const dim3 sg(max_levels, n_frames);
    static_assert(kSortMaxN == 16 * kSortThreads, "sort instantiations");
    if (max_N <= 4 * kSortThreads) hipLaunchKernelGGL(sort_anchors_kernel<4>, sg, dim3(kSortThreads), 0, s, frames);
    else if (max_N <= 8 * kSortThreads) hipLaunchKernelGGL(sort_anchors_kernel<8>, sg, dim3(kSortThreads), 0, s, frames);
    else hipLaunchKernelGGL(sort_anchors_kernel<16>, sg, dim3(kSortThreads), 0, s, frames);
    hipLaunchKernelGGL(gather_anchors_kernel, dim3((max_N + 63) / 64, max_levels, n_frames), dim3(256), 0, s, frames);
    return hipGetLastError();
}

}  // namespace pilot
