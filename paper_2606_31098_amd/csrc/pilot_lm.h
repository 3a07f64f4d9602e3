// pilot_lm.h -- per-hypothesis FP64 epilogue of one LM pass (device code):
// gravity and laser-range prior terms, the damped 6x6 Cholesky solve, the
// SE(3) update and the Levenberg-Marquardt accept/reject control.
#pragma once

#include "pilot_device.h"

namespace pilot {

// index of (a, b), a <= b, in the row-by-row upper triangle of a 6x6
__host__ __device__ constexpr int tri(int a, int b) { return a * 6 - a * (a - 1) / 2 + (b - a); }

// 1/x for finite nonzero x: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// log(1 + q), and rx = 1/(1 + q), for the Cauchy loss.  x = 1 + q (rounded)
// is split as 2^e m with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(t) with
// t = (m - 1)/(m + 1), |t| < 0.172, summed through t^21 (the first omitted
// term is below 2^-60 of the sum); the rounding of 1 + q adds (q - (x - 1))/x.
// Within about 2 ulp of log1p for finite q > -0.5 (the loss argument is a
// weighted squared residual, so q >= 0 up to rounding); a NaN or infinite q
// gives a NaN, which the LM treats as the non-finite cost log1p would give.
__device__ __forceinline__ double log1p_recip(double q, double &rx)
{
    constexpr double ln2_hi = 0x1.62e42fee00000p-1;   // ln 2 to 32 bits: e * ln2_hi is exact
    constexpr double ln2_lo = 0x1.a39ef35793c76p-33;  // ln 2 - ln2_hi
    const double x = 1.0 + q;
    const double u = x - 1.0;                           // exact while x < 2^53 (beyond, corr is negligible)
    rx = recip64(x);
    const double corr = (q - u) * rx;
    double m = __builtin_amdgcn_frexp_mant(x);
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) * recip64(m + 1.0);
    const double t2 = t * t;
    double p = 1.0 / 21.0;
    p = fma(p, t2, 1.0 / 19.0);
    p = fma(p, t2, 1.0 / 17.0);
    p = fma(p, t2, 1.0 / 15.0);
    p = fma(p, t2, 1.0 / 13.0);
    p = fma(p, t2, 1.0 / 11.0);
    p = fma(p, t2, 1.0 / 9.0);
    p = fma(p, t2, 1.0 / 7.0);
    p = fma(p, t2, 1.0 / 5.0);
    p = fma(p, t2, 1.0 / 3.0);
    const double s2 = 2.0 * t;
    const double logm = fma(s2 * t2, p, s2);
    const double de = (double)e;
    return fma(de, ln2_hi, logm + fma(de, ln2_lo, corr));
}

__device__ __forceinline__ void robust_f64(int kind, double b, double s, double &rho, double &drho)
{
    if (kind == 0) {                       // Cauchy: b log(1 + s/b), weight 1/(1 + s/b)
        rho = b * log1p_recip(s * (1.0 / b), drho);
    } else if (kind == 1) {                // Huber
        if (s <= b) {
            rho = s;
            drho = 1.0;
        } else {
            double r = sqrt(b * s);
            rho = 2.0 * r - b;
            drho = b / r;
        }
    } else {
        rho = s;
        drho = 1.0;
    }
}

// SE(3) exponential of xi = (rho, omega): rotation by Rodrigues' formula,
// translation V rho (left Jacobian of SO(3)); Taylor coefficients near 0.
__device__ inline void se3_exp(const double xi[6], double E[12])
{
    const double wx = xi[3], wy = xi[4], wz = xi[5];
    const double t2 = wx * wx + wy * wy + wz * wz;
    double a, b, c;
    if (t2 < 1e-8) {
        a = 1.0 - t2 * (1.0 / 6.0) + t2 * t2 * (1.0 / 120.0);
        b = 0.5 - t2 * (1.0 / 24.0) + t2 * t2 * (1.0 / 720.0);
        c = (1.0 / 6.0) - t2 * (1.0 / 120.0) + t2 * t2 * (1.0 / 5040.0);
    } else {
        const double t = sqrt(t2);
        double s, co;
        sincos(t, &s, &co);
        a = s / t;
        b = (1.0 - co) / t2;
        c = (t - s) / (t2 * t);
    }
    // W = [w]x ; W^2 = w w^T - t2 I
    const double W2[9] = {wx * wx - t2, wx * wy, wx * wz,
                          wy * wx, wy * wy - t2, wy * wz,
                          wz * wx, wz * wy, wz * wz - t2};
    const double W[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double V[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double I = (i == 0 || i == 4 || i == 8) ? 1.0 : 0.0;
        E[i] = I + a * W[i] + b * W2[i];
        V[i] = I + b * W[i] + c * W2[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) E[9 + i] = V[3 * i] * xi[0] + V[3 * i + 1] * xi[1] + V[3 * i + 2] * xi[2];
}

// out = A * B for world->camera poses
__device__ inline void se3_mul(const double A[12], const double B[12], double out[12])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            out[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
        out[9 + i] = A[3 * i] * B[9] + A[3 * i + 1] * B[10] + A[3 * i + 2] * B[11] + A[9 + i];
    }
}

// (H + lam I) x = -g by Cholesky; false if a pivot is not positive/finite.
// 1/sqrt(x) for finite x > 0: the hardware estimate refined by two Newton
// steps (about one ulp).
__device__ __forceinline__ double rsqrt64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * fma(-h * r, r, 1.5);
    r = r * fma(-h * r, r, 1.5);
    return r;
}

// Cholesky factor of H + lam I and the two triangular solves.  Each column
// keeps the reciprocal of its diagonal, 1/L_jj = 1/sqrt(s_jj), so the chain
// of dependent operations holds six reciprocal square roots and no divisions.
__device__ inline bool damped_solve(const double H[21], const double g[6], double lam, double x[6])
{
    double L[21], inv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = H[tri(j, i)] + (i == j ? lam : 0.0);
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[tri(k, i)] * L[tri(k, j)];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                inv[i] = rsqrt64(s);
                L[tri(i, i)] = s * inv[i];
            } else {
                L[tri(j, i)] = s * inv[j];
            }
        }
    }
    // L stored transposed in the upper triangle: L(i,k) = L[tri(k, i)]
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = -g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[tri(k, i)] * y[k];
        y[i] = s * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[tri(i, k)] * x[k];
        x[i] = s * inv[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
        if (!isfinite(x[i])) return false;
    return true;
}

// Bilinear DSM height and gradient (per metre), clamp-to-edge.
__device__ inline void dsm_lookup(const FrameDev &f, double x, double y, double &h, double &hx, double &hy)
{
    double fj = (x - f.dsm_x0) / f.dsm_gsd, fi = (y - f.dsm_y0) / f.dsm_gsd;
    const bool cj = !(fj >= 0.0 && fj <= f.Wd - 1.0), ci = !(fi >= 0.0 && fi <= f.Hd - 1.0);
    fj = fmin(fmax(fj, 0.0), f.Wd - 1.0);
    fi = fmin(fmax(fi, 0.0), f.Hd - 1.0);
    const int j0 = min((int)fj, f.Wd - 2), i0 = min((int)fi, f.Hd - 2);
    const double a = fj - j0, b = fi - i0;
    const float *row0 = f.dsm + (size_t)i0 * f.Wd + j0;
    const float *row1 = row0 + f.Wd;
    const double d00 = row0[0], d01 = row0[1], d10 = row1[0], d11 = row1[1];
    const double top = d00 + a * (d01 - d00), bot = d10 + a * (d11 - d10);
    h = top + b * (bot - top);
    hx = cj ? 0.0 : ((d01 - d00) + b * ((d11 - d10) - (d01 - d00))) / f.dsm_gsd;
    hy = ci ? 0.0 : (bot - top) / f.dsm_gsd;
}

// Gravity residual of Eq. (3) at pose T: gc = R g_world, r = gc - g_imu.
// Under T <- Exp(xi) T the Jacobian is [0 | -[gc]x].
__device__ inline void gravity_residual(const FrameDev &f, const double T[12], double gc[3], double r[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gc[i] = T[3 * i] * f.g_world[0] + T[3 * i + 1] * f.g_world[1] + T[3 * i + 2] * f.g_world[2];
        r[i] = gc[i] - f.g_imu[i];
    }
}

// Range residual of Eqs. (4)-(6) at pose T and its Jacobian row J.
__device__ inline double range_residual(const FrameDev &f, const double T[12], double J[6])
{
    const double qt[3] = {f.q[0] - T[9], f.q[1] - T[10], f.q[2] - T[11]};
    double P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = T[i] * qt[0] + T[3 + i] * qt[1] + T[6 + i] * qt[2];   // R^T qt
    double h, hx, hy;
    dsm_lookup(f, P[0], P[1], h, hx, hy);
    // dr/dP = a = (-hx, -hy, 1); J = [-R a, (R a) x q]
    double Ra[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Ra[i] = -T[3 * i] * hx - T[3 * i + 1] * hy + T[3 * i + 2];
    J[0] = -Ra[0];
    J[1] = -Ra[1];
    J[2] = -Ra[2];
    J[3] = Ra[1] * f.q[2] - Ra[2] * f.q[1];
    J[4] = Ra[2] * f.q[0] - Ra[0] * f.q[2];
    J[5] = Ra[0] * f.q[1] - Ra[1] * f.q[0];
    return P[2] - h;
}

// Prior residuals at one pose with their robust losses, before any scale:
// gravity (Eq. (3)) and laser range (Eqs. (4)-(6)).  They depend on the pose
// alone, so the epilogue can evaluate them while the photometric sums of the
// same pose are still being reduced.
struct PriorTerms {
    double gc[3], rg[3], sg, rho_g, drho_g;   // gravity: R g_world, residual, |r|^2, loss
    double J[6], rr, rho_r, drho_r;           // range: Jacobian row, residual, loss
};

__device__ inline void prior_terms(const FrameDev &f, const double T[12], PriorTerms &p)
{
    if (f.use_g) {
        gravity_residual(f, T, p.gc, p.rg);
        p.sg = p.rg[0] * p.rg[0] + p.rg[1] * p.rg[1] + p.rg[2] * p.rg[2];
        robust_f64(f.grav_kind, f.grav_b, p.sg, p.rho_g, p.drho_g);
    }
    if (f.use_r) {
        p.rr = range_residual(f, T, p.J);
        robust_f64(f.range_kind, f.range_b, p.rr * p.rr, p.rho_r, p.drho_r);
    }
}

// Add the gravity and range terms with scales ag, ar (the lambda of Eq. (7),
// the alpha of the supplement's H_total, g_total).
__device__ inline void add_priors(const FrameDev &f, const PriorTerms &p, double ag, double ar, double H[21],
                                  double g[6], double &cost)
{
    if (f.use_g) {
        cost += ag * p.rho_g;
        const double W = ag * p.drho_g;
        const double *gc = p.gc, *r = p.rg;
        // J^T J = |gc|^2 I - gc gc^T,  J^T r = gc x r  (rotation block)
        const double n2 = gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) H[tri(3 + a, 3 + b)] += W * ((a == b ? n2 : 0.0) - gc[a] * gc[b]);
        g[3] += W * (gc[1] * r[2] - gc[2] * r[1]);
        g[4] += W * (gc[2] * r[0] - gc[0] * r[2]);
        g[5] += W * (gc[0] * r[1] - gc[1] * r[0]);
    }
    if (f.use_r) {
        cost += ar * p.rho_r;
        const double W = ar * p.drho_r;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
#pragma unroll
            for (int b = a; b < 6; ++b) H[tri(a, b)] += W * p.J[a] * p.J[b];
            g[a] += W * p.J[a] * p.rr;
        }
    }
}

__device__ inline void add_priors(const FrameDev &f, const double T[12], double ag, double ar, double H[21],
                                  double g[6], double &cost)
{
    PriorTerms p{};
    prior_terms(f, T, p);
    add_priors(f, p, ag, ar, H, g, cost);
}

// Prior scales from the prior terms at the level's starting pose and the
// visual gradient gv there (supplement, Sensor-Prior Fusion in LM): each
// enabled prior's base scale is reduced so that its gradient does not exceed
// alpha_ratio times the visual one, and by (gate / |r|)^2 when its residual
// exceeds the gate.  Fixed scales unless f.adaptive; 0 for a disabled prior.
__device__ inline void prior_scales(const FrameDev &f, const PriorTerms &p, const double gv[6], double alpha[2])
{
    alpha[0] = f.use_g ? f.lam_imu : 0.0;
    alpha[1] = f.use_r ? f.lam_range : 0.0;
    if (!f.adaptive) return;
    double nv = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) nv += gv[a] * gv[a];
    nv = sqrt(nv);
    if (f.use_g) {
        const double *gc = p.gc, *r = p.rg;
        // unit-scale gradient drho * J^T r = drho * (0, gc x r)
        const double c0 = gc[1] * r[2] - gc[2] * r[1], c1 = gc[2] * r[0] - gc[0] * r[2],
                     c2 = gc[0] * r[1] - gc[1] * r[0];
        const double gn = fabs(p.drho_g) * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        const double rn = sqrt(p.sg);
        if (f.alpha_ratio > 0.0 && f.lam_imu * gn > f.alpha_ratio * nv) alpha[0] *= f.alpha_ratio * nv / (f.lam_imu * gn);
        if (f.grav_gate > 0.0 && rn > f.grav_gate) alpha[0] *= (f.grav_gate / rn) * (f.grav_gate / rn);
    }
    if (f.use_r) {
        double n2 = 0.0;
#pragma unroll
        for (int a = 0; a < 6; ++a) n2 += p.J[a] * p.J[a];
        const double gn = fabs(p.drho_r * p.rr) * sqrt(n2);
        const double rn = fabs(p.rr);
        if (f.alpha_ratio > 0.0 && f.lam_range * gn > f.alpha_ratio * nv)
            alpha[1] *= f.alpha_ratio * nv / (f.lam_range * gn);
        if (f.range_gate > 0.0 && rn > f.range_gate) alpha[1] *= (f.range_gate / rn) * (f.range_gate / rn);
    }
}

__device__ inline void store_pose(PoseEval &p, const double T[12])
{
#pragma unroll
    for (int i = 0; i < 12; ++i) p.v[i] = T[i];
}

// Finish the hypothesis' current level with status `st`: move to the next
// level's start (re-evaluated at the accepted pose) or finish.
__device__ inline void level_done(const FrameDev &f, HypState &s, int st, PoseEval &p32, int &hlev)
{
    s.status = st;
    if (f.keep_top > 0 && s.level == f.prune_level && s.level + 1 < f.n_levels) {
        hlev = HLEV_WAIT;                          // the pruning kernel decides who continues
    } else if (s.level + 1 < f.n_levels) {
        s.level += 1;
        s.phase = PHASE_START;
        store_pose(p32, s.T);
        hlev = s.level;
    } else {
        hlev = -1;
    }
}

// Solve for the next candidate (consuming iterations on failed
// factorisations) or end the level when iterations or damping run out.
__device__ inline void propose(const FrameDev &f, HypState &s, PoseEval &p32, int &hlev)
{
    const int iters = f.lv[s.level].iters;
    for (;;) {
        if (s.it_level >= iters) {
            level_done(f, s, ST_MAX_ITERS, p32, hlev);
            return;
        }
        s.it_level += 1;
        s.it_total += 1;
        double dx[6];
        if (!damped_solve(s.H, s.g, s.lam, dx)) {
            s.lam *= f.up;
            if (s.lam >= s.lmax) {
                level_done(f, s, ST_STALLED, p32, hlev);
                return;
            }
            continue;
        }
        double E[12];
        se3_exp(dx, E);
        se3_mul(E, s.T, s.Tc);
#pragma unroll
        for (int i = 0; i < 6; ++i) s.dxi[i] = dx[i];
        s.phase = PHASE_CAND;
        store_pose(p32, s.Tc);
        hlev = s.level;
        return;
    }
}

// Consume one evaluation (photo sums S: H21, g6, count, cost; prior terms P)
// of the hypothesis at its pending pose (T at a level start, else Tc) and
// advance its LM state.
__device__ inline void lm_advance(const FrameDev &f, HypState &s, const double *S, const PriorTerms &P, PoseEval &p32,
                                  int &hlev)
{
    double H[21], g[6];
#pragma unroll
    for (int i = 0; i < 21; ++i) H[i] = S[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) g[i] = S[21 + i];
    double cost = S[kCostSlot];
    const int n = (int)S[27];
    // the prior scales are set at the level's starting pose and held for the
    // level, so its objective is fixed and a cost decrease is well defined
    if (s.phase == PHASE_START) prior_scales(f, P, g, s.alpha);
    add_priors(f, P, s.alpha[0], s.alpha[1], H, g, cost);

    bool finite = isfinite(cost);
#pragma unroll
    for (int i = 0; i < 21; ++i) finite = finite && isfinite(H[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) finite = finite && isfinite(g[i]);

    if (s.phase == PHASE_START) {
        double D = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) D = fmax(D, H[tri(i, i)]);
        s.cost = cost;
        s.nvalid = n;
        if (n < f.min_valid || !finite || !(D > 0.0)) {
            s.status = ST_DEGENERATE;
            hlev = -1;
            return;
        }
#pragma unroll
        for (int i = 0; i < 21; ++i) s.H[i] = H[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) s.g[i] = g[i];
        s.lam = f.tau * D;
        s.lmin = f.lmin_rel * D;
        s.lmax = f.lmax_rel * D;
        s.it_level = 0;
        propose(f, s, p32, hlev);
        return;
    }
    // candidate evaluation; a cost flat to within cost_tol ends the level
    const bool flat = finite && f.cost_tol > 0.0 && fabs(cost - s.cost) <= f.cost_tol * s.cost;
    if (finite && cost < s.cost) {
#pragma unroll
        for (int i = 0; i < 12; ++i) s.T[i] = s.Tc[i];
#pragma unroll
        for (int i = 0; i < 21; ++i) s.H[i] = H[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) s.g[i] = g[i];
        s.cost = cost;
        s.nvalid = n;
        s.lam = fmax(s.lam / f.down, s.lmin);
        const double nt = sqrt(s.dxi[0] * s.dxi[0] + s.dxi[1] * s.dxi[1] + s.dxi[2] * s.dxi[2]);
        const double nr = sqrt(s.dxi[3] * s.dxi[3] + s.dxi[4] * s.dxi[4] + s.dxi[5] * s.dxi[5]);
        if ((nt < f.tol_t && nr < f.tol_r) || flat) {
            level_done(f, s, ST_CONVERGED, p32, hlev);
            return;
        }
    } else if (flat) {
        level_done(f, s, ST_CONVERGED, p32, hlev);
        return;
    } else {
        s.lam *= f.up;
        if (s.lam >= s.lmax) {
            level_done(f, s, ST_STALLED, p32, hlev);
            return;
        }
    }
    propose(f, s, p32, hlev);
}

}  // namespace pilot
