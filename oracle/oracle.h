/*
 * oracle.h -- plain FP64 CPU reference of the sensor-prior featuremetric
 * Levenberg-Marquardt pose solver (PiLoT v2, arXiv 2606.31098).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path never
 * does.  It shares no code, header or constant with the GPU library.
 *
 * Conventions (each reading of the paper is listed in the design notes):
 *   pose      world->camera, double[12] = R row-major (9), t (3);
 *             X_cam = R X + t.
 *   update    T <- Exp(xi) * T with xi = (rho; omega), translation first.
 *   pixels    integer coordinates are pixel centres; a point is visible iff
 *             Z > z_min and 0 <= u <= W-1 and 0 <= v <= H-1.
 *   features  channels-last H x W x C; reference descriptors N x C.
 *   DSM       Hd x Wd heights; sample (i, j) sits at (x0 + j*gsd, y0 + i*gsd);
 *             bilinear with clamp-to-edge.
 */
#ifndef PILOT_ORACLE_H
#define PILOT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_CAUCHY = 0, ORC_HUBER = 1, ORC_L2 = 2 };
enum { ORC_CONVERGED = 0, ORC_MAX_ITERS = 1, ORC_STALLED = 2, ORC_DEGENERATE = 3, ORC_PRUNED = 4 };

typedef struct {
    int H, W, C;
    const double *feat;      /* H*W*C */
    const double *qconf;     /* H*W or NULL (query confidence, treated as constant in J) */
    double fx, fy, cx, cy;
    int N;
    const double *P;         /* N*3 world points */
    const double *ref;       /* N*C reference descriptors */
    const double *ref_w;     /* N or NULL */
    int iters;
    int loss_kind;
    double loss_scale;
} orc_level;

typedef struct {
    int n_levels;
    orc_level lv[4];
    int use_gravity;
    double g_imu[3], g_world[3], lambda_imu;
    int grav_loss_kind;
    double grav_loss_scale;
    int use_range;
    double d_range, pc[2], lambda_range;
    int range_loss_kind;
    double range_loss_scale;
    const double *dsm;
    int Hd, Wd;
    double dsm_x0, dsm_y0, dsm_gsd;
    double tau, up, down, lam_min_rel, lam_max_rel, tol_t, tol_r, z_min;
    int min_valid;
    /* top-K pruning (supplement, Multi-Hypothesis Refinement): after level
     * prune_level every hypothesis has finished that level; only the keep_top
     * lowest costs continue (0 = no pruning) */
    int keep_top, prune_level;
    /* adaptive prior scales (supplement, Sensor-Prior Fusion in LM): when
     * adaptive != 0 the scales of the gravity and range terms are set at the
     * start of every level from the relative gradient magnitudes (cap ratio
     * alpha_ratio) and residual gates (grav_gate, range_gate), then held for
     * that level; see orc_prior_scales */
    int adaptive;
    double alpha_ratio, grav_gate, range_gate;
    /* function tolerance: a candidate whose cost differs from the current
     * one by at most cost_tol * cost ends the level as CONVERGED (accepted
     * if lower); 0 switches the rule off */
    double cost_tol;
} orc_frame;

/* SE(3) */
void orc_exp(const double xi[6], double T[12]);
void orc_log(const double T[12], double xi[6]);
void orc_compose(const double A[12], const double B[12], double AB[12]);

/* robust loss rho(s) and its derivative rho'(s) */
void orc_robust(int kind, double b, double s, double *rho, double *drho);

/* bilinear value and derivatives d/du, d/dv of a channels-last map (C values
 * each); requires 0 <= u <= W-1, 0 <= v <= H-1, H, W >= 2 */
void orc_bilinear(const double *F, int H, int W, int C, double u, double v,
                  double *val, double *du, double *dv);

/* DSM height and gradient (per metre) at world (x, y) */
void orc_dsm(const orc_frame *f, double x, double y, double *h, double *hx, double *hy);

/* Photo residual of anchor j at level l: r (C), dense Jacobian J (C*6,
 * row-major), weight w.  Returns 1 if visible, 0 otherwise (r, J untouched). */
int orc_photo_point(const orc_frame *f, int l, const double T[12], int j,
                    double *r, double *J, double *w);

/* gravity residual r (3) and Jacobian J (3*6) */
void orc_gravity(const orc_frame *f, const double T[12], double r[3], double J[18]);

/* laser-range residual and Jacobian (1*6) */
void orc_range(const orc_frame *f, const double T[12], double *r, double J[6]);

/* total objective at level l and its Gauss-Newton system with the fixed
 * prior scales lambda_imu, lambda_range:
 * H (6*6), g (6) = J^T W r, cost, number of visible anchors */
void orc_linearize(const orc_frame *f, int l, const double T[12],
                   double H[36], double g[6], double *cost, int *nvalid);

/* the visual term alone (photo residuals and out-of-view penalties) */
void orc_linearize_visual(const orc_frame *f, int l, const double T[12],
                          double H[36], double g[6], double *cost, int *nvalid);

/* add the gravity and range terms (those enabled) with scales a_grav,
 * a_range to H, g, cost */
void orc_add_priors(const orc_frame *f, const double T[12], double a_grav, double a_range,
                    double H[36], double g[6], double *cost);

/* Adaptive prior scales at pose T given the visual gradient g_vis:
 * for each enabled prior s with base scale lambda_s, unit-scale gradient
 * g_s = J_s^T rho_s' r_s and residual norm |r_s|,
 *   alpha_s = lambda_s * min(1, alpha_ratio |g_vis| / (lambda_s |g_s|))
 *                      * min(1, (gate_s / |r_s|)^2),
 * where a factor is 1 when its parameter is <= 0 (or |g_s| = 0).  A
 * disabled prior gets 0.  With adaptive == 0: alpha = (lambda_imu,
 * lambda_range) of the enabled priors. */
void orc_prior_scales(const orc_frame *f, const double T[12], const double g_vis[6], double alpha[2]);

/* (A) x = b for a 6x6 SPD A by Cholesky; returns 0, or -1 if not PD */
int orc_cholesky_solve6(const double A[36], const double b[6], double x[6]);

/* LM over hypotheses [m0, m1) of poses_in (M*12).  Outputs are indexed by m.
 * With pruning, the ranking is over the hypotheses in [m0, m1).
 * trace (optional): per hypothesis `trace_stride` rows of 4 doubles
 * (level, cost before, candidate cost or NaN, accepted 0/1), one row per
 * iteration; unused rows are NaN. */
void orc_solve(const orc_frame *f, const double *poses_in, int m0, int m1,
               double *poses_out, double *cost, int *iterations, int *status,
               double *trace, int trace_stride);

/* the prior scales (gravity, range) each hypothesis used at the last level it
 * started, indexed by m, after orc_solve_alpha's run (alpha: M*2) */
void orc_solve_alpha(const orc_frame *f, const double *poses_in, int m0, int m1,
                     double *poses_out, double *cost, int *iterations, int *status,
                     double *trace, int trace_stride, double *alpha);

/* Geo-anchor lift (supplement, Geo-anchor Construction): anchor j at DSM-crop
 * sample coordinates (u_j, v_j) becomes P = (x0 + u gsd, y0 + v gsd, D(u, v))
 * (bilinear, clamp-to-edge), and its reference descriptor is the bilinear
 * sample (clamp-to-edge) of an Hr x Wr x C reference map at
 * (scale (u + 1/2) - 1/2, scale (v + 1/2) - 1/2): map pixels cover the crop
 * with `scale` map pixels per DSM sample, centres aligned. */
void orc_lift(const double *dsm, int Hd, int Wd, double x0, double y0, double gsd,
              const double *uv, int N, const double *ref_map, int Hr, int Wr, int C, double scale,
              double *P, double *ref);

/* lowest finite cost among non-degenerate hypotheses, ties -> lowest index,
 * -1 if none */
int orc_best(const double *cost, const int *status, int M);

void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
