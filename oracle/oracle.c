/*
 * oracle.c -- plain FP64 CPU reference of the sensor-prior featuremetric LM
 * pose solver of PiLoT v2 (arXiv 2606.31098).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  Shares no code
 * with the GPU library.  Written for a reader holding the paper: every
 * function names the passage it follows, and nothing is blocked, fused or
 * reordered beyond what that passage states (the only parallelism is an
 * OpenMP loop over independent hypotheses).
 *
 * Pins (tests/test_oracle_*.py): SE(3) against scipy's rotation-vector map
 * and exp/log round trips; bilinear exactness on affine fields; analytic
 * Jacobians against central finite differences; g = 1/2 grad(cost) by
 * finite differences; H against J^T W J with finite-difference J; Cholesky
 * against LAPACK; zero residuals at the ground truth of noise-free synthetic
 * frames (the synthetic scene has its own projection, bilinear sampler and
 * DSM ray march); LM convergence to the ground truth; accepted costs never
 * increase.  End-to-end values on noisy frames: parity unpinned by the paper
 * (it prints no worked example); they are pinned only through the above.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;

void orc_set_threads(int n) { g_threads = n; }

int orc_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* small 3x3 helpers                                                   */
/* ------------------------------------------------------------------ */
static void skew(const double w[3], double S[9])
{
    S[0] = 0.0;   S[1] = -w[2]; S[2] = w[1];
    S[3] = w[2];  S[4] = 0.0;   S[5] = -w[0];
    S[6] = -w[1]; S[7] = w[0];  S[8] = 0.0;
}

static void mat3_mul(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void mat3_vec(const double A[9], const double x[3], double y[3])
{
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

static void mat3T_vec(const double A[9], const double x[3], double y[3])
{
    for (int i = 0; i < 3; ++i) y[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
}

/* ------------------------------------------------------------------ */
/* SE(3) exponential, logarithm, composition                           */
/* The update of Eq. (9) (Method, Multi-Sensor Optimization) is        */
/* T <- exp(dxi) T.  exp is the full SE(3) exponential:                */
/* R = I + A W + B W^2, t = V rho, V = I + B W + C' W^2, W = [omega]x,  */
/* A = sin(th)/th, B = (1-cos th)/th^2, C' = (th - sin th)/th^3.       */
/* ------------------------------------------------------------------ */
void orc_exp(const double xi[6], double T[12])
{
    const double *rho = xi, *w = xi + 3;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B, Cp;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        Cp = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        Cp = (th - sin(th)) / (th2 * th);
    }
    double W[9], W2[9];
    skew(w, W);
    mat3_mul(W, W, W2);
    double V[9];
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        T[i] = I + A * W[i] + B * W2[i];
        V[i] = I + B * W[i] + Cp * W2[i];
    }
    mat3_vec(V, rho, T + 9);
}

void orc_log(const double T[12], double xi[6])
{
    const double *R = T;
    double v[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
    double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(s, c);
    double w[3];
    if (th < 1e-6) {
        for (int i = 0; i < 3; ++i) w[i] = v[i] * (1.0 + th * th / 6.0);
    } else if (M_PI - th < 1e-6 || s < 1e-9) {
        /* near pi: axis from the symmetric part (R + R^T)/2 - cos(th) I */
        double S[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                S[3 * i + j] = 0.5 * (R[3 * i + j] + R[3 * j + i]) - (i == j ? c : 0.0);
        int k = 0;
        for (int i = 1; i < 3; ++i)
            if (S[4 * i] > S[4 * k]) k = i;
        double n[3] = {S[3 * k], S[3 * k + 1], S[3 * k + 2]};
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double sg = (n[0] * v[0] + n[1] * v[1] + n[2] * v[2]) < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i) w[i] = sg * th * n[i] / nn;
    } else {
        for (int i = 0; i < 3; ++i) w[i] = th / s * v[i];
    }
    /* rho = V^{-1} t by solving V rho = t (Gaussian elimination, 3x3) */
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double B, Cp;
    if (th < 1e-4) {
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        Cp = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        B = (1.0 - cos(th)) / th2;
        Cp = (th - sin(th)) / (th2 * th);
    }
    double W[9], W2[9], V[12];
    skew(w, W);
    mat3_mul(W, W, W2);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            V[4 * i + j] = (i == j ? 1.0 : 0.0) + B * W[3 * i + j] + Cp * W2[3 * i + j];
        V[4 * i + 3] = T[9 + i];
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(V[4 * r + col]) > fabs(V[4 * piv + col])) piv = r;
        for (int k = 0; k < 4; ++k) {
            double tmp = V[4 * col + k];
            V[4 * col + k] = V[4 * piv + k];
            V[4 * piv + k] = tmp;
        }
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            double fct = V[4 * r + col] / V[4 * col + col];
            for (int k = 0; k < 4; ++k) V[4 * r + k] -= fct * V[4 * col + k];
        }
    }
    for (int i = 0; i < 3; ++i) xi[i] = V[4 * i + 3] / V[4 * i + i];
    for (int i = 0; i < 3; ++i) xi[3 + i] = w[i];
}

void orc_compose(const double A[12], const double B[12], double AB[12])
{
    mat3_mul(A, B, AB);
    double Rt[3];
    mat3_vec(A, B + 9, Rt);
    for (int i = 0; i < 3; ++i) AB[9 + i] = Rt[i] + A[9 + i];
}

/* ------------------------------------------------------------------ */
/* Robust loss (Eq. (2) uses Huber; Cauchy and plain L2 selectable).    */
/* Cauchy: rho = b ln(1 + s/b), rho' = 1/(1 + s/b).                     */
/* Huber:  rho = s (s <= b), 2 sqrt(b s) - b otherwise;                 */
/*         rho' = 1 (s <= b), sqrt(b/s) otherwise.                      */
/* ------------------------------------------------------------------ */
void orc_robust(int kind, double b, double s, double *rho, double *drho)
{
    if (kind == ORC_CAUCHY) {
        *rho = b * log1p(s / b);
        *drho = 1.0 / (1.0 + s / b);
    } else if (kind == ORC_HUBER) {
        if (s <= b) {
            *rho = s;
            *drho = 1.0;
        } else {
            double r = sqrt(b * s);
            *rho = 2.0 * r - b;
            *drho = b / r;
        }
    } else {
        *rho = s;
        *drho = 1.0;
    }
}

/* ------------------------------------------------------------------ */
/* Bilinear interpolation of a channels-last map and the exact          */
/* derivatives of the interpolant (descriptor interpolation and local   */
/* feature gradient, supplement "Optimizer implementation").           */
/* ------------------------------------------------------------------ */
void orc_bilinear(const double *F, int H, int W, int C, double u, double v,
                  double *val, double *du, double *dv)
{
    int x0 = (int)floor(u), y0 = (int)floor(v);
    if (x0 > W - 2) x0 = W - 2;
    if (y0 > H - 2) y0 = H - 2;
    double ax = u - x0, ay = v - y0;
    const double *f00 = F + ((size_t)y0 * W + x0) * C;
    const double *f10 = F + ((size_t)y0 * W + x0 + 1) * C;
    const double *f01 = F + ((size_t)(y0 + 1) * W + x0) * C;
    const double *f11 = F + ((size_t)(y0 + 1) * W + x0 + 1) * C;
    for (int c = 0; c < C; ++c) {
        val[c] = (1.0 - ax) * (1.0 - ay) * f00[c] + ax * (1.0 - ay) * f10[c]
               + (1.0 - ax) * ay * f01[c] + ax * ay * f11[c];
        du[c] = (1.0 - ay) * (f10[c] - f00[c]) + ay * (f11[c] - f01[c]);
        dv[c] = (1.0 - ax) * (f01[c] - f00[c]) + ax * (f11[c] - f10[c]);
    }
}

/* DSM lookup D(x, y) of Eq. (6), bilinear with clamp-to-edge. */
void orc_dsm(const orc_frame *f, double x, double y, double *h, double *hx, double *hy)
{
    double fj = (x - f->dsm_x0) / f->dsm_gsd;
    double fi = (y - f->dsm_y0) / f->dsm_gsd;
    int cj = 0, ci = 0;
    if (!(fj >= 0.0)) { fj = 0.0; cj = 1; }          /* also NaN */
    if (fj > f->Wd - 1.0) { fj = f->Wd - 1.0; cj = 1; }
    if (!(fi >= 0.0)) { fi = 0.0; ci = 1; }
    if (fi > f->Hd - 1.0) { fi = f->Hd - 1.0; ci = 1; }
    int j0 = (int)floor(fj), i0 = (int)floor(fi);
    if (j0 > f->Wd - 2) j0 = f->Wd - 2;
    if (i0 > f->Hd - 2) i0 = f->Hd - 2;
    double a = fj - j0, b = fi - i0;
    const double *D = f->dsm;
    double d00 = D[(size_t)i0 * f->Wd + j0], d01 = D[(size_t)i0 * f->Wd + j0 + 1];
    double d10 = D[(size_t)(i0 + 1) * f->Wd + j0], d11 = D[(size_t)(i0 + 1) * f->Wd + j0 + 1];
    *h = (1 - a) * (1 - b) * d00 + a * (1 - b) * d01 + (1 - a) * b * d10 + a * b * d11;
    *hx = cj ? 0.0 : ((1 - b) * (d01 - d00) + b * (d11 - d10)) / f->dsm_gsd;
    *hy = ci ? 0.0 : ((1 - a) * (d10 - d00) + a * (d11 - d01)) / f->dsm_gsd;
}

/* ------------------------------------------------------------------ */
/* Photo residual, Eq. (1): r = f_q(pi(K_l, T, P_j)) - f_r(p_j), with   */
/* the dense C x 6 Jacobian J = dF/d(u,v) * dpi/dX * dX/dxi,            */
/* dX/dxi = [I | -[X]x] for the left perturbation T <- Exp(xi) T.        */
/* ------------------------------------------------------------------ */
int orc_photo_point(const orc_frame *f, int l, const double T[12], int j,
                    double *r, double *J, double *w)
{
    const orc_level *L = &f->lv[l];
    const double *P = L->P + 3 * (size_t)j;
    double X[3];
    mat3_vec(T, P, X);
    for (int i = 0; i < 3; ++i) X[i] += T[9 + i];
    if (!(X[2] > f->z_min)) return 0;
    double u = L->fx * X[0] / X[2] + L->cx;
    double v = L->fy * X[1] / X[2] + L->cy;
    if (!(u >= 0.0 && u <= L->W - 1.0 && v >= 0.0 && v <= L->H - 1.0)) return 0;

    int C = L->C;
    double Fv[512], Fu[512], Fw[512];
    orc_bilinear(L->feat, L->H, L->W, C, u, v, Fv, Fu, Fw);
    for (int c = 0; c < C; ++c) r[c] = Fv[c] - L->ref[(size_t)j * C + c];

    double dpi[6] = {L->fx / X[2], 0.0, -L->fx * X[0] / (X[2] * X[2]),
                     0.0, L->fy / X[2], -L->fy * X[1] / (X[2] * X[2])};
    double S[9];
    skew(X, S);
    double dX[18]; /* 3 x 6 : [I | -S] */
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 6; ++k)
            dX[6 * a + k] = (k < 3) ? (a == k ? 1.0 : 0.0) : -S[3 * a + (k - 3)];
    double Jp[12]; /* 2 x 6 */
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 6; ++k) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += dpi[3 * a + m] * dX[6 * m + k];
            Jp[6 * a + k] = s;
        }
    for (int c = 0; c < C; ++c)
        for (int k = 0; k < 6; ++k) J[6 * c + k] = Fu[c] * Jp[k] + Fw[c] * Jp[6 + k];

    double wq = 1.0;
    if (L->qconf) {
        double q, qu, qv;
        orc_bilinear(L->qconf, L->H, L->W, 1, u, v, &q, &qu, &qv);
        wq = q;
    }
    *w = (L->ref_w ? L->ref_w[j] : 1.0) * wq;
    return 1;
}

/* Gravity residual, Eq. (3): the hypothesis' rotation maps the world      */
/* gravity direction into the camera, r = R g_W - g_imu (our R is world->   */
/* camera, the transpose of the paper's camera->world rotation).  Under     */
/* T <- Exp(xi) T, R g_W -> g_c + omega x g_c, so J = [0 | -[g_c]x].        */
void orc_gravity(const orc_frame *f, const double T[12], double r[3], double J[18])
{
    double gc[3];
    mat3_vec(T, f->g_world, gc);
    for (int i = 0; i < 3; ++i) r[i] = gc[i] - f->g_imu[i];
    double S[9];
    skew(gc, S);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 6; ++k) J[6 * a + k] = (k < 3) ? 0.0 : -S[3 * a + (k - 3)];
}

/* Laser range residual, Eqs. (4)-(6): unit ray of the range pixel through   */
/* the finest level's intrinsics, range point P = C + R_wc (d v) expressed   */
/* as P = R^T (d v - t), residual r = P_z - D(P_x, P_y).  Under              */
/* T <- Exp(xi) T: dP/drho = -R^T, dP/domega = R^T [q]x with q = d v.       */
void orc_range(const orc_frame *f, const double T[12], double *r, double J[6])
{
    const orc_level *L = &f->lv[f->n_levels - 1];
    double ray[3] = {(f->pc[0] - L->cx) / L->fx, (f->pc[1] - L->cy) / L->fy, 1.0};
    double n = sqrt(ray[0] * ray[0] + ray[1] * ray[1] + ray[2] * ray[2]);
    double q[3], qt[3], P[3];
    for (int i = 0; i < 3; ++i) {
        q[i] = f->d_range * ray[i] / n;
        qt[i] = q[i] - T[9 + i];
    }
    mat3T_vec(T, qt, P);
    double h, hx, hy;
    orc_dsm(f, P[0], P[1], &h, &hx, &hy);
    *r = P[2] - h;
    double dr[3] = {-hx, -hy, 1.0};
    double Q[9], RtQ[9];
    skew(q, Q);
    /* R^T [q]x */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += T[3 * m + a] * Q[3 * m + b];
            RtQ[3 * a + b] = s;
        }
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += dr[a] * ((k < 3) ? -T[3 * k + a] : RtQ[3 * a + (k - 3)]);
        J[k] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Total objective of Eq. (7) at level l and its damped-normal-equation   */
/* terms of Eq. (8): H = J^T W J, g = J^T W r, accumulated per term as in  */
/* the supplement ("Sensor-Prior Fusion in LM") with fixed prior scales.    */
/* W holds the IRLS weight rho'(s) times the confidence w, s = w |r|^2      */
/* (Eq. (2)).  Anchors outside the view add the constant rho(2 w_ref).      */
/* ------------------------------------------------------------------ */
void orc_linearize_visual(const orc_frame *f, int l, const double T[12],
                          double H[36], double g[6], double *cost, int *nvalid)
{
    const orc_level *L = &f->lv[l];
    int C = L->C;
    double r[512], J[512 * 6];
    memset(H, 0, 36 * sizeof(double));
    memset(g, 0, 6 * sizeof(double));
    double c = 0.0;
    int n = 0;
    for (int j = 0; j < L->N; ++j) {
        double w;
        double rho, drho;
        if (!orc_photo_point(f, l, T, j, r, J, &w)) {
            double wr = L->ref_w ? L->ref_w[j] : 1.0;
            orc_robust(L->loss_kind, L->loss_scale, 2.0 * wr, &rho, &drho);
            c += rho;
            continue;
        }
        n++;
        double s = 0.0;
        for (int k = 0; k < C; ++k) s += r[k] * r[k];
        s *= w;
        orc_robust(L->loss_kind, L->loss_scale, s, &rho, &drho);
        c += rho;
        double W = drho * w;
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) {
                double sum = 0.0;
                for (int k = 0; k < C; ++k) sum += J[6 * k + a] * J[6 * k + b];
                H[6 * a + b] += W * sum;
            }
            double sg = 0.0;
            for (int k = 0; k < C; ++k) sg += J[6 * k + a] * r[k];
            g[a] += W * sg;
        }
    }
    *cost = c;
    *nvalid = n;
}

/* Gravity and range terms of Eq. (7) with scales a_grav, a_range (the
 * lambda_imu, lambda_range of Eq. (7); the alpha of the supplement's
 * H_total, g_total). */
void orc_add_priors(const orc_frame *f, const double T[12], double a_grav, double a_range,
                    double H[36], double g[6], double *cost)
{
    double c = *cost;
    if (f->use_gravity) {
        double rg[3], Jg[18], rho, drho;
        orc_gravity(f, T, rg, Jg);
        double s = rg[0] * rg[0] + rg[1] * rg[1] + rg[2] * rg[2];
        orc_robust(f->grav_loss_kind, f->grav_loss_scale, s, &rho, &drho);
        c += a_grav * rho;
        double W = a_grav * drho;
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) {
                double sum = 0.0;
                for (int k = 0; k < 3; ++k) sum += Jg[6 * k + a] * Jg[6 * k + b];
                H[6 * a + b] += W * sum;
            }
            double sg = 0.0;
            for (int k = 0; k < 3; ++k) sg += Jg[6 * k + a] * rg[k];
            g[a] += W * sg;
        }
    }
    if (f->use_range) {
        double rr, Jr[6], rho, drho;
        orc_range(f, T, &rr, Jr);
        orc_robust(f->range_loss_kind, f->range_loss_scale, rr * rr, &rho, &drho);
        c += a_range * rho;
        double W = a_range * drho;
        for (int a = 0; a < 6; ++a) {
            for (int b = 0; b < 6; ++b) H[6 * a + b] += W * Jr[a] * Jr[b];
            g[a] += W * Jr[a] * rr;
        }
    }
    *cost = c;
}

void orc_linearize(const orc_frame *f, int l, const double T[12],
                   double H[36], double g[6], double *cost, int *nvalid)
{
    orc_linearize_visual(f, l, T, H, g, cost, nvalid);
    orc_add_priors(f, T, f->lambda_imu, f->lambda_range, H, g, cost);
}

/* One prior's unit-scale gradient norm and residual norm. */
static void prior_unit(const orc_frame *f, const double T[12], int which, double *gnorm, double *rnorm)
{
    double gs[6] = {0, 0, 0, 0, 0, 0};
    if (which == 0) {
        double r[3], J[18], rho, drho;
        orc_gravity(f, T, r, J);
        const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        orc_robust(f->grav_loss_kind, f->grav_loss_scale, s, &rho, &drho);
        for (int a = 0; a < 6; ++a)
            for (int k = 0; k < 3; ++k) gs[a] += J[6 * k + a] * drho * r[k];
        *rnorm = sqrt(s);
    } else {
        double r, J[6], rho, drho;
        orc_range(f, T, &r, J);
        orc_robust(f->range_loss_kind, f->range_loss_scale, r * r, &rho, &drho);
        for (int a = 0; a < 6; ++a) gs[a] = J[a] * drho * r;
        *rnorm = fabs(r);
    }
    double n2 = 0.0;
    for (int a = 0; a < 6; ++a) n2 += gs[a] * gs[a];
    *gnorm = sqrt(n2);
}

/* Adaptive prior scales (supplement, Sensor-Prior Fusion in LM): a prior's
 * scale shrinks when its gradient would dominate the visual one (relative
 * gradient magnitudes) and when its residual is implausibly large (the
 * residual-dependent gate). */
void orc_prior_scales(const orc_frame *f, const double T[12], const double g_vis[6], double alpha[2])
{
    const int use[2] = {f->use_gravity, f->use_range};
    const double lam[2] = {f->lambda_imu, f->lambda_range};
    const double gate[2] = {f->grav_gate, f->range_gate};
    double gv = 0.0;
    for (int a = 0; a < 6; ++a) gv += g_vis[a] * g_vis[a];
    gv = sqrt(gv);
    for (int s = 0; s < 2; ++s) {
        if (!use[s]) {
            alpha[s] = 0.0;
            continue;
        }
        alpha[s] = lam[s];
        if (!f->adaptive) continue;
        double gn, rn;
        prior_unit(f, T, s, &gn, &rn);
        if (f->alpha_ratio > 0.0 && lam[s] * gn > f->alpha_ratio * gv)
            alpha[s] *= f->alpha_ratio * gv / (lam[s] * gn);
        if (gate[s] > 0.0 && rn > gate[s]) alpha[s] *= (gate[s] / rn) * (gate[s] / rn);
    }
}

/* Damped 6x6 solve of Eq. (8) by Cholesky factorisation A = L L^T. */
int orc_cholesky_solve6(const double A[36], const double b[6], double x[6])
{
    double L[36];
    memset(L, 0, sizeof(L));
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return -1;
                L[6 * i + i] = sqrt(s);
            } else {
                L[6 * i + j] = s / L[6 * j + j];
            }
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
        x[i] = s / L[6 * i + i];
    }
    return 0;
}

static int all_finite(const double *a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Multi-hypothesis coarse-to-fine LM (Method, Multi-Sensor             */
/* Optimization; supplement, Multi-Hypothesis Refinement).  Every        */
/* hypothesis is refined independently: at each level the objective is   */
/* linearised at the current pose, the damped system of Eq. (8) is solved, */
/* the candidate Exp(dxi) T of Eq. (9) is re-evaluated on the total        */
/* objective and accepted iff its cost is lower.                           */
/* ------------------------------------------------------------------ */
typedef struct {
    double T[12];
    double c;
    double alpha[2];
    int status, total_it, row, finished;
} hyp_state;

/* objective at level l with the level's frozen prior scales */
static void linearize_at(const orc_frame *f, int l, const double T[12], const double alpha[2],
                         double H[36], double g[6], double *cost, int *nvalid)
{
    orc_linearize_visual(f, l, T, H, g, cost, nvalid);
    orc_add_priors(f, T, alpha[0], alpha[1], H, g, cost);
}

/* One level of LM for one hypothesis. */
static void run_level(const orc_frame *f, int l, hyp_state *st, double *trace, int trace_stride)
{
    double H[36], g[6], c;
    int n;
    /* the scales are chosen once at the level's starting pose and held for
     * the level, so the level's objective is fixed and a decrease of the cost
     * is well defined */
    orc_linearize_visual(f, l, st->T, H, g, &c, &n);
    orc_prior_scales(f, st->T, g, st->alpha);
    orc_add_priors(f, st->T, st->alpha[0], st->alpha[1], H, g, &c);
    st->c = c;
    double D = 0.0;
    for (int i = 0; i < 6; ++i)
        if (H[7 * i] > D) D = H[7 * i];
    if (n < f->min_valid || !isfinite(c) || !all_finite(H, 36) || !all_finite(g, 6) || !(D > 0.0)) {
        st->status = ORC_DEGENERATE;
        st->finished = 1;
        return;
    }
    double lam = f->tau * D, lam_min = f->lam_min_rel * D, lam_max = f->lam_max_rel * D;
    int lvl_status = ORC_MAX_ITERS;
    for (int it = 0; it < f->lv[l].iters; ++it) {
        st->total_it++;
        double A[36], mg[6], dx[6];
        memcpy(A, H, sizeof(A));
        for (int i = 0; i < 6; ++i) {
            A[7 * i] += lam;
            mg[i] = -g[i];
        }
        double *tr = (trace && st->row < trace_stride) ? trace + 4 * st->row : NULL;
        st->row++;
        if (orc_cholesky_solve6(A, mg, dx) != 0) {
            if (tr) { tr[0] = l; tr[1] = c; tr[2] = NAN; tr[3] = 0; }
            lam *= f->up;
            if (lam >= lam_max) { lvl_status = ORC_STALLED; break; }
            continue;
        }
        double E[12], Tc[12], Hc[36], gc[6], cc;
        int nc;
        orc_exp(dx, E);
        orc_compose(E, st->T, Tc);
        linearize_at(f, l, Tc, st->alpha, Hc, gc, &cc, &nc);
        if (tr) { tr[0] = l; tr[1] = c; tr[2] = cc; tr[3] = 0; }
        /* the cost is flat to within cost_tol: nothing left to gain */
        const int flat = f->cost_tol > 0.0 && fabs(cc - c) <= f->cost_tol * c;
        if (cc < c) {
            if (tr) tr[3] = 1;
            memcpy(st->T, Tc, sizeof(Tc));
            memcpy(H, Hc, sizeof(H));
            memcpy(g, gc, sizeof(g));
            c = cc;
            st->c = c;
            lam = lam / f->down;
            if (lam < lam_min) lam = lam_min;
            double nt = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
            double nr = sqrt(dx[3] * dx[3] + dx[4] * dx[4] + dx[5] * dx[5]);
            if ((nt < f->tol_t && nr < f->tol_r) || flat) { lvl_status = ORC_CONVERGED; break; }
        } else if (flat) {
            lvl_status = ORC_CONVERGED;
            break;
        } else {
            lam *= f->up;
            if (lam >= lam_max) { lvl_status = ORC_STALLED; break; }
        }
    }
    st->status = lvl_status;
}

void orc_solve(const orc_frame *f, const double *poses_in, int m0, int m1,
               double *poses_out, double *cost, int *iterations, int *status,
               double *trace, int trace_stride)
{
    orc_solve_alpha(f, poses_in, m0, m1, poses_out, cost, iterations, status, trace, trace_stride, NULL);
}

void orc_solve_alpha(const orc_frame *f, const double *poses_in, int m0, int m1,
                     double *poses_out, double *cost, int *iterations, int *status,
                     double *trace, int trace_stride, double *alpha)
{
    const int k = m1 - m0;
    if (trace)
        for (long i = 0; i < (long)k * trace_stride * 4; ++i) trace[i] = NAN;
    hyp_state *st = (hyp_state *)calloc((size_t)(k > 0 ? k : 1), sizeof(hyp_state));
    for (int i = 0; i < k; ++i) {
        memcpy(st[i].T, poses_in + 12 * (size_t)(m0 + i), sizeof(st[i].T));
        st[i].c = NAN;
        st[i].status = ORC_MAX_ITERS;
    }
    const int prune = f->keep_top > 0 && f->prune_level >= 0 && f->prune_level < f->n_levels - 1;
    const int split = prune ? f->prune_level + 1 : f->n_levels;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(orc_get_threads())
#endif
    for (int i = 0; i < k; ++i)
        for (int l = 0; l < split && !st[i].finished; ++l)
            run_level(f, l, &st[i], trace ? trace + (size_t)i * trace_stride * 4 : NULL, trace_stride);
    if (prune) {
        /* rank by the cost after the pruning level: lower cost first, ties
         * to the lower index; degenerate hypotheses are not ranked */
        for (int i = 0; i < k; ++i) {
            if (st[i].finished) continue;
            int better = 0;
            for (int j = 0; j < k; ++j) {
                if (j == i || st[j].finished) continue;
                if (st[j].c < st[i].c || (st[j].c == st[i].c && j < i)) better++;
            }
            if (better >= f->keep_top) st[i].status = ORC_PRUNED;
        }
        for (int i = 0; i < k; ++i)
            if (st[i].status == ORC_PRUNED) st[i].finished = 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(orc_get_threads())
#endif
        for (int i = 0; i < k; ++i)
            for (int l = split; l < f->n_levels && !st[i].finished; ++l)
                run_level(f, l, &st[i], trace ? trace + (size_t)i * trace_stride * 4 : NULL, trace_stride);
    }
    for (int i = 0; i < k; ++i) {
        memcpy(poses_out + 12 * (size_t)(m0 + i), st[i].T, sizeof(st[i].T));
        cost[m0 + i] = st[i].c;
        iterations[m0 + i] = st[i].total_it;
        status[m0 + i] = st[i].status;
        if (alpha) {
            alpha[2 * (m0 + i)] = st[i].alpha[0];
            alpha[2 * (m0 + i) + 1] = st[i].alpha[1];
        }
    }
    free(st);
}

/* Bilinear sample with clamp-to-edge of a channels-last map at (u, v). */
static void sample_clamped(const double *F, int H, int W, int C, double u, double v, double *out)
{
    if (!(u >= 0.0)) u = 0.0;
    if (u > W - 1.0) u = W - 1.0;
    if (!(v >= 0.0)) v = 0.0;
    if (v > H - 1.0) v = H - 1.0;
    double du[512], dv[512];
    orc_bilinear(F, H, W, C, u, v, out, du, dv);
}

void orc_lift(const double *dsm, int Hd, int Wd, double x0, double y0, double gsd,
              const double *uv, int N, const double *ref_map, int Hr, int Wr, int C, double scale,
              double *P, double *ref)
{
    for (int j = 0; j < N; ++j) {
        const double u = uv[2 * j], v = uv[2 * j + 1];
        double h;
        sample_clamped(dsm, Hd, Wd, 1, u, v, &h);
        P[3 * j] = x0 + u * gsd;
        P[3 * j + 1] = y0 + v * gsd;
        P[3 * j + 2] = h;
        sample_clamped(ref_map, Hr, Wr, C, scale * (u + 0.5) - 0.5, scale * (v + 0.5) - 0.5, ref + (size_t)j * C);
    }
}

/* Selection of the output pose: the hypothesis with the lowest final
 * objective (Method, Multi-Sensor Optimization).  Non-finite costs and
 * degenerate hypotheses never win; ties go to the lowest index. */
int orc_best(const double *cost, const int *status, int M)
{
    int best = -1;
    for (int m = 0; m < M; ++m) {
        if (status[m] == ORC_DEGENERATE || status[m] == ORC_PRUNED || !isfinite(cost[m])) continue;
        if (best < 0 || cost[m] < cost[best]) best = m;
    }
    return best;
}
