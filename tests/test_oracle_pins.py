"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(closed forms, library routines, finite differences, the synthetic scene's
own ground truth).  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

import oracle
from synth import frames as S

HERE = os.path.dirname(os.path.abspath(__file__))


def small_frame(noise=True, seed=5, N=96, M=3, levels=((60, 80, 16), (120, 160, 32)), iters=(8, 8)):
    return S.make_frame(2, 0, noise=noise, N=N, M=M, level_shapes=levels, iters=iters,
                        dsm_side=128, seed=seed)


def rand_pose(rng, scale_t=1.0, scale_r=0.3):
    return oracle.se3_exp(np.concatenate([rng.normal(0, scale_t, 3), rng.normal(0, scale_r, 3)]))


def left_perturb(T, d):
    return oracle.compose(oracle.se3_exp(d), T)


def mask_cell_edges(frame, pose, eps=1e-3):
    """ref_w = 0 for anchors whose projection lies within eps px of a pixel
    row/column or of the image border at any level (the bilinear gradient
    jumps there, so finite differences across it are meaningless)."""
    R = pose[:9].reshape(3, 3)
    for L in frame.levels:
        P = np.stack([L.x, L.y, L.z], 1).astype(np.float64)
        X = P @ R.T + pose[9:]
        u = L.K[0] * X[:, 0] / X[:, 2] + L.K[2]
        v = L.K[1] * X[:, 1] / X[:, 2] + L.K[3]
        near = (np.abs(u - np.round(u)) < eps) | (np.abs(v - np.round(v)) < eps)
        w = np.ones(len(u), np.float32) if L.ref_w is None else L.ref_w.copy()
        w[near] = 0.0
        L.ref_w = w
    return frame


# ---------------------------------------------------------------- SE(3)
def test_exp_matches_matrix_exponential():
    rng = np.random.default_rng(0)
    for scale in (1e-9, 1e-5, 1e-3, 0.1, 1.0, 3.0):
        xi = np.concatenate([rng.normal(0, 5, 3), rng.normal(0, scale, 3)])
        T = oracle.se3_exp(xi)
        tw = np.zeros((4, 4))
        w = xi[3:]
        tw[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
        tw[:3, 3] = xi[:3]
        E = scipy.linalg.expm(tw)
        assert np.allclose(T[:9].reshape(3, 3), E[:3, :3], atol=1e-13, rtol=0)
        assert np.allclose(T[9:], E[:3, 3], atol=1e-12, rtol=0)
        assert np.allclose(T[:9].reshape(3, 3), Rotation.from_rotvec(w).as_matrix(), atol=1e-13)


def test_exp_log_round_trip_and_orthonormal():
    rng = np.random.default_rng(1)
    for scale in (0.0, 1e-8, 1e-4, 0.5, 2.0, 3.1):
        xi = np.concatenate([rng.normal(0, 10, 3), rng.normal(0, 1, 3)])
        if scale == 0.0:
            xi[3:] = 0
        else:
            xi[3:] *= scale / np.linalg.norm(xi[3:])
        T = oracle.se3_exp(xi)
        R = T[:9].reshape(3, 3)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        assert np.allclose(oracle.se3_log(T), xi, atol=1e-12 * max(1, np.abs(xi).max()))


def test_exp_small_angle_branch_is_continuous():
    w = np.array([0.3, -0.2, 0.9])
    w /= np.linalg.norm(w)
    rho = np.array([2.0, -1.0, 0.5])
    a = oracle.se3_exp(np.concatenate([rho, w * (1e-4 * (1 - 1e-9))]))
    b = oracle.se3_exp(np.concatenate([rho, w * (1e-4 * (1 + 1e-9))]))
    assert np.abs(a - b).max() < 1e-12


def test_compose_is_matrix_product():
    rng = np.random.default_rng(2)
    A, B = rand_pose(rng), rand_pose(rng)

    def m4(T):
        M = np.eye(4)
        M[:3, :3] = T[:9].reshape(3, 3)
        M[:3, 3] = T[9:]
        return M
    AB = oracle.compose(A, B)
    assert np.allclose(m4(AB), m4(A) @ m4(B), atol=1e-14)


# ---------------------------------------------------------------- losses
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_robust_derivative_and_values(kind):
    b = 0.37
    for s in (1e-4, 0.1, 0.37, 0.5, 3.0, 40.0):
        rho, d = oracle.robust(kind, b, s)
        h = 1e-6 * max(s, 1e-3)
        fd = (oracle.robust(kind, b, s + h)[0] - oracle.robust(kind, b, s - h)[0]) / (2 * h)
        if kind == 1 and abs(s - b) < 2 * h:
            continue
        assert abs(fd - d) < 1e-6 * max(1, abs(d))
    if kind == 0:
        assert abs(oracle.robust(0, b, b)[0] - b * math.log(2)) < 1e-15
    if kind == 1:
        lo, hi = oracle.robust(1, b, b * (1 - 1e-12))[0], oracle.robust(1, b, b * (1 + 1e-12))[0]
        assert abs(lo - hi) < 1e-10
        assert oracle.robust(1, b, 4 * b)[0] == pytest.approx(3 * b, rel=1e-14)


# ---------------------------------------------------------------- bilinear
def test_bilinear_exact_on_affine_fields():
    rng = np.random.default_rng(3)
    H, W, C = 7, 9, 5
    a, b, c = rng.normal(size=C), rng.normal(size=C), rng.normal(size=C)
    vv, uu = np.mgrid[0:H, 0:W]
    F = uu[..., None] * a + vv[..., None] * b + c
    for u, v in [(0.0, 0.0), (8.0, 6.0), (3.25, 2.5), (7.999, 0.001), (4.0, 3.0)]:
        val, du, dv = oracle.bilinear(F, u, v)
        assert np.allclose(val, a * u + b * v + c, atol=1e-13)
        assert np.allclose(du, a, atol=1e-13)
        assert np.allclose(dv, b, atol=1e-13)


def test_bilinear_integer_coordinates_and_cell_derivatives():
    rng = np.random.default_rng(4)
    F = rng.normal(size=(6, 8, 3))
    for (u, v) in [(0, 0), (3, 2), (7, 5), (6, 5)]:
        val, _, _ = oracle.bilinear(F, float(u), float(v))
        assert np.array_equal(val, F[v, u])
    u, v = 2.3, 3.6
    val, du, dv = oracle.bilinear(F, u, v)
    h = 1e-6
    fu = (oracle.bilinear(F, u + h, v)[0] - oracle.bilinear(F, u - h, v)[0]) / (2 * h)
    fv = (oracle.bilinear(F, u, v + h)[0] - oracle.bilinear(F, u, v - h)[0]) / (2 * h)
    assert np.allclose(fu, du, atol=1e-8) and np.allclose(fv, dv, atol=1e-8)


# ---------------------------------------------------------------- projection
def test_projection_closed_form_through_affine_features():
    """With an affine descriptor field and zero reference, the residual
    channels read back (u, v): pins the pinhole of Eq. (1)."""
    f = small_frame(N=4, M=1, levels=((40, 60, 2),), iters=(1,))
    L = f.levels[0]
    vv, uu = np.mgrid[0:L.H, 0:L.W]
    L.feat = np.stack([uu, vv], -1).astype(np.float32)
    L.K = (50.0, 40.0, 29.5, 19.5)
    L.x[:] = [0.0, 1.0, -2.0, 0.5]
    L.y[:] = [0.0, 2.0, 1.0, -1.0]
    L.z[:] = [10.0, 10.0, 20.0, 5.0]
    L.ref = np.zeros((4, 2), np.float32)
    of = oracle.OracleFrame(f)
    T = np.concatenate([np.eye(3).ravel(), np.zeros(3)])
    for j, (x, y, z) in enumerate([(0, 0, 10), (1, 2, 10), (-2, 1, 20), (0.5, -1, 5)]):
        ok, r, J, w = oracle.photo_point(of, 0, T, j)
        assert ok and w == 1.0
        assert r[0] == pytest.approx(50.0 * x / z + 29.5, abs=1e-12)
        assert r[1] == pytest.approx(40.0 * y / z + 19.5, abs=1e-12)
    # a translated camera: X_cam = X + t
    T2 = T.copy()
    T2[9:] = [1.0, -1.0, 10.0]
    ok, r, _, _ = oracle.photo_point(of, 0, T2, 1)
    assert r[0] == pytest.approx(50.0 * 2.0 / 20.0 + 29.5) and r[1] == pytest.approx(40.0 * 1.0 / 20.0 + 19.5)
    # behind the camera / outside the image -> not visible
    T3 = T.copy()
    T3[9:] = [0, 0, -30.0]
    assert not oracle.photo_point(of, 0, T3, 0)[0]
    T4 = T.copy()
    T4[9:] = [100.0, 0, 0]
    assert not oracle.photo_point(of, 0, T4, 0)[0]


def test_out_of_view_penalty():
    f = small_frame(N=8, M=1, levels=((40, 60, 4),), iters=(1,))
    f.use_gravity = f.use_range = 0
    T = f.gt_pose.copy()
    T[9:] += [0, 0, -1e4]                       # everything behind the camera
    of = oracle.OracleFrame(f)
    H, g, c, n = oracle.linearize(of, 0, T)
    b = f.levels[0].loss[1]
    assert n == 0 and np.all(H == 0) and np.all(g == 0)
    assert c == pytest.approx(8 * b * math.log1p(2.0 / b), rel=1e-14)


# ---------------------------------------------------------------- confidence weights
def _in_view_frame(seed, poses, margin=1.5, N=120, loss=None):
    """A two-level frame without priors whose anchors all project at least
    `margin` px inside every level under every pose in `poses` (so no anchor
    takes the out-of-view penalty, which carries the per-anchor weight only)."""
    f = small_frame(seed=seed, N=N, M=1)
    f.use_gravity = f.use_range = 0
    keep = np.ones(N, bool)
    for L in f.levels:
        P = np.stack([L.x, L.y, L.z], 1).astype(np.float64)
        for T in poses:
            X = P @ T[:9].reshape(3, 3).T + T[9:]
            u = L.K[0] * X[:, 0] / X[:, 2] + L.K[2]
            v = L.K[1] * X[:, 1] / X[:, 2] + L.K[3]
            keep &= (X[:, 2] > 1.0) & (u >= margin) & (u <= L.W - 1 - margin) & (v >= margin) & (v <= L.H - 1 - margin)
    assert keep.sum() >= N // 2
    for L in f.levels:
        L.x, L.y, L.z, L.ref = L.x[keep], L.y[keep], L.z[keep], L.ref[keep]
        if loss is not None:
            L.loss = (loss, L.loss[1])
    return f


def _pix(L, T):
    P = np.stack([L.x, L.y, L.z], 1).astype(np.float64)
    X = P @ T[:9].reshape(3, 3).T + T[9:]
    return L.K[0] * X[:, 0] / X[:, 2] + L.K[2], L.K[1] * X[:, 1] / X[:, 2] + L.K[3]


def _close(a, b, rtol):
    Ha, ga, ca, na = a
    Hb, gb, cb, nb = b
    assert na == nb
    assert np.linalg.norm(Ha - Hb) <= rtol * np.linalg.norm(Hb)
    assert np.linalg.norm(ga - gb) <= rtol * np.linalg.norm(gb)
    assert abs(ca - cb) <= rtol * abs(cb)


@pytest.mark.parametrize("loss", [0, 1])
def test_constant_query_confidence_equals_scaled_anchor_weights(loss):
    """W of Eq. (8) multiplies the anchor weight by the query confidence at
    the projection: a constant confidence map kappa gives exactly the system
    of the same frame with every anchor weight scaled by kappa."""
    rng = np.random.default_rng(21)
    base = small_frame(seed=13, N=120, M=1)
    poses = [left_perturb(base.gt_pose, np.concatenate([rng.normal(0, 1.0, 3), rng.normal(0, 0.01, 3)]))
             for _ in range(3)]
    kappa = 0.37
    a = _in_view_frame(13, poses, loss=loss)
    b = _in_view_frame(13, poses, loss=loss)
    for La, Lb in zip(a.levels, b.levels):
        La.qconf = np.full((La.H, La.W), kappa)
        Lb.ref_w = np.full(len(Lb.x), kappa)
    oa, ob = oracle.OracleFrame(a), oracle.OracleFrame(b)
    for l in range(2):
        for T in poses:
            _close(oracle.linearize(oa, l, T), oracle.linearize(ob, l, T), 1e-12)


@pytest.mark.parametrize("loss", [0, 1])
def test_affine_query_confidence_is_read_at_the_projection(loss):
    """Bilinear interpolation reproduces an affine confidence field exactly,
    so q(u, v) = q0 + qu u + qv v must equal anchor weights set to that
    affine value at each anchor's projection (computed here with numpy).
    Different slopes along u and v expose a transposed lookup."""
    rng = np.random.default_rng(22)
    base = small_frame(seed=14, N=120, M=1)
    poses = [left_perturb(base.gt_pose, np.concatenate([rng.normal(0, 1.0, 3), rng.normal(0, 0.01, 3)]))
             for _ in range(2)]
    for T in poses:
        a = _in_view_frame(14, [T], loss=loss)
        b = _in_view_frame(14, [T], loss=loss)
        for La, Lb in zip(a.levels, b.levels):
            q0, qu, qv = 0.3, 0.7 / La.W, -0.2 / La.H       # positive over the map
            vv, uu = np.mgrid[0:La.H, 0:La.W]
            La.qconf = q0 + qu * uu + qv * vv
            u, v = _pix(Lb, T)
            Lb.ref_w = q0 + qu * u + qv * v
        oa, ob = oracle.OracleFrame(a), oracle.OracleFrame(b)
        for l in range(2):
            _close(oracle.linearize(oa, l, T), oracle.linearize(ob, l, T), 1e-11)


@pytest.mark.parametrize("loss", [0, 1, 2])
def test_confidence_weight_sits_inside_the_robust_loss(loss):
    """Eq. (2) applies rho to w |r|^2.  For the Cauchy and Huber losses
    rho_b(kappa s) = kappa rho_{b / kappa}(s) (and rho'_b(kappa s) kappa =
    kappa rho'_{b / kappa}(s)), so weights kappa at scale b give kappa times
    the visual system of unit weights at scale b / kappa -- out-of-view
    penalties included.  A weight applied outside rho breaks this."""
    rng = np.random.default_rng(23)
    f = small_frame(seed=15, N=96, M=1)
    f.use_gravity = f.use_range = 0
    # a pose that leaves about 40 % of the anchors out of view
    T = left_perturb(f.gt_pose, np.concatenate([rng.normal(0, 3.0, 3), rng.normal(0, 0.2, 3)]))
    kappa = 4.5
    a = small_frame(seed=15, N=96, M=1)
    b = small_frame(seed=15, N=96, M=1)
    for fr in (a, b):
        fr.use_gravity = fr.use_range = 0
    for La, Lb in zip(a.levels, b.levels):
        scale = La.loss[1]
        La.loss = (loss, scale)
        La.ref_w = np.full(len(La.x), kappa)
        Lb.loss = (loss, scale / kappa)
    oa, ob = oracle.OracleFrame(a), oracle.OracleFrame(b)
    for l in range(2):
        Ha, ga, ca, na = oracle.linearize_visual(oa, l, T)
        Hb, gb, cb, nb = oracle.linearize_visual(ob, l, T)
        assert na == nb and 0 < na < 96               # both visible anchors and penalties
        _close((Ha, ga, ca, na), (kappa * Hb, kappa * gb, kappa * cb, nb), 1e-12)


# ---------------------------------------------------------------- Jacobians
def fd_jacobian(fun, T, h=1e-6):
    cols = []
    for k in range(6):
        d = np.zeros(6)
        d[k] = h
        cols.append((np.atleast_1d(fun(left_perturb(T, d))) - np.atleast_1d(fun(left_perturb(T, -d)))) / (2 * h))
    return np.stack(cols, -1)


def test_photo_jacobian_matches_finite_differences():
    f = small_frame()
    of = oracle.OracleFrame(f)
    rng = np.random.default_rng(6)
    T = left_perturb(f.gt_pose, np.concatenate([rng.normal(0, 0.5, 3), rng.normal(0, 0.005, 3)]))
    mask_cell_edges(f, T, eps=1e-2)
    checked = 0
    for l in range(2):
        for j in range(f.levels[l].N):
            if f.levels[l].ref_w[j] == 0:
                continue
            ok, r, J, w = oracle.photo_point(of, l, T, j)
            if not ok:
                continue
            Jfd = fd_jacobian(lambda X: oracle.photo_point(of, l, X, j)[1], T, h=1e-7)
            assert np.allclose(J, Jfd, atol=1e-5 * max(1, np.abs(J).max()))
            checked += 1
    assert checked > 100


def test_gravity_zero_at_truth_null_space_and_fd():
    f = small_frame(noise=False)
    of = oracle.OracleFrame(f)
    r, J = oracle.gravity(of, f.gt_pose)
    assert np.abs(r).max() < 1e-14
    T = left_perturb(f.gt_pose, np.array([0.3, -0.1, 0.2, 0.02, -0.03, 0.01]))
    r, J = oracle.gravity(of, T)
    assert np.allclose(J, fd_jacobian(lambda X: oracle.gravity(of, X)[0], T), atol=1e-8)
    gc = T[:9].reshape(3, 3) @ np.array(f.g_world)
    assert np.abs(J @ np.concatenate([np.zeros(3), gc])).max() < 1e-14     # yaw about gravity
    assert np.abs(J[:, :3]).max() == 0.0                                  # no translation


def test_range_zero_at_truth_and_fd():
    f = small_frame(noise=False)
    of = oracle.OracleFrame(f)
    r, J = oracle.range_term(of, f.gt_pose)
    assert abs(r) < 1e-7
    T = left_perturb(f.gt_pose, np.array([0.3, -0.1, 0.2, 0.002, -0.003, 0.001]))
    r, J = oracle.range_term(of, T)
    assert np.allclose(J, fd_jacobian(lambda X: oracle.range_term(of, X)[0], T, h=1e-7)[0], atol=1e-5)


def test_dsm_lookup_against_raster():
    f = small_frame()
    of = oracle.OracleFrame(f)
    D = f.dsm
    for (i, j) in [(0, 0), (5, 7), (127, 127), (60, 3)]:
        h, _, _ = oracle.dsm(of, D.x0 + j * D.gsd, D.y0 + i * D.gsd)
        assert h == pytest.approx(float(D.heights[i, j]), abs=1e-12)
    h, hx, hy = oracle.dsm(of, D.x0 - 100.0, D.y0 + 3 * D.gsd)        # clamped in x
    assert h == pytest.approx(float(D.heights[3, 0])) and hx == 0.0


def test_non_finite_pose_is_degenerate_not_a_crash():
    f = small_frame(M=3)
    P = f.poses.copy()
    P[1, 0] = np.nan
    P[2, 9:] = [0.0, 0.0, -1e5]
    f.poses = P
    of = oracle.OracleFrame(f)
    assert math.isnan(oracle.dsm(of, float("nan"), 0.0)[0]) is False
    r = oracle.solve(f, threads=2)
    assert r["status"][1] == oracle.DEGENERATE and r["status"][2] == oracle.DEGENERATE
    assert r["best"] == 0


# ---------------------------------------------------------------- normal equations
def total_cost(of, l, T):
    return oracle.linearize(of, l, T)[2]


@pytest.mark.parametrize("loss", [0, 1, 2])
def test_gradient_is_half_cost_gradient(loss):
    """Gauss-Newton with IRLS weights: g = J^T W r = 1/2 d(cost)/d(xi)."""
    f = small_frame(seed=11)
    rng = np.random.default_rng(7)
    T = left_perturb(f.gt_pose, np.concatenate([rng.normal(0, 0.8, 3), rng.normal(0, 0.008, 3)]))
    mask_cell_edges(f, T, eps=5e-3)
    for L in f.levels:
        L.loss = (loss, L.loss[1])
    f.gravity_loss = (loss, f.gravity_loss[1])
    f.range_loss = (loss, f.range_loss[1])
    f.lambda_range = 5.0          # make the prior terms visible in the sum
    f.lambda_imu = 500.0
    of = oracle.OracleFrame(f)
    for l in range(2):
        H, g, c, n = oracle.linearize(of, l, T)
        fd = fd_jacobian(lambda X: total_cost(of, l, X), T, h=1e-7)[0]
        assert np.allclose(g, 0.5 * fd, rtol=1e-5, atol=1e-6 * np.abs(g).max())


def test_hessian_is_jtwj_with_fd_jacobian():
    f = small_frame(N=16, seed=12)
    rng = np.random.default_rng(8)
    T = left_perturb(f.gt_pose, np.concatenate([rng.normal(0, 0.5, 3), rng.normal(0, 0.005, 3)]))
    mask_cell_edges(f, T, eps=1e-2)
    f.lambda_range = 3.0
    of = oracle.OracleFrame(f)
    l = 1
    L = f.levels[l]
    Href = np.zeros((6, 6))
    for j in range(L.N):
        ok, r, J, w = oracle.photo_point(of, l, T, j)
        if not ok:
            continue
        Jfd = fd_jacobian(lambda X: oracle.photo_point(of, l, X, j)[1], T, h=1e-7)
        s = w * float(r @ r)
        Href += oracle.robust(L.loss[0], L.loss[1], s)[1] * w * Jfd.T @ Jfd
    rg, _ = oracle.gravity(of, T)
    Jg = fd_jacobian(lambda X: oracle.gravity(of, X)[0], T)
    Href += f.lambda_imu * oracle.robust(*f.gravity_loss, float(rg @ rg))[1] * Jg.T @ Jg
    rr, _ = oracle.range_term(of, T)
    Jr = fd_jacobian(lambda X: oracle.range_term(of, X)[0], T, h=1e-7)
    Href += f.lambda_range * oracle.robust(*f.range_loss, rr * rr)[1] * Jr.T @ Jr
    H, g, c, n = oracle.linearize(of, l, T)
    assert np.allclose(H, Href, rtol=1e-5, atol=1e-6 * np.abs(H).max())


def test_cholesky_matches_lapack():
    rng = np.random.default_rng(9)
    for _ in range(20):
        A = rng.normal(size=(6, 6))
        A = A @ A.T + 1e-3 * np.eye(6)
        b = rng.normal(size=6)
        rc, x = oracle.cholesky_solve6(A, b)
        assert rc == 0
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    A = np.diag([1.0, 1, 1, 1, 1, -1e-3])
    assert oracle.cholesky_solve6(A, np.ones(6))[0] == -1


# ---------------------------------------------------------------- LM
def test_noise_free_frames_converge_to_ground_truth():
    for cfg, kw in [(1, {}), (2, dict(N=512, M=1, level_shapes=((60, 80, 16), (120, 160, 32), (240, 320, 32)),
                                      iters=(15, 15, 15)))]:
        f = S.make_frame(cfg, 0, noise=False, **kw)
        r = oracle.solve(f, threads=4)
        te, re = S.pose_errors(r["poses"], f.gt_pose)
        assert te[0] < 1e-6 and re[0] < 1e-6, (cfg, te, re)
        assert r["status"][0] == oracle.CONVERGED


def test_accepted_costs_never_increase():
    f = S.make_frame(2, 3, N=400, M=6, level_shapes=((60, 80, 16), (120, 160, 32)), iters=(25, 25))
    f.lm["step_tol_t"] = f.lm["step_tol_r"] = f.lm["cost_tol"] = 0.0      # run every iteration
    r = oracle.solve(f, threads=4, trace=True)
    tr = r["trace"]
    for m in range(tr.shape[0]):
        rows = tr[m][~np.isnan(tr[m][:, 0])]
        for lvl in np.unique(rows[:, 0]):
            R = rows[rows[:, 0] == lvl]
            cur = R[:, 1]
            assert np.all(np.diff(cur) <= 0)
            acc = R[:, 3] == 1
            assert np.all(R[acc, 2] < R[acc, 1])
            assert np.all(R[~acc & ~np.isnan(R[:, 2]), 2] >= R[~acc & ~np.isnan(R[:, 2]), 1])


def test_top_k_pruning_keeps_the_lowest_post_coarse_costs():
    """Supplement, Multi-Hypothesis Refinement: after the coarse level only the
    best-ranked hypotheses continue.  The survivors must be exactly the K
    lowest costs of a run that stops after the coarse level."""
    f = S.make_frame(2, 4, N=300, M=12, level_shapes=((30, 40, 16), (60, 80, 32)), iters=(4, 3),
                     dsm_side=128, seed=77)
    coarse_only = S.make_frame(2, 4, N=300, M=12, level_shapes=((30, 40, 16),), iters=(4,),
                               dsm_side=128, seed=77)
    r0 = oracle.solve(coarse_only, threads=4)
    f.keep_top, f.prune_level = 5, 0
    r = oracle.solve(f, threads=4)
    alive = r0["status"] != oracle.DEGENERATE
    order = sorted(np.flatnonzero(alive), key=lambda m: (r0["cost"][m], m))
    expect = set(order[:5])
    kept = set(np.flatnonzero(r["status"] != oracle.PRUNED)) - set(np.flatnonzero(~alive))
    assert kept == expect
    for m in range(f.M):
        if r["status"][m] == oracle.PRUNED:       # pruned: pose and cost stay at the coarse result
            assert np.array_equal(r["poses"][m], r0["poses"][m]) and r["cost"][m] == r0["cost"][m]
            assert r["iterations"][m] == r0["iterations"][m]
    assert r["best"] in expect


def test_lift_at_grid_points_and_affine_maps():
    """Anchors at integer DSM samples lift to the raster's own heights and
    coordinates; an affine reference map is reproduced exactly, clamped at
    the border."""
    rng = np.random.default_rng(12)
    D = rng.uniform(0, 50, size=(9, 11))
    uv = np.array([[0, 0], [10, 8], [3, 4], [2.5, 7.25], [-3.0, 1.0], [10.7, 8.9]])
    Hr, Wr, Cc, sc = 18, 22, 3, 2.0
    a, b, c = rng.normal(size=Cc), rng.normal(size=Cc), rng.normal(size=Cc)
    vv, uu = np.mgrid[0:Hr, 0:Wr]
    Fm = uu[..., None] * a + vv[..., None] * b + c
    P, ref = oracle.lift(D, -5.0, 7.0, 0.5, uv, Fm, sc)
    for k in range(3):
        u, v = uv[k].astype(int)
        assert P[k, 2] == D[v, u] and P[k, 0] == -5.0 + 0.5 * u and P[k, 1] == 7.0 + 0.5 * v
    for k in range(len(uv)):
        mu = np.clip(sc * (uv[k, 0] + 0.5) - 0.5, 0, Wr - 1)
        mv = np.clip(sc * (uv[k, 1] + 0.5) - 0.5, 0, Hr - 1)
        assert np.allclose(ref[k], a * mu + b * mv + c, atol=1e-12)
    assert P[4, 2] == pytest.approx(D[1, 0])        # clamped in u


def test_selection_rule():
    cost = np.array([3.0, np.nan, 1.0, 1.0, 0.5])
    st = np.array([1, 1, 0, 1, 3], np.int32)
    import ctypes as C
    b = oracle.lib().orc_best(cost.ctypes.data_as(C.POINTER(C.c_double)), st.ctypes.data_as(C.POINTER(C.c_int)), 5)
    assert b == 2


# ---------------------------------------------------------------- paper constants
def test_paper_hypothesis_grid():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    g = gold["hypothesis_grid"]
    offs = S.paper_grid_offsets()
    assert len(offs) == g["count"] == 1210
    assert len(set((round(a, 9), round(b, 9), round(c, 12)) for a, b, c in offs)) == 1210
    yaws = sorted(set(round(math.degrees(c), 9) for _, _, c in offs))
    assert yaws == sorted([s * a for a in g["yaw_offsets_deg"] for s in (1, -1)])
    xs = sorted(set(round(a, 9) for a, _, _ in offs))
    assert xs[0] == -g["xy_range_m"] and xs[-1] == g["xy_range_m"] and len(xs) == 11
    assert sum(gold["schedule"]["iters_coarse_to_fine"]) == gold["schedule"]["unrolled_steps"]


# ---------------------------------------------------------------- adaptive prior scales
def _prior_parts(f, level, T):
    """Visual gradient, unit-scale gravity and range gradients and residual
    norms, taken from the fixed-scale objective with the priors switched on
    one at a time."""
    import copy
    base = copy.copy(f)
    base.use_gravity = base.use_range = 0
    gv = oracle.linearize(oracle.OracleFrame(base), level, T)[1]
    fg = copy.copy(f)
    fg.use_range, fg.lambda_imu = 0, 1.0
    g1 = oracle.linearize(oracle.OracleFrame(fg), level, T)[1]
    fr = copy.copy(f)
    fr.use_gravity, fr.lambda_range = 0, 1.0
    g2 = oracle.linearize(oracle.OracleFrame(fr), level, T)[1]
    of = oracle.OracleFrame(f)
    return gv, g1 - gv, g2 - gv, np.linalg.norm(oracle.gravity(of, T)[0]), abs(oracle.range_term(of, T)[0])


def _off_pose(f):
    # 4 m and 1.5 deg of roll off the truth: both prior residuals are large
    return left_perturb(f.gt_pose, np.array([2.0, -3.0, 1.5, math.radians(1.5), 0.0, 0.0]))


def test_adaptive_scales_reduce_to_fixed_without_cap_or_gate():
    f = small_frame(M=4)
    fixed = oracle.solve(f, threads=2)
    assert np.array_equal(fixed["alpha"], np.tile([f.lambda_imu, f.lambda_range], (4, 1)))
    f.adaptive_priors, f.alpha_ratio, f.gravity_gate, f.range_gate = 1, 0.0, 0.0, 0.0
    T = _off_pose(f)
    a = oracle.prior_scales(oracle.OracleFrame(f), T, np.ones(6))
    assert a[0] == f.lambda_imu and a[1] == f.lambda_range
    ad = oracle.solve(f, threads=2)
    for k in ("poses", "cost", "iterations", "status", "alpha"):
        assert np.array_equal(ad[k], fixed[k]), k
    f.use_gravity = 0
    assert oracle.prior_scales(oracle.OracleFrame(f), T, np.ones(6))[0] == 0.0


def test_ratio_cap_balances_prior_and_visual_gradients():
    f = small_frame()
    T = _off_pose(f)
    gv, gg, gr, _, _ = _prior_parts(f, 1, T)
    nv, ng, nr = np.linalg.norm(gv), np.linalg.norm(gg), np.linalg.norm(gr)
    f.adaptive_priors, f.gravity_gate, f.range_gate = 1, 0.0, 0.0
    for beta in (1e-4, 1e-2, 1.0, 1e6):
        f.alpha_ratio = beta
        a = oracle.prior_scales(oracle.OracleFrame(f), T, gv)
        for s, lam, n in ((0, f.lambda_imu, ng), (1, f.lambda_range, nr)):
            if lam * n > beta * nv:            # capped: the scaled prior gradient equals beta |g_vis|
                assert a[s] < lam
                assert a[s] * n == pytest.approx(beta * nv, rel=1e-8)
            else:
                assert a[s] == lam
    f.alpha_ratio = 1e-4
    a = oracle.prior_scales(oracle.OracleFrame(f), T, gv)
    assert a[0] < f.lambda_imu and a[1] < f.lambda_range           # the small ratio binds both


def test_residual_gate_scales_by_inverse_square():
    f = small_frame()
    T = _off_pose(f)
    gv, _, _, rg, rr = _prior_parts(f, 1, T)
    assert rg > 1e-3 and rr > 0.1
    f.adaptive_priors, f.alpha_ratio = 1, 0.0
    for k in (0.25, 0.5, 1.0, 2.0):
        f.gravity_gate, f.range_gate = k * rg, k * rr
        a = oracle.prior_scales(oracle.OracleFrame(f), T, gv)
        expect = min(1.0, k * k)
        assert a[0] == pytest.approx(f.lambda_imu * expect, rel=1e-12)
        assert a[1] == pytest.approx(f.lambda_range * expect, rel=1e-12)


def test_solve_reports_the_scales_of_the_level_start():
    f = small_frame(M=3, levels=((120, 160, 32),), iters=(0,))
    f.adaptive_priors, f.alpha_ratio = 1, 0.05
    r = oracle.solve(f, threads=2)
    of = oracle.OracleFrame(f)
    for m in range(3):
        gv = oracle.linearize_visual(of, 0, f.poses[m])[1]
        assert np.array_equal(r["alpha"][m], oracle.prior_scales(of, f.poses[m], gv))


def test_adaptive_accepted_costs_never_increase_within_a_level():
    f = S.make_frame(2, 3, N=400, M=6, level_shapes=((60, 80, 16), (120, 160, 32)), iters=(25, 25))
    f.lm["step_tol_t"] = f.lm["step_tol_r"] = f.lm["cost_tol"] = 0.0
    f.adaptive_priors, f.alpha_ratio = 1, 0.05
    r = oracle.solve(f, threads=4, trace=True)
    tr = r["trace"]
    for m in range(tr.shape[0]):
        rows = tr[m][~np.isnan(tr[m][:, 0])]
        for lvl in np.unique(rows[:, 0]):
            R = rows[rows[:, 0] == lvl]
            assert np.all(np.diff(R[:, 1]) <= 0)


def test_gate_protects_against_a_corrupted_range_reading():
    """A range reading 40 m too long pulls a fixed-scale solve off the truth;
    with the residual gate the solution stays with the visual one."""
    f = S.make_frame(1, 0, noise=False)
    f.lambda_range = 1.0
    f.d_range += 40.0
    fixed = oracle.solve(f, threads=2)
    f.adaptive_priors = 1
    gated = oracle.solve(f, threads=2)
    f.use_range = 0
    visual = oracle.solve(f, threads=2)
    e_fixed = S.pose_errors(fixed["poses"][0], f.gt_pose)[0][0]
    e_gated = S.pose_errors(gated["poses"][0], f.gt_pose)[0][0]
    e_vis = S.pose_errors(visual["poses"][0], f.gt_pose)[0][0]
    assert e_vis < 1e-5
    assert e_fixed > 10.0, e_fixed                      # the bad reading wins at a fixed scale
    assert e_gated < 0.5 and e_gated < e_fixed / 50.0, (e_gated, e_fixed)


# ---------------------------------------------------------------- LM stopping rules
def test_cost_tolerance_stops_exactly_where_the_cost_goes_flat():
    """With the function tolerance on, a level ends at the first candidate
    whose cost is within cost_tol of the current cost and not before."""
    f = S.make_frame(2, 3, N=400, M=6, level_shapes=((60, 80, 16), (120, 160, 32)), iters=(25, 25))
    f.lm["step_tol_t"] = f.lm["step_tol_r"] = 0.0        # only the cost rule may stop a level
    tol = f.lm["cost_tol"] = 1e-9
    r = oracle.solve(f, threads=4, trace=True)
    tr = r["trace"]
    stopped = 0
    for m in range(tr.shape[0]):
        rows = tr[m][~np.isnan(tr[m][:, 0])]
        for lvl in np.unique(rows[:, 0]):
            R = rows[rows[:, 0] == lvl]
            flat = np.abs(R[:, 2] - R[:, 1]) <= tol * R[:, 1]
            assert not flat[:-1].any()                    # never ran past a flat candidate
            stopped += bool(flat[-1])
            if len(R) < f.levels[int(lvl)].iters:         # ended early: only the cost rule can do that
                assert flat[-1] or r["status"][m] == oracle.STALLED
    assert stopped > 0
    # a huge tolerance ends every level at its first candidate
    f.lm["cost_tol"] = 1.0
    r = oracle.solve(f, threads=4)
    ok = r["status"] != oracle.DEGENERATE
    assert np.all(r["iterations"][ok] == len(f.levels)) and np.all(r["status"][ok] == oracle.CONVERGED)
