"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle with a second, independent route (a closed
form, a library routine, a finite difference, a brute-force search or an
exact construction whose answer is known), so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import (angle_deg, apply_h, bilinear_scipy, bilinear_scipy_many, huber,
                           plane_homography, random_unit_cap, ray, rot, smooth_texture)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rand_case(rng):
    K = (rng.uniform(100, 700), rng.uniform(100, 700), rng.uniform(40, 400), rng.uniform(30, 300))
    R = rot(rng.normal(size=3), math.radians(rng.uniform(0, 5)))
    t = rng.normal(size=3) * 0.1
    n = random_unit_cap(rng, 50)
    us = (rng.uniform(0, 600), rng.uniform(0, 400))
    id_s = rng.uniform(0.25, 1.0)
    return K, R, t, n, us, id_s


# --- Eq. 3 (inverse depth of a pixel on the surfel plane) -------------------

def test_eq3_matches_ray_plane_intersection_by_linear_solve():
    """Eq. 3 against a plane given by three points and a 3x3 linear solve."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        K, R, t, n, us, id_s = _rand_case(rng)
        ps = ray(K, *us) / id_s                     # Eq. 1
        # two in-plane directions, independent of how the oracle writes Eq. 3
        a = np.cross(n, [0.3, 0.5, 0.7]); a /= np.linalg.norm(a)
        b = np.cross(n, a)
        u = (us[0] + rng.uniform(-6, 6), us[1] + rng.uniform(-6, 6))
        ru = ray(K, *u)
        # solve lam * ru = ps + s a + q b for (lam, s, q)
        M = np.stack([ru, -a, -b], axis=1)
        lam, _, _ = np.linalg.solve(M, ps)
        got = oracle.pixel_inverse_depth(K, us, id_s, n, u)
        assert got == pytest.approx(1.0 / lam, rel=1e-11)


def test_eq3_special_cases():
    rng = np.random.default_rng(2)
    for _ in range(50):
        K, R, t, n, us, id_s = _rand_case(rng)
        # at the surfel's own centre pixel the plane gives id_s back
        assert oracle.pixel_inverse_depth(K, us, id_s, n, us) == pytest.approx(id_s, rel=1e-14)
        # a fronto-parallel plane has one inverse depth everywhere
        u = (rng.uniform(0, 600), rng.uniform(0, 400))
        assert oracle.pixel_inverse_depth(K, us, id_s, [0, 0, -1.0], u) == pytest.approx(id_s, rel=1e-14)
        # scale invariance in n (the normal has only two degrees of freedom)
        assert oracle.pixel_inverse_depth(K, us, id_s, 3.7 * n, u) == pytest.approx(
            oracle.pixel_inverse_depth(K, us, id_s, n, u), rel=1e-13)


# --- Eq. 6 (warp) -----------------------------------------------------------

def test_eq6_equals_plane_homography():
    """The back-project / transform / project chain equals the closed-form
    plane-induced homography K (R + t n^T / d) K^-1 (to 1e-9 px)."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        K, R, t, n, us, id_s = _rand_case(rng)
        ps = ray(K, *us) / id_s
        d = float(n @ ps)
        Hm = plane_homography(K, R, t, n, d)
        u = (us[0] + rng.uniform(-8, 8), us[1] + rng.uniform(-8, 8))
        id_u = oracle.pixel_inverse_depth(K, us, id_s, n, u)
        ok, uv = oracle.warp(K, R, t, u, id_u)
        if not ok:
            continue
        hx, hy = apply_h(Hm, *u)
        assert uv[0] == pytest.approx(hx, abs=1e-9)
        assert uv[1] == pytest.approx(hy, abs=1e-9)


def test_eq6_special_cases():
    K = (500.0, 480.0, 320.0, 240.0)
    rng = np.random.default_rng(4)
    for _ in range(50):
        u = (rng.uniform(0, 640), rng.uniform(0, 480))
        idu = rng.uniform(0.2, 1.0)
        ok, uv = oracle.warp(K, np.eye(3), np.zeros(3), u, idu)      # identity pose
        assert ok and uv[0] == pytest.approx(u[0], abs=1e-10) and uv[1] == pytest.approx(u[1], abs=1e-10)
        tx, ty = rng.normal(size=2) * 0.05                              # pure sideways motion
        ok, uv = oracle.warp(K, np.eye(3), np.array([tx, ty, 0.0]), u, idu)
        assert uv[0] == pytest.approx(u[0] + K[0] * tx * idu, abs=1e-10)
        assert uv[1] == pytest.approx(u[1] + K[1] * ty * idu, abs=1e-10)
    # behind the camera
    ok, _ = oracle.warp(K, np.eye(3), np.array([0, 0, -5.0]), (10, 10), 0.5)
    assert not ok


# --- bilinear sample and gradient -------------------------------------------

def test_bilinear_matches_scipy_and_linear_images():
    rng = np.random.default_rng(5)
    img = rng.uniform(size=(13, 17))
    for _ in range(500):
        x, y = rng.uniform(0, 15.999), rng.uniform(0, 11.999)
        ok, out = oracle.bilinear(img, x, y)
        assert ok
        assert out[0] == pytest.approx(bilinear_scipy(img, x, y), abs=1e-13)
    # on a linear image the interpolant is exact and its gradient constant
    ys, xs = np.mgrid[0:9, 0:11].astype(np.float64)
    lin = 0.25 * xs - 0.125 * ys + 0.5
    for _ in range(100):
        x, y = rng.uniform(0, 9.99), rng.uniform(0, 7.99)
        ok, out = oracle.bilinear(lin, x, y)
        assert out[0] == pytest.approx(0.25 * x - 0.125 * y + 0.5, abs=1e-14)
        assert out[1] == pytest.approx(0.25, abs=1e-14)
        assert out[2] == pytest.approx(-0.125, abs=1e-14)


def test_bilinear_gradient_is_derivative_of_interpolant():
    rng = np.random.default_rng(6)
    img = rng.uniform(size=(10, 10))
    h = 1e-7
    for _ in range(300):
        x0, y0 = rng.integers(0, 8, size=2)
        x = x0 + rng.uniform(0.01, 0.99)
        y = y0 + rng.uniform(0.01, 0.99)
        _, c = oracle.bilinear(img, x, y)
        _, px = oracle.bilinear(img, x + h, y)
        _, mx = oracle.bilinear(img, x - h, y)
        _, py = oracle.bilinear(img, x, y + h)
        _, my = oracle.bilinear(img, x, y - h)
        assert c[1] == pytest.approx((px[0] - mx[0]) / (2 * h), abs=1e-7)
        assert c[2] == pytest.approx((py[0] - my[0]) / (2 * h), abs=1e-7)


def test_bilinear_validity_edges():
    img = np.ones((6, 8))
    assert oracle.bilinear(img, 0.0, 0.0)[0]
    assert oracle.bilinear(img, 7.0 - 1e-9, 5.0 - 1e-9)[0]
    assert not oracle.bilinear(img, 7.0, 2.0)[0]
    assert not oracle.bilinear(img, 2.0, 5.0)[0]
    assert not oracle.bilinear(img, -1e-12, 2.0)[0]
    assert not oracle.bilinear(img, float("nan"), 2.0)[0]


def test_tangent_basis_orthonormal_right_handed():
    rng = np.random.default_rng(7)
    normals = [rng.normal(size=3) for _ in range(200)] + [[1, 0, 0], [0.95, 0.1, 0.0], [0, 0, -1]]
    for n in normals:
        n = np.asarray(n, float) / np.linalg.norm(n)
        b1, b2 = oracle.tangent_basis(n)
        B = np.stack([b1, b2, n])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(np.stack([b1, b2, n], axis=1)) == pytest.approx(1.0, abs=1e-13)


# --- Eq. 7-9 (Jacobian by the chain rule) -----------------------------------

def _jacobian_case(depth_only=False, seed=8, trials=300):
    rng = np.random.default_rng(seed)
    img = smooth_texture(96, 80, 11)
    checked = 0
    for _ in range(trials):
        K = (120.0, 118.0, 48.0, 40.0)
        R = rot(rng.normal(size=3), math.radians(rng.uniform(0, 3)))
        t = rng.normal(size=3) * 0.05
        n = random_unit_cap(rng, 40)
        us = (rng.uniform(20, 76), rng.uniform(20, 60))
        u = (us[0] + rng.uniform(-4, 4), us[1] + rng.uniform(-4, 4))
        id_s = rng.uniform(0.3, 1.0)
        kfv = rng.uniform()
        b1, b2 = oracle.tangent_basis(n)

        def res(th):
            nn = n + th[1] * b1 + th[2] * b2
            nn = nn / np.linalg.norm(nn)
            ok, r, _ = oracle.eval_sample(K, R, t, img, kfv, us, u, id_s + th[0], nn, depth_only)
            return ok, r

        ok, r, J = oracle.eval_sample(K, R, t, img, kfv, us, u, id_s, n, depth_only)
        if not ok:
            continue
        h = 1e-6
        # skip samples whose finite-difference stencil crosses a pixel cell
        ok0, uv0 = oracle.warp(K, R, t, u, oracle.pixel_inverse_depth(K, us, id_s, n, u))
        cell = (math.floor(uv0[0]), math.floor(uv0[1]))
        frac = (uv0[0] - cell[0], uv0[1] - cell[1])
        if min(frac[0], 1 - frac[0], frac[1], 1 - frac[1]) < 1e-3:
            continue
        fd = np.zeros(3)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            okp, rp = res(e)
            okm, rm = res(-e)
            fd[k] = (rp - rm) / (2 * h)
        if depth_only:
            assert J[1] == 0.0 and J[2] == 0.0
            assert J[0] == pytest.approx(fd[0], rel=1e-5, abs=1e-9)
        else:
            assert np.allclose(J, fd, rtol=1e-5, atol=1e-8 * max(1.0, np.abs(fd).max()))
        checked += 1
    assert checked > trials // 2


def test_jacobian_matches_finite_differences():
    _jacobian_case()


def test_depth_only_jacobian_keeps_the_inverse_depth_column():
    _jacobian_case(depth_only=True, seed=9)


# --- exact constructions: zero residual, fixed point, convergence ----------

def _construction_i(S=4, W=48, H=40):
    """Fronto-parallel plane at id = 0.5, R = I, t_z = 0, shifts fx t_x id and
    fy t_y id integers.  Every quantity of the chain is exact in binary."""
    K = (128.0, 128.0, 24.0, 20.0)
    shifts = [(2, 0), (0, 3)]

    def tex(x, y):
        rng = np.random.default_rng(3)
        out = 0.5
        for _ in range(6):
            ang = rng.uniform(0, 2 * math.pi)
            per = math.exp(rng.uniform(math.log(10), math.log(30)))
            ph = rng.uniform(0, 2 * math.pi)
            out = out + 0.06 * np.sin(2 * math.pi * (math.cos(ang) * x + math.sin(ang) * y) / per + ph)
        return out

    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    kfimg = tex(X, Y)
    nb = np.stack([tex(X - dx, Y - dy) for dx, dy in shifts])
    Rs = np.stack([np.eye(3)] * len(shifts))
    ts = np.array([[dx / (128 * 0.5), dy / (128 * 0.5), 0.0] for dx, dy in shifts])
    okf = oracle.OracleKeyframe(K, kfimg, nb, Rs, ts, S)
    m = (W // S) * (H // S)
    return okf, np.full(m, 0.5), np.tile([0.0, 0.0, -1.0], (m, 1))


def test_construction_i_zero_residual_and_exact_fixed_point():
    okf, gt_id, gt_n = _construction_i()
    st = oracle.new_state(gt_id, gt_n)
    oracle.optimize(okf, st, oracle.OracleParams(iters=3))
    assert np.array_equal(st["inv_depth"], gt_id)
    assert np.array_equal(np.stack([st["nx"], st["ny"], st["nz"]], 1), gt_n)
    ok_flags = (st["flags"] & oracle.SOLVE_FAIL) == 0
    assert np.all(st["cost"] == 0.0)
    assert ok_flags.mean() > 0.9   # only corner tiles with few in-bounds samples fail


def test_construction_i_converges_to_ground_truth():
    okf, gt_id, gt_n = _construction_i()
    rng = np.random.default_rng(0)
    m = gt_id.size
    init_id = gt_id * rng.uniform(0.97, 1.03, m)
    init_n = np.array([rot(np.cross(gt_n[0], rng.normal(size=3)),
                           math.radians(rng.uniform(0, 3))) @ gt_n[0] for _ in range(m)])
    st = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, st, oracle.OracleParams(iters=10))
    good = (st["flags"] & (oracle.SOLVE_FAIL | oracle.FEW_SAMPLES)) == 0
    n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert good.mean() > 0.9
    assert np.max(np.abs(st["inv_depth"][good] / gt_id[good] - 1)) < 1e-10
    assert np.max(angle_deg(n[good], gt_n[good])) < 1e-8


def _construction_ii(seed=5):
    """One neighbour, general plane and pose; the keyframe is synthesised
    from the neighbour through the plane homography with scipy's bilinear
    interpolation, so the ground-truth plane has zero residual."""
    W, H, S = 64, 48, 8
    K = (80.0, 80.0, 32.0, 24.0)
    rng = np.random.default_rng(seed)
    I1 = smooth_texture(W, H, 7, periods=(10, 30))
    n = random_unit_cap(rng, 30)
    p0 = ray(K, W / 2, H / 2) * 2.0
    d = float(n @ p0)
    R = rot(rng.normal(size=3), math.radians(1.5))
    t = 0.1 * rng.normal(size=3) / math.sqrt(3)
    Hm = plane_homography(K, R, t, n, d)
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    pts = Hm @ np.stack([X.ravel(), Y.ravel(), np.ones(X.size)])
    kfimg = bilinear_scipy_many(I1, pts[0] / pts[2], pts[1] / pts[2]).reshape(H, W)
    okf = oracle.OracleKeyframe(K, kfimg, I1[None], R[None], t[None], S)
    gw, gh = W // S, H // S
    ids = np.array([(n @ ray(K, S * tx + (S - 1) / 2, S * ty + (S - 1) / 2)) / d
                    for ty in range(gh) for tx in range(gw)])
    return okf, ids, np.tile(n, (ids.size, 1)), rng


def test_construction_ii_fixed_point_and_convergence():
    okf, ids, ns, rng = _construction_ii()
    st = oracle.new_state(ids, ns)
    oracle.optimize(okf, st, oracle.OracleParams(iters=3))
    n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert np.max(np.abs(st["inv_depth"] / ids - 1)) < 1e-12
    assert np.max(angle_deg(n, ns)) < 1e-9
    assert st["cost"].max() < 1e-24
    init_id = ids * rng.uniform(0.97, 1.03, ids.size)
    init_n = np.array([rot(np.cross(ns[0], rng.normal(size=3)),
                           math.radians(rng.uniform(0, 3))) @ ns[0] for _ in range(ids.size)])
    st = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, st, oracle.OracleParams(iters=10))
    n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert np.max(np.abs(st["inv_depth"] / ids - 1)) < 1e-10
    assert np.max(angle_deg(n, ns)) < 1e-8


def test_no_parallax_gives_zero_jacobian_and_solve_failure():
    okf, gt_id, gt_n = _construction_i()
    img = okf._kf_arr
    z = oracle.OracleKeyframe((128.0, 128.0, 24.0, 20.0), img, np.stack([img, img]),
                              np.stack([np.eye(3)] * 2), np.zeros((2, 3)), 4)
    st = oracle.new_state(gt_id * 1.05, gt_n)
    before = st["inv_depth"].copy()
    oracle.optimize(z, st, oracle.OracleParams(iters=2))
    assert np.all(st["flags"] & oracle.SOLVE_FAIL)
    assert np.array_equal(st["inv_depth"], before)
    H, b, cost, nv = oracle.linearize(z, 3, 3, 0.5, [0, 0, -1.0])
    assert np.all(H == 0) and np.all(b == 0) and nv == 32


def test_degenerate_plane_through_camera_centre():
    okf, gt_id, gt_n = _construction_i()
    m = gt_id.size
    K = (128.0, 128.0, 24.0, 20.0)
    # normal orthogonal to the ray of surfel 7 -> flagged, state untouched
    gw = 12
    tx, ty = 7 % gw, 7 // gw
    rs = ray(K, 4 * tx + 1.5, 4 * ty + 1.5)
    nd = np.cross(rs, [0.0, 1.0, 0.0])
    nd /= np.linalg.norm(nd)
    ns = gt_n.copy()
    ns[7] = nd
    st = oracle.new_state(gt_id, ns)
    oracle.optimize(okf, st, oracle.OracleParams(iters=2))
    assert st["flags"][7] & oracle.DEGENERATE
    assert st["inv_depth"][7] == 0.5 and st["nvalid"][7] == 0
    assert not np.any(st["flags"][np.arange(m) != 7] & oracle.DEGENERATE)


def test_few_samples_when_warp_leaves_the_image():
    okf, gt_id, gt_n = _construction_i()
    m = gt_id.size
    st = oracle.new_state(np.full(m, 50.0), gt_n)    # huge parallax: every sample out of bounds
    oracle.optimize(okf, st, oracle.OracleParams(iters=1))
    assert np.all(st["flags"] & oracle.FEW_SAMPLES)
    assert np.all(st["inv_depth"] == 50.0)


# --- Huber weighting (Eq. 5, Eq. 8) -----------------------------------------

def test_huber_weight_and_cost_single_pixel_surfels():
    """With 1x1 surfels and one neighbour, each surfel holds one sample:
    H = w J J^T and b = w J r with w = min(1, k/|r|), cost = huber(r)."""
    okf, gt_id, gt_n = _construction_i(S=1, W=24, H=20)
    k = 0.004
    rng = np.random.default_rng(12)
    hits = {"in": 0, "out": 0}
    for _ in range(200):
        tx, ty = rng.integers(2, 14), rng.integers(2, 12)
        ids = 0.5 * rng.uniform(0.6, 1.4)
        n = np.array([0.0, 0.0, -1.0])
        H, b, cost, nv = oracle.linearize(okf, tx, ty, ids, n, huber_k=k)
        # one neighbour at a time
        tot_H = np.zeros((3, 3)); tot_b = np.zeros(3); tot_c = 0.0
        for f in range(2):
            R = np.array(okf._poses[f].R[:]).reshape(3, 3)
            t = np.array(okf._poses[f].t[:])
            ok, r, J = oracle.eval_sample((128.0, 128.0, 24.0, 20.0), R, t, okf._nbr_arrs[f],
                                          okf._kf_arr[ty, tx], (tx, ty), (tx, ty), ids, n)
            if not ok:
                continue
            w = 1.0 if abs(r) <= k else k / abs(r)
            hits["in" if abs(r) <= k else "out"] += 1
            tot_H += w * np.outer(J, J)
            tot_b += w * J * r
            tot_c += huber(r, k)
        assert np.allclose(H, tot_H, rtol=1e-12, atol=1e-300)
        assert np.allclose(b, tot_b, rtol=1e-12, atol=1e-300)
        assert cost == pytest.approx(tot_c, rel=1e-12, abs=1e-300)
    assert hits["in"] > 10 and hits["out"] > 10


def test_huber_weight_of_a_nan_residual_is_one():
    """A keyframe pixel that is not a number: with 1x1 surfels its surfel's
    samples have NaN residuals and weight 1, so J^T W J is the unweighted
    sum of J J^T (finite) while J^T W r and the cost are NaN."""
    okf, gt_id, gt_n = _construction_i(S=1, W=24, H=20)
    tx, ty = 7, 6
    okf._kf_arr[ty, tx] = np.nan
    ids = 0.45
    n = np.array([0.0, 0.0, -1.0])
    H, b, cost, nv = oracle.linearize(okf, tx, ty, ids, n, huber_k=0.004)
    tot_H = np.zeros((3, 3))
    for f in range(2):
        R = np.array(okf._poses[f].R[:]).reshape(3, 3)
        t = np.array(okf._poses[f].t[:])
        ok, r, J = oracle.eval_sample((128.0, 128.0, 24.0, 20.0), R, t, okf._nbr_arrs[f],
                                      okf._kf_arr[ty, tx], (tx, ty), (tx, ty), ids, n)
        if ok:
            assert np.isnan(r)
            tot_H += np.outer(J, J)
    assert nv >= 1 and np.all(np.isfinite(H))
    assert np.allclose(H, tot_H, rtol=1e-12, atol=1e-300)
    assert np.all(np.isnan(b)) and np.isnan(cost)


def _bilinear_grad(img, u, v):
    """Bilinear value and exact gradient of the interpolant at (u, v) (arrays),
    written out directly for the cross-check below."""
    x0 = np.floor(u).astype(int)
    y0 = np.floor(v).astype(int)
    ax, ay = u - x0, v - y0
    x0 = np.clip(x0, 0, img.shape[1] - 2)
    y0 = np.clip(y0, 0, img.shape[0] - 2)
    i00, i01 = img[y0, x0], img[y0, x0 + 1]
    i10, i11 = img[y0 + 1, x0], img[y0 + 1, x0 + 1]
    top = i00 + ax * (i01 - i00)
    bot = i10 + ax * (i11 - i10)
    return top + ay * (bot - top), (i01 - i00) + ay * ((i11 - i10) - (i01 - i00)), bot - top


def _fit_affine_inverse_depth(K, kfimg, nbrs, Rs, ts, S, tx, ty, p, k, iters):
    """Gauss-Newton with Huber IRLS weights on the same cost (Eq. 5), with the
    surfel written as an affine inverse-depth map id_u = a + b dx + c dy
    (dx, dy: pixel offsets from the centre) instead of (id_s, normal); the
    warp's derivative in id_u by central differences."""
    fx, fy, cx, cy = K
    H, W = kfimg.shape
    ys, xs = np.mgrid[S * ty:S * ty + S, S * tx:S * tx + S]
    xs = xs.ravel().astype(np.float64)
    ys = ys.ravel().astype(np.float64)
    dx, dy = xs - (S * tx + (S - 1) / 2), ys - (S * ty + (S - 1) / 2)
    r_u = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)])
    ikf = kfimg[ys.astype(int), xs.astype(int)]
    p = np.array(p, np.float64)

    def warp(f, idv):
        Xn = Rs[f] @ (r_u / idv) + ts[f][:, None]
        return fx * Xn[0] / Xn[2] + cx, fy * Xn[1] / Xn[2] + cy, Xn[2]

    for _ in range(iters):
        idu = p[0] + p[1] * dx + p[2] * dy
        A = np.zeros((3, 3))
        g = np.zeros(3)
        for f in range(len(nbrs)):
            u, v, z = warp(f, idu)
            h = 1e-6 * idu
            up, vp, _ = warp(f, idu + h)
            um, vm, _ = warp(f, idu - h)
            ok = (idu > 0) & (z > 0) & (u >= 0) & (u < W - 1) & (v >= 0) & (v < H - 1)
            val, gx, gy = _bilinear_grad(nbrs[f], u, v)
            r = val - ikf
            w = np.minimum(1.0, k / np.abs(r))
            jd = gx * (up - um) / (2 * h) + gy * (vp - vm) / (2 * h)
            J = np.stack([jd, jd * dx, jd * dy])[:, ok]
            A += (J * w[ok]) @ J.T
            g += (J * w[ok]) @ r[ok]
        p = p - np.linalg.solve(A, g)
    return p


def test_affine_inverse_depth_cross_check():
    """The oracle's Gauss-Newton in (id_s, tangent normal step) and an
    independent one in the affine inverse-depth parameterisation (a plane's
    inverse depth is affine in the pixel, Eq. 3) converge to the same plane
    on noisy three-frame scenes: a pin of the whole linearise-solve-update
    path, Jacobian and Huber weights included."""
    W, H, S = 96, 64, 16
    K = (90.0, 90.0, 48.0, 32.0)
    rng = np.random.default_rng(21)
    kfimg = smooth_texture(W, H, 17, periods=(9, 30))
    n_gt = random_unit_cap(rng, 30)
    d = float(n_gt @ (ray(K, W / 2, H / 2) * 2.0))
    Rs, ts, nbrs = [], [], []
    Y, X = np.mgrid[0:H, 0:W].astype(np.float64)
    for f in range(3):
        R = rot(rng.normal(size=3), math.radians(1.5))
        t = 0.12 * rng.normal(size=3) / math.sqrt(3)
        Hinv = np.linalg.inv(plane_homography(K, R, t, n_gt, d))
        pts = Hinv @ np.stack([X.ravel(), Y.ravel(), np.ones(X.size)])
        img = bilinear_scipy_many(kfimg, pts[0] / pts[2], pts[1] / pts[2]).reshape(H, W)
        nbrs.append(img + rng.normal(0.0, 0.01, size=img.shape))
        Rs.append(R)
        ts.append(t)
    Rs, ts, nbrs = np.stack(Rs), np.stack(ts), np.stack(nbrs)
    okf = oracle.OracleKeyframe(K, kfimg, nbrs, Rs, ts, S)
    gw, gh = W // S, H // S
    fx, fy, cx, cy = K
    k = 9.0 / 255.0
    checked = 0
    for ty in range(1, gh - 1):
        for tx in range(1, gw - 1):
            rs = ray(K, S * tx + (S - 1) / 2, S * ty + (S - 1) / 2)
            id0 = float(n_gt @ rs) / d * 1.02
            n0 = rot(np.cross(n_gt, rng.normal(size=3)), math.radians(2.0)) @ n_gt
            full = oracle.new_state(np.full(gw * gh, id0), np.tile(n0, (gw * gh, 1)))
            oracle.optimize(okf, full, oracle.OracleParams(iters=40, huber_k=k))
            i = ty * gw + tx
            assert full["flags"][i] == 0
            id1 = full["inv_depth"][i]
            n1 = np.array([full["nx"][i], full["ny"][i], full["nz"][i]])
            # the same start in the affine form: id_u = id_s (n . r_u) / (n . r_s)
            c0 = float(n0 @ rs)
            p0 = (id0, id0 * n0[0] / (fx * c0), id0 * n0[1] / (fy * c0))
            a, b, c = _fit_affine_inverse_depth(K, kfimg, nbrs, Rs, ts, S, tx, ty, p0, k, 40)
            # id_u = alpha . r_u: alpha is the plane's normal over its distance
            alpha = np.array([b * fx, c * fy, a - b * fx * rs[0] - c * fy * rs[1]])
            assert a == pytest.approx(id1, rel=1e-8)
            assert angle_deg(alpha / np.linalg.norm(alpha), n1)[0] < 1e-5
            # both moved off the start (2 % in depth, 2 degrees in the normal)
            # to the noisy images' minimum, close to the true depth
            assert abs(id1 / id0 - 1) > 1e-3 and angle_deg(n1, n0)[0] > 1e-2
            assert abs(id1 * d / float(n_gt @ rs) - 1) < 3e-2
            checked += 1
    assert checked == (gw - 2) * (gh - 2)


# --- 3x3 solve and conditioning ---------------------------------------------

def test_solve3_matches_numpy_on_spd_matrices():
    rng = np.random.default_rng(13)
    for _ in range(400):
        cond = 10 ** rng.uniform(0, 10)
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        ev = np.array([1.0, cond ** 0.5, cond]) * 10 ** rng.uniform(-4, 4)
        Hm = Q @ np.diag(ev) @ Q.T
        Hm = 0.5 * (Hm + Hm.T)
        b = rng.normal(size=3)
        st, d = oracle.solve3(Hm, b)
        assert st == 0
        ref = np.linalg.solve(Hm, -b)
        assert np.linalg.norm(d - ref) <= 1e-13 * cond * np.linalg.norm(ref) + 1e-300


def test_solve3_rejects_non_positive_definite():
    assert oracle.solve3(np.diag([1.0, -1.0, 1.0]), np.ones(3))[0] == oracle.SOLVE_FAIL
    assert oracle.solve3(np.zeros((3, 3)), np.ones(3))[0] == oracle.SOLVE_FAIL
    v = np.array([1.0, 2.0, 3.0])
    assert oracle.solve3(np.outer(v, v), np.ones(3))[0] == oracle.SOLVE_FAIL
    assert oracle.solve3(np.diag([1.0, 1.0, np.nan]), np.ones(3))[0] == oracle.SOLVE_FAIL


def test_kappa_eq_matches_numpy_condition_number():
    rng = np.random.default_rng(14)
    for _ in range(200):
        A = rng.normal(size=(5, 3)) * rng.uniform(0.01, 100, size=3)
        Hm = A.T @ A
        D = np.diag(1 / np.sqrt(np.diag(Hm)))
        ref = np.linalg.cond(D @ Hm @ D)
        assert oracle.kappa_eq(Hm) == pytest.approx(ref, rel=1e-9)
    assert oracle.kappa_eq(np.diag([1.0, 0.0, 2.0])) == float("inf")


# --- cost minimum: GN result against a brute-force search -------------------

def test_gauss_newton_reaches_the_brute_force_minimum():
    """On a small noisy patch the GN result is the minimum of the Huber cost
    of Eq. 5 over a dense grid of (id, two tilt angles) around it.  The cost
    is evaluated here independently (plane homography + scipy bilinear +
    Huber), not with the oracle's own cost routine."""
    okf, ids, ns, rng = _construction_ii(seed=21)
    # add noise to the keyframe so that the minimum is not exactly at GT
    noisy = okf._kf_arr + np.random.default_rng(22).normal(0, 2 / 255, okf._kf_arr.shape)
    K = (80.0, 80.0, 32.0, 24.0)
    R = np.array(okf._poses[0].R[:]).reshape(3, 3)
    t = np.array(okf._poses[0].t[:])
    okn = oracle.OracleKeyframe(K, noisy, okf._nbr_arrs[0][None], R[None], t[None], 8)
    k = 9 / 255
    tx, ty = 3, 2
    i = ty * 8 + tx
    st = oracle.new_state(ids * 1.02, ns)
    oracle.optimize(okn, st, oracle.OracleParams(iters=15, huber_k=k), subset=[i])
    id_gn = st["inv_depth"][i]
    n_gn = np.array([st["nx"][i], st["ny"][i], st["nz"][i]])
    us = (8 * tx + 3.5, 8 * ty + 3.5)
    I1 = okf._nbr_arrs[0]
    pix = [(8 * tx + px, 8 * ty + py) for py in range(8) for px in range(8)]

    def cost(id_s, n):
        ps = ray(K, *us) / id_s
        Hm = plane_homography(K, R, t, n, float(n @ ps))
        c = 0.0
        for (x, y) in pix:
            xp, yp = apply_h(Hm, x, y)
            assert 0 <= xp < 63 and 0 <= yp < 47
            c += huber(bilinear_scipy(I1, xp, yp) - noisy[y, x], k)
        return c

    assert cost(id_gn, n_gn) == pytest.approx(st["cost"][i], rel=1e-9)
    b1, b2 = oracle.tangent_basis(n_gn)
    c_gn = cost(id_gn, n_gn)
    span_id, span_a, m = 0.004, math.radians(1.5), 7
    best = (np.inf, None)
    for a in np.linspace(-1, 1, m):
        for b_ in np.linspace(-1, 1, m):
            for c_ in np.linspace(-1, 1, m):
                nn = n_gn + math.tan(b_ * span_a) * b1 + math.tan(c_ * span_a) * b2
                nn /= np.linalg.norm(nn)
                v = cost(id_gn * (1 + a * span_id), nn)
                if v < best[0]:
                    best = (v, (a, b_, c_))
    assert c_gn <= best[0] * (1 + 1e-9)
    assert best[1] == (0.0, 0.0, 0.0)


def test_costs_at_matches_an_independent_cost():
    """The cost evaluator the parity tests use to judge end points (Huber cost
    of Eq. 5 at given states, tiles and discs) against the plane homography,
    scipy's bilinear interpolation and the Huber norm, on several surfels
    and perturbed states at once."""
    okf, ids, ns, rng = _construction_ii(seed=41)
    noisy = okf._kf_arr + np.random.default_rng(42).normal(0, 2 / 255, okf._kf_arr.shape)
    K = (80.0, 80.0, 32.0, 24.0)
    R = np.array(okf._poses[0].R[:]).reshape(3, 3)
    t = np.array(okf._poses[0].t[:])
    okn = oracle.OracleKeyframe(K, noisy, okf._nbr_arrs[0][None], R[None], t[None], 8)
    k = 9 / 255
    I1 = okf._nbr_arrs[0]
    H_, W_ = noisy.shape
    idv = ids * rng.uniform(0.97, 1.03, ids.size)
    nv = np.array([rot(np.cross(n, rng.normal(size=3)), math.radians(rng.uniform(0, 4))) @ n for n in ns])
    pick = np.array([3, 10, 11, 18, 20, 26], np.int32)
    ux = np.array([8 * (i % 8) + 3.5 + rng.uniform(-2, 2) for i in range(ids.size)])
    uy = np.array([8 * (i // 8) + 3.5 + rng.uniform(-2, 2) for i in range(ids.size)])

    def cost(us, id_s, n, pix):
        ps = ray(K, *us) / id_s
        Hm = plane_homography(K, R, t, n, float(n @ ps))
        c, v = 0.0, 0
        for (x, y) in pix:
            xp, yp = apply_h(Hm, x, y)
            if 0 <= xp < W_ - 1 and 0 <= yp < H_ - 1:
                c += huber(bilinear_scipy(I1, xp, yp) - noisy[y, x], k)
                v += 1
        return c, v

    got, gnv = oracle.costs_at(okn, idv, nv, pick, k)
    dgot, dnv = oracle.costs_at(okn, idv, nv, pick, k, disc=(ux, uy, 5.5))
    for j, i in enumerate(pick):
        tx, ty = i % 8, i // 8
        tile = [(8 * tx + px, 8 * ty + py) for py in range(8) for px in range(8)]
        c, v = cost((8 * tx + 3.5, 8 * ty + 3.5), idv[i], nv[i], tile)
        assert got[j] == pytest.approx(c, rel=1e-9) and gnv[j] == v
        disc = [(x, y) for y in range(H_) for x in range(W_) if (x - ux[i]) ** 2 + (y - uy[i]) ** 2 < 5.5 ** 2]
        c, v = cost((ux[i], uy[i]), idv[i], nv[i], disc)
        assert dgot[j] == pytest.approx(c, rel=1e-9) and dnv[j] == v


# --- depth-only ablation ------------------------------------------------------

def test_depth_only_matches_one_dimensional_search():
    okf, ids, ns, rng = _construction_ii(seed=23)
    tilt = rot(np.cross(ns[0], [1.0, 0, 0]), math.radians(4.0)) @ ns[0]
    i = 2 * 8 + 3
    st = oracle.new_state(ids * 1.03, np.tile(tilt, (ids.size, 1)))
    oracle.optimize(okf, st, oracle.OracleParams(iters=25, depth_only=True), subset=[i])
    assert np.allclose([st["nx"][i], st["ny"][i], st["nz"][i]], tilt, atol=1e-15)
    # golden-section search of the oracle-independent cost along id only
    K = (80.0, 80.0, 32.0, 24.0)
    R = np.array(okf._poses[0].R[:]).reshape(3, 3)
    t = np.array(okf._poses[0].t[:])
    I1 = okf._nbr_arrs[0]
    us = (8 * 3 + 3.5, 8 * 2 + 3.5)

    def cost(id_s):
        ps = ray(K, *us) / id_s
        Hm = plane_homography(K, R, t, tilt, float(tilt @ ps))
        c = 0.0
        for py in range(8):
            for px in range(8):
                x, y = 8 * 3 + px, 8 * 2 + py
                xp, yp = apply_h(Hm, x, y)
                c += huber(bilinear_scipy(I1, xp, yp) - okf._kf_arr[y, x], 9 / 255)
        return c

    lo, hi = ids[i] * 0.9, ids[i] * 1.1
    g = (math.sqrt(5) - 1) / 2
    a, b = hi - g * (hi - lo), lo + g * (hi - lo)
    fa, fb = cost(a), cost(b)
    for _ in range(80):
        if fa < fb:
            hi, b, fb = b, a, fa
            a = hi - g * (hi - lo)
            fa = cost(a)
        else:
            lo, a, fa = a, b, fb
            b = lo + g * (hi - lo)
            fb = cost(b)
    assert st["inv_depth"][i] == pytest.approx(0.5 * (lo + hi), rel=2e-6)


# --- neighbour-plane initialisation ----------------------------------------

def _planar_keyframe(S=4, W=64, H=48):
    K = (90.0, 92.0, 31.0, 25.0)
    img = np.zeros((H, W))
    okf = oracle.OracleKeyframe(K, img, np.zeros((0, H, W)), np.zeros((0, 3, 3)), np.zeros((0, 3)), S)
    return okf, K


def test_init_is_exact_on_a_globally_planar_scene():
    """A new surfel surrounded by surfels of one plane gets that plane."""
    S = 4
    okf, K = _planar_keyframe(S)
    gw, gh = okf.grid
    n = np.array([0.2, -0.3, -0.9])
    n /= np.linalg.norm(n)
    d = -1.7
    ids = np.array([(n @ ray(K, S * tx + 1.5, S * ty + 1.5)) / d for ty in range(gh) for tx in range(gw)])
    yy, xx = np.mgrid[0:gh, 0:gw]
    is_new = ((xx + yy) % 2 == 1).astype(np.uint8).ravel()
    init_id = np.where(is_new == 1, 0.123, ids)
    init_n = np.tile(n, (ids.size, 1))
    init_n[is_new == 1] = [0.0, 0.0, -1.0]
    # flip the sign of some old normals: the mean must sign-align them
    flip = (np.arange(ids.size) % 3 == 0) & (is_new == 0)
    init_n[flip] *= -1
    st = oracle.new_state(init_id, init_n)
    oracle.init_from_neighbours(okf, st, is_new, oracle.OracleParams())
    new = is_new == 1
    got_n = np.stack([st["nx"], st["ny"], st["nz"]], 1)[new]
    assert np.max(np.abs(st["inv_depth"][new] / ids[new] - 1)) < 1e-12
    assert np.max(angle_deg(got_n, np.tile(n, (new.sum(), 1)))) < 1e-9
    assert not np.any(st["flags"] & oracle.UNINIT)
    # old surfels are untouched
    assert np.array_equal(st["inv_depth"][~new], ids[~new])


def test_init_neighbour_set_follows_the_pixel_distance_rule():
    """Checkerboard: the 4-connected tiles; a lone new tile: all 8 tiles
    around it (their nearest pixels are within S of its centre); a wider
    beta r adds the next ring only where a pixel lies closer than it."""
    S = 4
    okf, K = _planar_keyframe(S, 40, 40)
    gw, gh = okf.grid
    m = gw * gh
    rng = np.random.default_rng(31)
    ids = rng.uniform(0.3, 0.6, m)
    ns = np.tile([0.0, 0.0, -1.0], (m, 1))     # fronto-parallel: Eq. 3 gives id_j back
    c = 4 * gw + 4
    lone = np.zeros(m, np.uint8)
    lone[c] = 1
    st = oracle.new_state(ids, ns)
    oracle.init_from_neighbours(okf, st, lone, oracle.OracleParams())
    ring = [(4 + dx) + gw * (4 + dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy) != (0, 0)]
    assert st["inv_depth"][c] == pytest.approx(ids[ring].mean(), rel=1e-14)
    # checkerboard
    yy, xx = np.mgrid[0:gh, 0:gw]
    cb = ((xx + yy) % 2 == 1).astype(np.uint8).ravel()
    c2 = 4 * gw + 5
    st = oracle.new_state(ids, ns)
    oracle.init_from_neighbours(okf, st, cb, oracle.OracleParams())
    four = [c2 - 1, c2 + 1, c2 - gw, c2 + gw]
    assert st["inv_depth"][c2] == pytest.approx(ids[four].mean(), rel=1e-14)
    # corner of the grid: only in-grid neighbours
    st = oracle.new_state(ids, ns)
    corner = np.zeros(m, np.uint8)
    corner[0] = 1
    oracle.init_from_neighbours(okf, st, corner, oracle.OracleParams())
    assert st["inv_depth"][0] == pytest.approx(ids[[1, gw, gw + 1]].mean(), rel=1e-14)
    # a wider beta r (1.8 S) reaches tiles two steps away; the expected set
    # comes from an explicit pixel-distance computation
    br = 1.8 * S
    st = oracle.new_state(ids, ns)
    oracle.init_from_neighbours(okf, st, lone, oracle.OracleParams(beta_r=br))
    ux = uy = 4 * S + 1.5
    sel = []
    for ty in range(gh):
        for tx in range(gw):
            j = ty * gw + tx
            if j == c:
                continue
            dmin = min(math.hypot(S * tx + px - ux, S * ty + py - uy) for px in range(S) for py in range(S))
            if dmin < br:
                sel.append(j)
    assert len(sel) > 8
    assert st["inv_depth"][c] == pytest.approx(ids[sel].mean(), rel=1e-13)


def test_init_without_neighbours_flags_uninit():
    S = 4
    okf, K = _planar_keyframe(S, 16, 16)
    m = 16
    st = oracle.new_state(np.full(m, 0.4), np.tile([0.0, 0.0, -1.0], (m, 1)))
    oracle.init_from_neighbours(okf, st, np.ones(m, np.uint8), oracle.OracleParams())
    assert np.all(st["flags"] & oracle.UNINIT)
    assert np.all(st["inv_depth"] == 0.4)


# --- render (per-pixel inverse depth) ---------------------------------------

def test_render_matches_eq3_per_pixel():
    okf, ids, ns, rng = _construction_ii()
    st = oracle.new_state(ids, ns)
    st["flags"][5] = oracle.UNINIT
    idm, ind = oracle.render(okf, st)
    K = (80.0, 80.0, 32.0, 24.0)
    for _ in range(200):
        x, y = rng.integers(0, 64), rng.integers(0, 48)
        i = (y // 8) * 8 + x // 8
        if i == 5:
            assert idm[y, x] == 0.0 and ind[y, x] == -1
            continue
        ps = ray(K, 8 * (x // 8) + 3.5, 8 * (y // 8) + 3.5) / ids[i]
        # ray / plane intersection by a 3x3 solve: lam r_u = ps + s a + q b
        a = np.cross(ns[i], [0.3, 0.5, 0.7])
        b = np.cross(ns[i], a)
        lam = np.linalg.solve(np.stack([ray(K, x, y), -a, -b], 1), ps)[0]
        expect = 1.0 / lam
        assert idm[y, x] == pytest.approx(expect, rel=1e-13)
        assert ind[y, x] == i


# --- Eq. 10 (reference-frame change) ---------------------------------------

def test_transfer_round_trip_and_plane_consistency():
    rng = np.random.default_rng(41)
    K = (300.0, 300.0, 160.0, 120.0)
    R = rot(rng.normal(size=3), math.radians(4))
    t = rng.normal(size=3) * 0.1
    m = 50
    us = np.stack([rng.uniform(0, 320, m), rng.uniform(0, 240, m)], 1)
    ids = rng.uniform(0.3, 1.0, m)
    ns = np.array([random_unit_cap(rng, 40) for _ in range(m)])
    u1, id1, n1 = oracle.transfer(K, R, t, us, ids, ns)
    u0, id0, n0 = oracle.transfer(K, R.T, -R.T @ t, u1, id1, n1)
    assert np.allclose(u0, us, atol=1e-9) and np.allclose(id0, ids, rtol=1e-12)
    assert np.allclose(n0, ns, atol=1e-14)
    # another point of each original plane, moved by the pose, lies on the
    # transferred plane as described by Eq. 3 in the new frame
    for k in range(m):
        ps = ray(K, *us[k]) / ids[k]
        off = np.cross(ns[k], [0.1, 0.2, 0.3])
        q0 = ps + 0.05 * off / np.linalg.norm(off)
        q1 = R @ q0 + t
        u_new = (K[0] * q1[0] / q1[2] + K[2], K[1] * q1[1] / q1[2] + K[3])
        got = oracle.pixel_inverse_depth(K, u1[k], id1[k], n1[k], u_new)
        assert got == pytest.approx(1.0 / q1[2], rel=1e-10)


def _grid_state(gw, gh, ids, normals, flags=None):
    return oracle.new_state(np.asarray(ids, np.float64).reshape(-1),
                            np.asarray(normals, np.float64).reshape(-1, 3), flags)


def test_regrid_identity_pose_keeps_every_usable_surfel_in_its_tile():
    rng = np.random.default_rng(43)
    K, W, H, S = (200.0, 210.0, 80.0, 60.0), 160, 120, 4
    gw, gh = W // S, H // S
    m = gw * gh
    ids = rng.uniform(0.25, 1.0, m)
    ns = np.array([random_unit_cap(rng, 40) for _ in range(m)])
    flags = np.zeros(m, np.uint32)
    flags[rng.choice(m, 30, replace=False)] = oracle.DEGENERATE
    flags[rng.choice(m, 30, replace=False)] |= oracle.UNINIT
    st = _grid_state(gw, gh, ids, ns, flags)
    st["last_update"][:] = np.arange(m, dtype=np.uint32) + 7
    out, is_new, win, filled = oracle.transfer_regrid((K, W, H, S), st, np.eye(3), np.zeros(3),
                                                      (K, W, H, S))
    usable = (flags & (oracle.DEGENERATE | oracle.UNINIT)) == 0
    assert filled == usable.sum()
    assert np.array_equal(win.reshape(-1), np.where(usable, np.arange(m), -1))
    assert np.array_equal(is_new.reshape(-1), (~usable).astype(np.uint8))
    assert np.allclose(out["inv_depth"][usable], ids[usable], rtol=1e-13)
    got_n = np.stack([out["nx"], out["ny"], out["nz"]], 1)
    assert np.allclose(got_n[usable], ns[usable], atol=1e-14)
    assert np.all(out["flags"][~usable] == oracle.UNINIT) and np.all(out["inv_depth"][~usable] == 0)
    assert np.array_equal(out["last_update"][usable], st["last_update"][usable])


@pytest.mark.parametrize("S,k", [(4, 1), (4, 3), (8, 2)])
def test_regrid_sideways_motion_shifts_a_wall_by_whole_tiles(S, k):
    """A fronto-parallel wall at depth d and a sideways camera motion of
    S k d / fx move every surfel by exactly k tiles (pinhole geometry)."""
    K, W, H = (180.0, 180.0, 81.0, 59.0), 128, 96
    gw, gh = W // S, H // S
    d = 2.5
    st = _grid_state(gw, gh, np.full(gw * gh, 1 / d), np.tile([0.0, 0.0, -1.0], (gw * gh, 1)))
    t = np.array([-S * k * d / K[0], 0.0, 0.0])
    out, is_new, win, filled = oracle.transfer_regrid((K, W, H, S), st, np.eye(3), t, (K, W, H, S))
    idx = np.arange(gw * gh).reshape(gh, gw)
    expect = np.full((gh, gw), -1)
    expect[:, :gw - k] = idx[:, k:]
    assert np.array_equal(win, expect)
    assert np.array_equal(is_new, (expect < 0).astype(np.uint8))
    filled_mask = (expect >= 0).reshape(-1)
    assert np.allclose(out["inv_depth"][filled_mask], 1 / d, rtol=1e-13)
    assert np.allclose(out["nz"][filled_mask], -1.0, atol=1e-15)


def test_regrid_occlusion_keeps_the_closer_surface():
    """Near wall (left half, depth 1) and far wall (right half, depth 4);
    moving the camera sideways slides the near wall over the far one by
    integer tile counts (8 and 2 tiles): where both land the near one wins."""
    K, W, H, S = (160.0, 160.0, 95.5, 31.5), 192, 64, 4
    gw, gh = W // S, H // S
    ids = np.where(np.arange(gw) < gw // 2, 1.0, 0.25)
    st = _grid_state(gw, gh, np.tile(ids, gh), np.tile([0.0, 0.0, -1.0], (gw * gh, 1)))
    t = np.array([8 * S / K[0], 0.0, 0.0])          # shift = fx t_x id pixels
    out, is_new, win, filled = oracle.transfer_regrid((K, W, H, S), st, np.eye(3), t, (K, W, H, S))
    expect = np.full(gw, -1)
    for tx in range(gw):                              # brute force over sources, far first
        shift = 2 if tx >= gw // 2 else 8
        if tx + shift < gw and (expect[tx + shift] < 0 or ids[tx] > ids[expect[tx + shift]]):
            expect[tx + shift] = tx
    for ty in range(gh):
        want = np.where(expect >= 0, expect + ty * gw, -1)
        assert np.array_equal(win[ty], want)
    near_won = (expect >= 0) & (expect < gw // 2)
    assert near_won[gw // 2 + 2: gw // 2 + 8].all()   # overlapped columns
    assert np.allclose(out["inv_depth"].reshape(gh, gw)[:, expect >= 0],
                       np.tile(ids[expect[expect >= 0]], (gh, 1)), rtol=1e-13)


def test_regrid_tilted_planes_against_ray_plane_solve_and_brute_force_ztest():
    rng = np.random.default_rng(47)
    K0, K1 = (220.0, 230.0, 78.0, 62.0), (250.0, 240.0, 90.0, 55.0)
    W0, H0, S0 = 160, 120, 4
    W1, H1, S1 = 176, 112, 8
    gw0, gh0 = W0 // S0, H0 // S0
    gw1, gh1 = W1 // S1, H1 // S1
    m = gw0 * gh0
    ids = rng.uniform(0.3, 0.9, m)
    ns = np.array([random_unit_cap(rng, 35) for _ in range(m)])
    st = _grid_state(gw0, gh0, ids, ns)
    R = rot(rng.normal(size=3), math.radians(3))
    t = np.array([0.04, -0.03, -0.08])
    out, is_new, win, filled = oracle.transfer_regrid((K0, W0, H0, S0), st, R, t, (K1, W1, H1, S1))
    # landing of every source surfel by explicit projection
    best = {}
    for i in range(m):
        us = (S0 * (i % gw0) + 0.5 * (S0 - 1), S0 * (i // gw0) + 0.5 * (S0 - 1))
        p1 = R @ (ray(K0, *us) / ids[i]) + t
        if p1[2] <= 0:
            continue
        px = math.floor(K1[0] * p1[0] / p1[2] + K1[2] + 0.5)
        py = math.floor(K1[1] * p1[1] / p1[2] + K1[3] + 0.5)
        if not (0 <= px < gw1 * S1 and 0 <= py < gh1 * S1):
            continue
        j = (py // S1) * gw1 + px // S1
        if j not in best or 1 / p1[2] > best[j][0]:
            best[j] = (1 / p1[2], i, p1)
    assert filled > 0.5 * gw1 * gh1
    for j in range(gw1 * gh1):
        if j not in best:
            assert win.reshape(-1)[j] == -1 and is_new.reshape(-1)[j] == 1
            continue
        _, i, p1 = best[j]
        assert win.reshape(-1)[j] == i
        # the moved plane through p1 with normal R n, cut by the tile's centre ray
        nn = R @ ns[i]
        a = np.cross(nn, [0.3, -0.2, 0.9]); a /= np.linalg.norm(a)
        b = np.cross(nn, a)
        rt = ray(K1, S1 * (j % gw1) + 0.5 * (S1 - 1), S1 * (j // gw1) + 0.5 * (S1 - 1))
        lam = np.linalg.solve(np.stack([rt, -a, -b], 1), p1)[0]
        assert out["inv_depth"][j] == pytest.approx(1 / lam, rel=1e-11)
        got_n = np.array([out["nx"][j], out["ny"][j], out["nz"][j]])
        assert np.allclose(got_n, nn, atol=1e-13)


# --- Levenberg-Marquardt variant ---------------------------------------------

def test_levenberg_marquardt_never_increases_mean_cost_and_reaches_gn_point():
    okf, ids, ns, rng = _construction_ii(seed=27)
    init_id = ids * rng.uniform(0.95, 1.05, ids.size)
    init_n = np.array([rot(np.cross(ns[0], rng.normal(size=3)),
                           math.radians(rng.uniform(0, 5))) @ ns[0] for _ in range(ids.size)])
    st = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, st, oracle.OracleParams(iters=40, lm_lambda=1e-2))
    n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert np.median(np.abs(st["inv_depth"] / ids - 1)) < 1e-8
    assert np.median(angle_deg(n, ns)) < 1e-6


def test_levenberg_marquardt_refuses_a_step_that_raises_the_mean_cost():
    """Find starting states where one Gauss-Newton step raises the mean Huber
    cost (judged by an independent evaluation of the cost at both states);
    from there the damped variant with a negligible lambda must keep the
    state, and plain Gauss-Newton must take the step."""
    okf, ids, ns, rng = _construction_ii(seed=31)
    gw = okf.grid[0]
    found = 0
    for trial in range(400):
        i = int(rng.integers(ids.size))
        id0 = ids[i] * rng.uniform(0.6, 1.5)
        n0 = rot(np.cross(ns[i], rng.normal(size=3)), math.radians(rng.uniform(5, 35))) @ ns[i]
        one = np.array([i], np.int32)
        st = oracle.new_state(np.full(ids.size, id0), np.tile(n0, (ids.size, 1)))
        oracle.optimize(okf, st, oracle.OracleParams(iters=1), subset=one)
        n1 = np.array([st["nx"][i], st["ny"][i], st["nz"][i]])
        if st["inv_depth"][i] == id0:
            continue
        _, _, c0, v0 = oracle.linearize(okf, i % gw, i // gw, id0, n0)
        _, _, c1, v1 = oracle.linearize(okf, i % gw, i // gw, st["inv_depth"][i], n1)
        if v1 < 3 or not (c1 / v1 > (c0 / v0) * (1 + 1e-4)):
            continue
        found += 1
        lm = oracle.new_state(np.full(ids.size, id0), np.tile(n0, (ids.size, 1)))
        oracle.optimize(okf, lm, oracle.OracleParams(iters=1, lm_lambda=1e-9), subset=one)
        assert lm["inv_depth"][i] == id0
        assert np.array_equal([lm["nx"][i], lm["ny"][i], lm["nz"][i]], n0)
        if found >= 3:
            break
    assert found >= 1, "no cost-raising Gauss-Newton step found"


@pytest.mark.parametrize("eps", [5e-5, -5e-5, 1e-6, -1e-6])
def test_levenberg_marquardt_accepts_exactly_when_the_mean_cost_does_not_rise(eps):
    """The damped variant takes a candidate when its mean Huber cost per valid
    sample does not rise, and refuses any rise.  On a keyframe built so that
    the one damped step changes the mean cost by the factor 1 + eps (checked
    here by an independent evaluation of the cost: the sideways warp
    x + fx t_x id, scipy's bilinear interpolation and the Huber norm), one
    iteration must refuse the step for eps > 0 (state kept, no stamp) and
    take it for eps < 0; plain Gauss-Newton takes it either way."""
    from tests import lm_construction as lc
    lam = 2.0 ** -20
    case = lc.build(eps, lam)
    gw = lc.W // lc.S
    tx, ty = lc.SURFEL % gw, lc.SURFEL // gw
    fxt = lc.K[0] * case["t"][0][0]

    def cost(id_s):
        tot, nv = 0.0, 0
        for y in range(ty * lc.S, ty * lc.S + lc.S):
            for x in range(tx * lc.S, tx * lc.S + lc.S):
                xp = x + fxt * id_s
                assert 0 <= xp < lc.W - 1
                for f in range(lc.N_FRAMES):
                    r = bilinear_scipy(case["nbrs"][f], xp, y) - case["kf"][y, x]
                    tot += huber(r, 9.0 / 255.0)
                    nv += 1
        return tot / nv

    ratio = cost(case["candidate_id"]) / cost(lc.ID0)
    assert ratio == pytest.approx(1.0 + eps, abs=1e-9)
    okf = oracle.OracleKeyframe(lc.K, case["kf"], case["nbrs"], case["R"], case["t"], lc.S)
    one = np.array([lc.SURFEL], np.int32)
    for lm_lambda in (lam, 0.0):
        st = oracle.new_state(case["init_id"], case["init_n"])
        oracle.optimize(okf, st, oracle.OracleParams(iters=1, depth_only=True, lm_lambda=lm_lambda,
                                                     stamp=7), subset=one)
        taken = lm_lambda == 0.0 or eps < 0
        i = lc.SURFEL
        if taken:
            want = case["candidate_id"] if lm_lambda > 0 else lc.ID0 + 0.5
            assert st["inv_depth"][i] == pytest.approx(want, rel=1e-12)
            assert st["last_update"][i] == 7
        else:
            assert st["inv_depth"][i] == lc.ID0
            assert st["last_update"][i] == 0
        assert st["nvalid"][i] == 48
        assert st["flags"][i] == 0


# --- conditioning probe (test facility) --------------------------------------

def test_probe_is_off_by_default_and_small_when_on():
    okf, ids, ns, rng = _construction_ii(seed=29)
    init_id = ids * rng.uniform(0.97, 1.03, ids.size)
    init_n = np.array([rot(np.cross(ns[0], rng.normal(size=3)),
                           math.radians(rng.uniform(0, 3))) @ ns[0] for _ in range(ids.size)])
    a = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, a, oracle.OracleParams(iters=6))
    b = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, b, oracle.OracleParams(iters=6, perturb=0.0, perturb_seed=5))
    assert np.array_equal(a["inv_depth"], b["inv_depth"]) and np.array_equal(a["nz"], b["nz"])
    c = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, c, oracle.OracleParams(iters=6, perturb=1e-6, perturb_seed=5))
    d = oracle.new_state(init_id, init_n)
    oracle.optimize(okf, d, oracle.OracleParams(iters=6, perturb=1e-6, perturb_seed=6))
    assert not np.array_equal(c["inv_depth"], a["inv_depth"])
    assert not np.array_equal(c["inv_depth"], d["inv_depth"])
    # on this well-conditioned construction the perturbation stays small
    assert np.max(np.abs(c["inv_depth"] / a["inv_depth"] - 1)) < 1e-5
