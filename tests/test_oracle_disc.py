"""Pins of the oracle's disc-surfel functions (Eq. 4 support, the depth-
buffered render with its surfel-index map, the empty-area search and the
neighbour initialisation of the Surfel Initialization section) against
independent routes: lattice-point counts of the circle, odd tiles that are
exactly discs, ray/plane intersections by a linear solve, and brute force
over whole maps."""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import (angle_deg, bilinear_scipy_many, plane_homography, random_unit_cap,
                           ray, rot, smooth_texture)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# --- Eq. 4 support ------------------------------------------------------------

def test_disc_support_counts_lattice_points_of_the_circle():
    """The number of integer points with x^2 + y^2 <= r^2 is 317 for r = 10
    and 81 for r = 5 (Gauss's circle problem; OEIS A000328).  The support is
    strict (|u - u_s| < r), so the 12 representations of 100 = 10^2 + 0^2 =
    6^2 + 8^2 (and of 25 = 5^2 + 0^2 = 3^2 + 4^2) on the circle drop out."""
    xs, ys = oracle.disc_support(200, 200, (100.0, 100.0), 10.0)
    assert xs.size == 317 - 12
    xs5, _ = oracle.disc_support(200, 200, (50.0, 60.0), 5.0)
    assert xs5.size == 81 - 12
    # the image corner keeps one quadrant: of the 305 points, 1 is the
    # centre, 36 lie on the axes (1..9 in four directions) and the rest
    # split evenly over four open quadrants, 67 each; the closed quadrant
    # x, y >= 0 holds 1 + 9 + 9 + 67
    xc, yc = oracle.disc_support(200, 200, (0.0, 0.0), 10.0)
    assert xc.size == 86 and xc.min() == 0 and yc.min() == 0
    # a centre between four pixels with r = 1.5: only the four at distance
    # sqrt(0.5); the next ring is at sqrt(2.5)
    x4, y4 = oracle.disc_support(50, 50, (10.5, 20.5), 1.5)
    assert sorted(zip(x4.tolist(), y4.tolist())) == [(10, 20), (10, 21), (11, 20), (11, 21)]
    # r = 0.5 at a pixel: that pixel alone; pixels are listed row by row
    x1, y1 = oracle.disc_support(50, 50, (7.0, 9.0), 0.5)
    assert (x1.tolist(), y1.tolist()) == ([7], [9])
    assert np.all(np.diff(ys) >= 0)
    # the disc is the set of pixels strictly inside the circle, nothing else
    inside = (xs - 100.0) ** 2 + (ys - 100.0) ** 2
    assert inside.max() < 100 and len(set(zip(xs.tolist(), ys.tolist()))) == xs.size


def _general_scene(W, H, patch, seed=5):
    """One neighbour, general plane and pose; the keyframe is synthesised from
    the neighbour through the plane homography, so the plane has zero
    residual everywhere."""
    K = (80.0, 80.0, W / 2.0, H / 2.0)
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
    okf = oracle.OracleKeyframe(K, kfimg, I1[None], R[None], t[None], patch)
    return okf, K, n, d, rng


@pytest.mark.parametrize("S,r", [(3, 1.5), (5, 2.9)])
def test_odd_tiles_are_discs_and_optimise_identically(S, r):
    """An S x S tile (S odd) centred on its middle pixel is exactly the disc
    of radius r around it when sqrt(2) (S-1)/2 < r <= (S+1)/2: the tile path
    (pinned separately) and the disc path then see the same pixels in the
    same order and must agree bit for bit, through every iteration."""
    W, H = 60, 45
    okf, K, n, d, rng = _general_scene(W, H, S)
    gw, gh = okf.grid
    ux = np.array([S * tx + (S - 1) / 2 for ty in range(gh) for tx in range(gw)], np.float64)
    uy = np.array([S * ty + (S - 1) / 2 for ty in range(gh) for tx in range(gw)], np.float64)
    xs, ys = oracle.disc_support(W, H, (ux[7], uy[7]), r)
    assert xs.size == S * S
    m = gw * gh
    ids = np.array([(n @ ray(K, ux[i], uy[i])) / d for i in range(m)]) * rng.uniform(0.95, 1.05, m)
    ns = np.array([rot(np.cross(n, rng.normal(size=3)), math.radians(rng.uniform(0, 4))) @ n
                   for _ in range(m)])
    for prm in (oracle.OracleParams(iters=6), oracle.OracleParams(iters=6, lm_lambda=1e-2)):
        a = oracle.new_state(ids, ns)
        b = oracle.new_state(ids, ns)
        oracle.optimize(okf, a, prm)
        oracle.disc_optimize(okf, b, ux, uy, r, prm)
        for k in ("inv_depth", "nx", "ny", "nz", "flags", "cost", "nvalid"):
            assert np.array_equal(a[k], b[k]), k
    H1, b1, c1, n1 = oracle.linearize(okf, 3, 2, ids[0], ns[0])
    H2, b2, c2, n2 = oracle.disc_linearize(okf, (3 * S + (S - 1) / 2, 2 * S + (S - 1) / 2), r, ids[0], ns[0])
    assert n1 == n2 and np.array_equal(H1, H2) and np.array_equal(b1, b2) and c1 == c2


def test_disc_gauss_newton_fixed_point_and_convergence():
    """Discs of radius 10 at non-integer centres on a scene whose plane has
    zero residual: the plane is a fixed point, and perturbed starts converge
    to it."""
    W, H = 96, 72
    okf, K, n, d, rng = _general_scene(W, H, 1, seed=6)
    ux = rng.uniform(20, W - 20, 12)
    uy = rng.uniform(18, H - 18, 12)
    ids = np.array([(n @ ray(K, x, y)) / d for x, y in zip(ux, uy)])
    ns = np.tile(n, (12, 1))
    st = oracle.new_state(ids, ns)
    oracle.disc_optimize(okf, st, ux, uy, 10.0, oracle.OracleParams(iters=3))
    got_n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert np.max(np.abs(st["inv_depth"] / ids - 1)) < 1e-12
    assert np.max(angle_deg(got_n, ns)) < 1e-9
    assert st["cost"].max() < 1e-24 and np.all(st["nvalid"] > 250)
    init_id = ids * rng.uniform(0.97, 1.03, 12)
    init_n = np.array([rot(np.cross(n, rng.normal(size=3)), math.radians(rng.uniform(0, 3))) @ n
                       for _ in range(12)])
    st = oracle.new_state(init_id, init_n)
    oracle.disc_optimize(okf, st, ux, uy, 10.0, oracle.OracleParams(iters=10))
    got_n = np.stack([st["nx"], st["ny"], st["nz"]], 1)
    assert np.max(np.abs(st["inv_depth"] / ids - 1)) < 1e-10
    assert np.max(angle_deg(got_n, ns)) < 1e-8


# --- depth-buffered render ------------------------------------------------------

def _ray_plane_id(K, us, id_s, n, u):
    """Inverse depth where the ray of pixel u meets the plane through
    r_s / id_s with normal n, by a 3x3 solve: lam r_u = p_s + s a + q b."""
    ps = ray(K, *us) / id_s
    a = np.cross(n, [0.3, 0.5, 0.7])
    b = np.cross(n, a)
    lam = np.linalg.solve(np.stack([ray(K, *u), -a, -b], 1), ps)[0]
    return 1.0 / lam


def test_disc_render_keeps_the_nearest_plane():
    K = (70.0, 72.0, 30.0, 22.0)
    W, H = 60, 44
    okf = oracle.OracleKeyframe(K, np.zeros((H, W)), np.zeros((0, H, W)), np.zeros((0, 3, 3)),
                                np.zeros((0, 3)), 1)
    rng = np.random.default_rng(12)
    m = 30
    ux = rng.uniform(-3, W + 3, m)
    uy = rng.uniform(-3, H + 3, m)
    ids = rng.uniform(0.25, 1.0, m)
    ns = np.array([random_unit_cap(rng, 45) for _ in range(m)])
    flags = np.zeros(m, np.uint32)
    flags[4] = oracle.UNINIT
    flags[9] = oracle.DEGENERATE
    ids[11] = ids[12]                           # an exact tie on a shared plane
    ux[11], uy[11], ns[11] = ux[12], uy[12], ns[12]
    r = 7.5
    st = oracle.new_state(ids, ns, flags)
    idm, ind = oracle.disc_render(okf, st, ux, uy, r)
    # brute force: every pixel against every usable surfel
    for y in range(H):
        for x in range(W):
            best, who = 0.0, -1
            for i in range(m):
                if flags[i] or math.hypot(x - ux[i], y - uy[i]) >= r:
                    continue
                v = _ray_plane_id(K, (ux[i], uy[i]), ids[i], ns[i], (x, y))
                if v > 0 and v > best * (1 + 1e-12):
                    best, who = v, i
            if who < 0:
                assert ind[y, x] == -1 and idm[y, x] == 0.0
            else:
                assert idm[y, x] == pytest.approx(best, rel=1e-11)
                assert ind[y, x] == who or idm[y, x] == pytest.approx(
                    _ray_plane_id(K, (ux[ind[y, x]], uy[ind[y, x]]), ids[ind[y, x]], ns[ind[y, x]], (x, y)),
                    rel=1e-11)
    assert not np.any(ind == 4) and not np.any(ind == 9)
    assert np.any(ind == 11) and not np.any(ind == 12)        # the tie goes to the lower index


def test_disc_render_occlusion_by_hand():
    """Two fronto-parallel discs, at 1 m and 2 m: the overlap shows the near
    one; each shows itself elsewhere."""
    K = (50.0, 50.0, 20.0, 20.0)
    okf = oracle.OracleKeyframe(K, np.zeros((40, 40)), np.zeros((0, 40, 40)), np.zeros((0, 3, 3)),
                                np.zeros((0, 3)), 1)
    st = oracle.new_state([0.5, 1.0], [[0, 0, -1], [0, 0, -1]])
    idm, ind = oracle.disc_render(okf, st, [14.0, 22.0], [20.0, 20.0], 6.0)
    assert ind[20, 18] == 1 and idm[20, 18] == 1.0       # in both discs: the 1 m one
    assert ind[20, 10] == 0 and idm[20, 10] == 0.5       # only the far disc
    assert ind[20, 27] == 1 and ind[5, 5] == -1 and idm[5, 5] == 0.0


# --- the search for empty areas ------------------------------------------------

@pytest.mark.parametrize("seed,r,alpha", [(1, 6.0, 1.25), (2, 6.0, 1.25), (3, 8.0, 1.0), (4, 5.0, 2.0)])
def test_disc_search_matches_the_definition(seed, r, alpha):
    rng = np.random.default_rng(seed)
    W, H = 83, 61
    imap = np.full((H, W), -1, np.int32)
    for _ in range(6):                          # blobs of measurements
        cx, cy, rr = rng.uniform(0, W), rng.uniform(0, H), rng.uniform(4, 14)
        Y, X = np.mgrid[0:H, 0:W]
        imap[(X - cx) ** 2 + (Y - cy) ** 2 < rr * rr] = rng.integers(0, 50)
    spacing = 8
    xs, ys, found = oracle.disc_search(imap, r, alpha, spacing)
    # definition: no non-empty pixel within alpha r (full scan, no window)
    ney, nex = np.nonzero(imap >= 0)
    expect = []
    for cy in range(spacing // 2, H, spacing):
        for cx in range(spacing // 2, W, spacing):
            # integer squared distances: alpha r = 8 or 10 makes ties exact
            d2 = np.min((nex - cx) ** 2 + (ney - cy) ** 2) if nex.size else np.inf
            if d2 > (alpha * r) ** 2:
                expect.append((cx, cy))
    assert found == len(expect) and list(zip(xs.tolist(), ys.tolist())) == expect
    assert 0 < found < ((W + spacing - 1) // spacing) * ((H + spacing - 1) // spacing)
    # capacity: the first ones in lattice order, and the full count
    xs2, ys2, found2 = oracle.disc_search(imap, r, alpha, spacing, capacity=3)
    assert found2 == found and list(zip(xs2.tolist(), ys2.tolist())) == expect[:3]


# --- neighbour initialisation ----------------------------------------------------

def _blank_kf(K, W, H):
    return oracle.OracleKeyframe(K, np.zeros((H, W)), np.zeros((0, H, W)), np.zeros((0, 3, 3)),
                                 np.zeros((0, 3)), 1)


def test_disc_init_is_exact_on_one_plane_and_follows_the_distance_rule():
    K = (80.0, 82.0, 40.0, 30.0)
    W, H = 80, 60
    okf = _blank_kf(K, W, H)
    n = np.array([0.25, -0.3, -0.92])
    n /= np.linalg.norm(n)
    d = -2.1
    r = 6.0
    # old surfels on a lattice except a hole; their planes are one plane
    cx = [x for y in range(4, H, 8) for x in range(4, W, 8)]
    cy = [y for y in range(4, H, 8) for x in range(4, W, 8)]
    keep = [i for i in range(len(cx)) if not (30 <= cx[i] <= 52 and 20 <= cy[i] <= 44)]
    ux = np.array([cx[i] for i in keep], np.float64)
    uy = np.array([cy[i] for i in keep], np.float64)
    m = ux.size
    ids = np.array([(n @ ray(K, x, y)) / d for x, y in zip(ux, uy)])
    ns = np.tile(n, (m, 1))
    ns[::3] *= -1                               # flipped normals: the mean aligns them
    st = oracle.new_state(ids, ns)
    idm, imap = oracle.disc_render(okf, st, ux, uy, r)
    xs, ys, found = oracle.disc_search(imap, r, 1.0, 8)
    assert found >= 2
    allx = np.concatenate([ux, xs.astype(np.float64)])
    ally = np.concatenate([uy, ys.astype(np.float64)])
    st2 = oracle.new_state(np.concatenate([ids, np.zeros(found)]),
                           np.concatenate([ns, np.tile([0.0, 0.0, -1.0], (found, 1))]))
    beta = 2.5
    oracle.disc_init(okf, st2, allx, ally, imap, m, r, beta)
    new = np.arange(m, m + found)
    got_n = np.stack([st2["nx"], st2["ny"], st2["nz"]], 1)
    ney, nex = np.nonzero(imap >= 0)
    for i, (x, y) in zip(new, zip(xs, ys)):
        # the neighbour set by definition: owners of pixels within beta r
        near = np.hypot(nex - x, ney - y) < beta * r
        owners = np.unique(imap[ney[near], nex[near]])
        if owners.size == 0:
            assert st2["flags"][i] == oracle.UNINIT and st2["inv_depth"][i] == 0.0
            continue
        assert st2["flags"][i] == 0
        expect = _ray_plane_id(K, (ux[owners[0]], uy[owners[0]]), ids[owners[0]], ns[owners[0]], (x, y))
        assert st2["inv_depth"][i] == pytest.approx(expect, rel=1e-12)
        assert angle_deg(got_n[i], n)[0] < 1e-9
    assert np.any(st2["flags"][new] == 0)
    # old surfels are untouched
    assert np.array_equal(st2["inv_depth"][:m], ids)


def test_disc_init_mean_over_two_planes_and_uninit():
    K = (60.0, 60.0, 30.0, 30.0)
    okf = _blank_kf(K, 60, 60)
    # two neighbours with different fronto-parallel planes near (30, 30),
    # one far away, one whose nearest pixel (30, 38) is exactly beta r = 8
    # away (not a neighbour: the rule is strict); a second new surfel with
    # nobody near it
    ux = np.array([24.0, 37.0, 5.0, 30.0, 30.0, 55.0])
    uy = np.array([30.0, 30.0, 5.0, 41.5, 30.0, 55.0])
    ids = np.array([0.5, 0.25, 0.9, 0.8, 0.0, 0.0])
    ns = np.array([[0, 0, -1], [0, 0, 1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1]], np.float64)
    st = oracle.new_state(ids, ns)
    idm, imap = oracle.disc_render(okf, oracle.new_state(ids[:4], ns[:4]), ux[:4], uy[:4], 4.0)
    assert imap[38, 30] == 3 and imap[37, 30] == -1
    oracle.disc_init(okf, st, ux, uy, imap, 4, 4.0, 2.0)
    # owners within 8 px of (30, 30): surfel 0 (pixels from x = 21 to 27)
    # and surfel 1 (from x = 34); surfel 2 is 35 px away
    assert st["inv_depth"][4] == pytest.approx(0.375, rel=1e-15)
    assert np.allclose([st["nx"][4], st["ny"][4], st["nz"][4]], [0, 0, -1])
    assert st["flags"][4] == 0
    assert st["flags"][5] == oracle.UNINIT and st["inv_depth"][5] == 0.0


# --- Eq. 10 for disc surfels ------------------------------------------------------

def test_disc_transfer_identity_keeps_every_usable_surfel():
    K = (80.0, 82.0, 40.0, 30.0)
    rng = np.random.default_rng(21)
    m = 40
    ux, uy = rng.uniform(0, 79, m), rng.uniform(0, 59, m)
    ids = rng.uniform(0.2, 1.0, m)
    ns = np.array([random_unit_cap(rng, 40) for _ in range(m)])
    flags = np.zeros(m, np.uint32)
    flags[3] = oracle.UNINIT
    flags[7] = oracle.DEGENERATE
    ids[11] = 0.0
    st = oracle.new_state(ids, ns, flags)
    st["last_update"][:] = np.arange(m) + 100
    out, (dx, dy), idx, landed = oracle.disc_transfer(K, K, (80, 60), np.eye(3), np.zeros(3), st, ux, uy)
    keep = [i for i in range(m) if i not in (3, 7, 11)]
    assert landed == len(keep) and list(idx) == keep
    assert np.max(np.abs(dx - ux[keep])) < 1e-12 and np.max(np.abs(dy - uy[keep])) < 1e-12
    assert np.max(np.abs(out["inv_depth"] / ids[keep] - 1)) < 1e-14
    assert np.max(angle_deg(np.stack([out["nx"], out["ny"], out["nz"]], 1), ns[keep])) < 1e-12
    assert np.array_equal(out["last_update"], np.arange(m)[keep] + 100) and np.all(out["flags"] == 0)


def test_disc_transfer_sideways_wall_shifts_by_f_t_over_d():
    """A fronto-parallel wall at depth 2 m; the camera frame moves so that
    X' = X + (1/8, 0, 0): every centre shifts by fx (1/8) / 2 = 4 px, depth
    and normal are kept (every quantity is exact in binary with fx = 64,
    cx = 32); a centre landing exactly on the last column (x = 79) stays,
    centres pushed past it drop out, and a capacity keeps the first ones in
    source order.  A surfel of negative inverse depth is never moved, even
    where the pose would put its point in front of the camera."""
    K = (64.0, 64.0, 32.0, 30.0)
    xs = np.array([3.0, 9.0, 30.0, 57.5, 75.0, 76.0, 78.0])
    ux = np.tile(xs, 3)
    uy = np.repeat([5.0, 20.0, 41.5], xs.size)
    m = ux.size
    st = oracle.new_state(np.full(m, 0.5), np.tile([0.0, 0.0, -1.0], (m, 1)))
    out, (dx, dy), idx, landed = oracle.disc_transfer(K, K, (80, 60), np.eye(3), [0.125, 0.0, 0.0], st, ux, uy)
    inside = ux + 4.0 <= 79.0
    assert landed == inside.sum() and np.array_equal(idx, np.nonzero(inside)[0])
    assert np.array_equal(dx, ux[inside] + 4.0) and np.array_equal(dy, uy[inside])
    assert 79.0 in dx and np.all(out["inv_depth"] == 0.5)
    out2, _, idx2, landed2 = oracle.disc_transfer(K, K, (80, 60), np.eye(3), [0.125, 0.0, 0.0], st, ux, uy,
                                                  capacity=5)
    assert landed2 == landed and np.array_equal(idx2, idx[:5])
    # id = -0.5 at the principal point: p = (0, 0, -2), moved by t_z = 3 to z = 1
    neg = oracle.new_state([-0.5, 0.5], [[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    _, _, nidx, nland = oracle.disc_transfer(K, K, (80, 60), np.eye(3), [0.0, 0.0, 3.0], neg, [32.0, 40.0],
                                             [30.0, 30.0])
    assert nland == 1 and list(nidx) == [1]


def test_disc_transfer_round_trip_and_matrix_projection():
    """A general pose and its inverse bring every surfel back; the forward
    landing equals a 4x4 homogeneous-matrix projection of the back-projected
    centre."""
    K = (300.0, 310.0, 160.0, 120.0)
    rng = np.random.default_rng(22)
    m = 60
    ux, uy = rng.uniform(40, 280, m), rng.uniform(30, 210, m)
    ids = rng.uniform(0.3, 0.8, m)
    ns = np.array([random_unit_cap(rng, 40) for _ in range(m)])
    R = rot(rng.normal(size=3), math.radians(3.0))
    t = np.array([0.05, -0.03, 0.02])
    st = oracle.new_state(ids, ns)
    out, (dx, dy), idx, landed = oracle.disc_transfer(K, K, (320, 240), R, t, st, ux, uy)
    assert landed > 50
    fx, fy, cx, cy = K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    Km = np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1.0]])
    got_n = np.stack([out["nx"], out["ny"], out["nz"]], 1)
    assert np.max(np.abs(got_n - ns[idx] @ R.T)) < 1e-15      # n' = R n
    for j, i in enumerate(idx):
        P = np.append(np.linalg.solve(Km, [ux[i], uy[i], 1.0]) / ids[i], 1.0)
        q = Km @ (T @ P)[:3]
        assert q[0] / q[2] == pytest.approx(dx[j], abs=1e-9)
        assert q[1] / q[2] == pytest.approx(dy[j], abs=1e-9)
        assert 1.0 / (T @ P)[2] == pytest.approx(out["inv_depth"][j], rel=1e-12)
    back, (bx, by), bidx, _ = oracle.disc_transfer(K, K, (320, 240), R.T, -R.T @ t, out, dx, dy)
    src = idx[bidx]
    assert np.max(np.abs(bx - ux[src])) < 1e-9 and np.max(np.abs(by - uy[src])) < 1e-9
    assert np.max(np.abs(back["inv_depth"] / ids[src] - 1)) < 1e-12
    assert np.max(angle_deg(np.stack([back["nx"], back["ny"], back["nz"]], 1), ns[src])) < 1e-9
