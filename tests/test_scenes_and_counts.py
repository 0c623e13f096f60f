"""Host-side pieces on the CPU: the disc-surfel scene generator (lattice,
holes, ground truth at the centre, purity) and the disc pixel counts
bench.py prices the disc kernel with, against the oracle's Eq. 4 support."""
import dataclasses
import math

import numpy as np

import oracle
from scenegen import lattice, make_disc_surfels, make_keyframe, spec_for_config


def _kf(seed=5, w=160, h=120):
    spec = dataclasses.replace(spec_for_config(1), width=w, height=h, n_nbr=1, n_rects=5, seed=seed)
    return make_keyframe(spec)


def test_lattice_and_holes():
    xs, ys = lattice(100, 70, 14)
    assert xs.min() == 7 and ys.min() == 7 and xs.max() < 100 and ys.max() < 70
    assert xs.size == len(range(7, 100, 14)) * len(range(7, 70, 14))
    assert np.all(np.diff(ys) >= 0)                    # row by row
    kf = _kf()
    d = make_disc_surfels(kf, radius=10.0, n_holes=2, seed=3)
    assert d.spacing == math.floor(10.0 * math.sqrt(2.0)) == 14
    full_x, full_y = lattice(kf.width, kf.height, 14)
    assert d.ux.size < full_x.size
    for (x0, y0, x1, y1) in d.holes:
        inside = (d.ux >= x0) & (d.ux < x1) & (d.uy >= y0) & (d.uy < y1)
        assert not inside.any()
    # the same seed gives the same discs
    d2 = make_disc_surfels(kf, radius=10.0, n_holes=2, seed=3)
    assert np.array_equal(d.ux, d2.ux) and np.array_equal(d.init_id, d2.init_id)


def test_ground_truth_is_the_plane_at_the_centre_and_purity():
    kf = _kf(seed=8)
    d = make_disc_surfels(kf, radius=6.0, n_holes=0)
    fx, fy, cx, cy = kf.K
    for i in range(0, d.ux.size, 7):
        x, y = int(d.ux[i]), int(d.uy[i])
        p = kf.planes[int(kf.kf_plane_id[y, x])]
        r = np.array([(x - cx) / fx, (y - cy) / fy, 1.0])
        # ray / plane intersection: lam r on the plane through p0 with normal n
        lam = float(p.n @ p.p0) / float(p.n @ r)
        assert abs(d.gt_id[i] * lam - 1) < 1e-12
        xs, ys = oracle.disc_support(kf.width, kf.height, (float(d.ux[i]), float(d.uy[i])), 6.0)
        same = np.all(kf.kf_plane_id[ys, xs] == kf.kf_plane_id[y, x])
        # the generator clips at the border instead of dropping pixels, so a
        # disc it calls pure is pure on its in-image pixels
        if d.pure[i]:
            assert same
    assert 0.3 < d.pure.mean() < 1.0


def test_bench_disc_pixel_counts_equal_the_oracle_support():
    import bench
    rng = np.random.default_rng(9)
    W, H = 120, 90
    ux = np.concatenate([rng.uniform(-5, W + 5, 200), [0.0, 119.0, 60.5, 60.0]]).astype(np.float32)
    uy = np.concatenate([rng.uniform(-5, H + 5, 200), [0.0, 89.0, 45.5, 45.0]]).astype(np.float32)
    for r in (1.5, 5.0, 10.0, 12.0):
        got = bench.disc_pixel_counts(ux, uy, r, W, H)
        want = [oracle.disc_support(W, H, (float(x), float(y)), r)[0].size for x, y in zip(ux, uy)]
        assert np.array_equal(got, want)
