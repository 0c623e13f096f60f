"""The allocation-free entry point sgn_transfer_surfels_static (static device
scratch, no workspace argument) against sgn_transfer_surfels with a caller
workspace, through the C ABI: every output field bitwise equal, on two calls
in a row (the second with a smaller destination grid, so the static scratch
holds the first call's larger contents), and the size limit refused."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.helpers import random_unit_cap, rot

pytestmark = pytest.mark.gpu


def _src(rng, W, H, S):
    import oracle
    from paper_1910_01997_amd import surfgn as sg
    m = (W // S) * (H // S)
    ids = rng.uniform(0.25, 1.0, m).astype(np.float32)
    ns = np.array([random_unit_cap(rng, 40) for _ in range(m)], np.float32)
    flags = np.zeros(m, np.uint32)
    flags[rng.choice(m, m // 20, replace=False)] = oracle.UNINIT
    src = sg.SurfelState.from_arrays(ids, ns, flags=flags)
    src.last_update.copy_(torch.as_tensor(rng.integers(1, 1000, m).astype(np.int32), device="cuda"))
    return src


def _dst(m):
    from paper_1910_01997_amd import surfgn as sg
    dst = sg.SurfelState.from_arrays(np.full(m, 7.0, np.float32), np.ones((m, 3), np.float32))
    return (dst, torch.full((m,), 9, dtype=torch.uint8, device="cuda"),
            torch.full((m,), -5, dtype=torch.int32, device="cuda"))


def _host(out):
    dst, is_new, win = out
    h = dst.to_host()
    h["is_new"] = is_new.cpu().numpy()
    h["win"] = win.cpu().numpy()
    return h


def test_static_scratch_transfer_equals_workspace_transfer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import surfgn as sg
    ctx = sg.Context(0)
    try:
        rng = np.random.default_rng(11)
        cases = [  # (source grid, destination grid): the second call is the smaller one
            (((600.0, 600.0, 320.0, 240.0), 640, 480, 4), ((1100.0, 1100.0, 640.0, 360.0), 1280, 720, 4)),
            (((300.0, 300.0, 160.0, 120.0), 320, 240, 4), ((290.0, 305.0, 150.0, 118.0), 320, 240, 8)),
        ]
        for k, (sgrid, dgrid) in enumerate(cases):
            (K0, W0, H0, S0), (K1, W1, H1, S1) = sgrid, dgrid
            print(f"case static scratch call {k}: {W0}x{H0}/{S0} -> {W1}x{H1}/{S1}", flush=True)
            src = _src(rng, W0, H0, S0)
            R = rot(rng.normal(size=3), math.radians(3))
            t = np.array([0.05, -0.02, -0.06])
            m1 = (W1 // S1) * (H1 // S1)
            g0, g1, pose = sg.grid_of(K0, W0, H0, S0), sg.grid_of(K1, W1, H1, S1), sg.pose_of(R, t)
            a = _dst(m1)
            sg.sgn_transfer_surfels(ctx.handle, g0, src.c, pose, g1, a[0].c, a[1].data_ptr(), a[2].data_ptr(),
                                    ctx.workspace(sg.sgn_transfer_workspace_bytes([g1])))
            b = _dst(m1)
            sg.sgn_transfer_surfels_static(ctx.handle, g0, src.c, pose, g1, b[0].c, b[1].data_ptr(),
                                           b[2].data_ptr())
            torch.cuda.synchronize()
            ha, hb = _host(a), _host(b)
            assert int((ha["win"] >= 0).sum()) > 1000          # surfels landed
            for f in ("inv_depth", "n", "flags", "cost", "nvalid", "last_update", "is_new", "win"):
                assert np.array_equal(ha[f], hb[f]), f"call {k}: {f} differs"
        # a destination grid beyond the static scratch is refused, nothing enqueued
        big = sg.grid_of((3000.0, 3000.0, 2048.0, 1080.0), 4096, 2160, 4)
        m = (4096 // 4) * (2160 // 4)
        assert sg.sgn_transfer_workspace_bytes([big]) > sg.STATIC_SCRATCH_BYTES
        src = _src(rng, 64, 64, 4)
        c = _dst(m)
        with pytest.raises(sg.SurfgnError, match="SGN_STATIC_SCRATCH_BYTES"):
            sg.sgn_transfer_surfels_static(ctx.handle, sg.grid_of((60.0, 60.0, 32.0, 32.0), 64, 64, 4), src.c,
                                           sg.pose_of(np.eye(3), np.zeros(3)), big, c[0].c, c[1].data_ptr(),
                                           None)
        torch.cuda.synchronize()
        assert np.all(c[1].cpu().numpy() == 9)
    finally:
        ctx.close()
