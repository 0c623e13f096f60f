"""16 x 16-pixel surfels on the device (each lane of the wavefront owns four
pixels of the one surfel) against the FP64 oracle: the Gauss-Newton update
with neighbour-plane initialisation in every storage form, the damped
variant, depth-only, the render, batch == plain bitwise, and the plans and
autotuner choices this patch size has."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from scenegen import make_keyframe, spec_for_config
from tests.parity import assert_parity, assert_render, check_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import surfgn as sg
    c = sg.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _mods():
    from paper_1910_01997_amd import engine, surfgn
    return surfgn, engine


def _spec(**kw):
    base = dataclasses.replace(spec_for_config(1), width=192, height=144, patch=16, n_nbr=4,
                               n_rects=4, seed=41, iters=10)
    return dataclasses.replace(base, **kw)


def _state_equal(a: dict, b: dict):
    for k in ("inv_depth", "n", "flags", "cost", "nvalid"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_patch16_update_with_init_matches_oracle(ctx, storage):
    sg, engine = _mods()
    kf = make_keyframe(_spec(), device="cuda")
    print(f"case S16 192x144 N4 init {storage}", flush=True)
    d = engine.DeviceKeyframe.from_scene(ctx, kf, storage=storage)
    engine.update_plain(ctx, d, sg.params(iters=10))
    torch.cuda.synchronize()
    dev = d.state.to_host()
    assert dev["inv_depth"].size == 12 * 9
    res = check_parity(d, dev, kf.init_id, kf.init_n, kf.is_new, oracle.OracleParams(iters=10),
                       label=f"S16 {storage}")
    assert_parity(res, label=f"S16 {storage}", max_unstable=0.06)  # measured 0.028-0.037
    # the rendered map against the oracle's render of the device's own state
    assert_render(d, dev, d.inv_depth_out.cpu().numpy())


@pytest.mark.parametrize("W,H,N", [(200, 130, 2), (16, 16, 3), (264, 200, 8)])
def test_patch16_ragged_sizes(ctx, W, H, N):
    sg, engine = _mods()
    kf = make_keyframe(_spec(width=W, height=H, n_nbr=N, half_new=False, seed=42), device="cuda")
    print(f"case S16 ragged {W}x{H} N{N}", flush=True)
    d = engine.DeviceKeyframe.from_scene(ctx, kf, storage="f16")
    engine.update_batch(ctx, [d], sg.params(iters=8))
    torch.cuda.synchronize()
    dev = d.state.to_host()
    assert dev["inv_depth"].size == (W // 16) * (H // 16)
    res = check_parity(d, dev, kf.init_id, kf.init_n, None, oracle.OracleParams(iters=8),
                       label=f"S16 ragged {W}x{H} N{N}")
    # probe-unstable measured: 0, 0, 0.031
    assert_parity(res, label=f"S16 ragged {W}x{H} N{N}", max_unstable={200: 0.02, 16: 0.0, 264: 0.06}[W])
    dm = d.inv_depth_out.cpu().numpy()
    assert np.all(dm[(H // 16) * 16:, :] == 0) and np.all(dm[:, (W // 16) * 16:] == 0)


def test_patch16_damped_and_depth_only(ctx):
    sg, engine = _mods()
    kf = make_keyframe(_spec(seed=43), device="cuda")
    for name, prm, oprm in (
            ("LM", sg.params(iters=10, lm_lambda=1e-3), oracle.OracleParams(iters=10, lm_lambda=1e-3)),
            ("depth-only", sg.params(iters=10, depth_only=True), oracle.OracleParams(iters=10, depth_only=True))):
        print(f"case S16 {name}", flush=True)
        d = engine.DeviceKeyframe.from_scene(ctx, kf)
        engine.update_plain(ctx, d, prm)
        torch.cuda.synchronize()
        dev = d.state.to_host()
        res = check_parity(d, dev, kf.init_id, kf.init_n, kf.is_new, oprm, label=f"S16 {name}")
        # probe-unstable measured: LM 0.259, depth-only 0 (108 surfels; the
        # depth-only run has 3 at the valid-window edge); reclassified under
        # LM: 8 or 9 of the 108 with the kernel's rounding (0.074-0.083)
        assert_parity(res, label=f"S16 {name}", max_unstable={"LM": 0.28}.get(name, 0.02),
                      max_reclassified={"LM": 0.10}.get(name, 0.02), max_edge=0.05)


def test_patch16_batch_equals_plain_and_autotune(ctx):
    sg, engine = _mods()
    kfs = [make_keyframe(dataclasses.replace(_spec(width=640, height=480, n_nbr=8), seed=50 + i),
                         device="cuda") for i in range(3)]
    print("case S16 640x480 batch of 3 == plain", flush=True)
    prm = sg.params(iters=6)
    ref = []
    for k in kfs:
        d = engine.DeviceKeyframe.from_scene(ctx, k, storage="f16")
        engine.update_plain(ctx, d, prm)
        torch.cuda.synchronize()
        ref.append((d.state.to_host(), d.inv_depth_out.cpu().numpy()))
    for pl in (None, sg.plan(1, 1, 0, 0, 0, 0, groups=1), sg.plan(1, 1, 1, 0, 0, 1, groups=1)):
        ds = [engine.DeviceKeyframe.from_scene(ctx, k, storage="f16") for k in kfs]
        engine.update_batch(ctx, ds, prm, pl)
        torch.cuda.synchronize()
        for d, (st, dm) in zip(ds, ref):
            _state_equal(d.state.to_host(), st)
            assert np.array_equal(d.inv_depth_out.cpu().numpy(), dm)
    # the autotuner only offers this patch size's one work-item shape, and
    # leaves the state as it found it
    ds = [engine.DeviceKeyframe.from_scene(ctx, k, storage="f16") for k in kfs]
    items = sg.batch_array([d.item() for d in ds])
    best = engine.autotune(ctx, items, len(ds), prm)
    torch.cuda.synchronize()
    assert (best.tiles_x, best.tiles_y, best.groups) == (1, 1, 1)
    for d, k in zip(ds, kfs):
        assert np.array_equal(d.state.to_host()["inv_depth"], k.init_id.reshape(-1))
    # sampled oracle parity for the first keyframe of the batch
    okf = kfs[0]
    res = check_parity(engine.DeviceKeyframe.from_scene(ctx, okf, storage="f16"), ref[0][0],
                       okf.init_id, okf.init_n, okf.is_new, oracle.OracleParams(iters=6),
                       label="S16 640x480 batch item 0")
    assert_parity(res, label="S16 640x480 batch item 0", max_unstable=0.13)  # measured 0.103


def test_patch16_refuses_other_plans(ctx):
    sg, engine = _mods()
    L = sg.lib()
    kf = make_keyframe(_spec(half_new=False), device="cuda")
    d = engine.DeviceKeyframe.from_scene(ctx, kf)
    prm = sg.params(iters=3)
    print("case S16 unsupported plans", flush=True)
    for pl in (sg.plan(2, 2, groups=1), sg.plan(1, 1, groups=2), sg.plan(1, 1, groups=4),
               sg.plan(4, 1, groups=1)):
        assert L.sgn_optimize_keyframe(ctx.handle, d.view.c, d.state.c, prm, pl) == sg.SGN_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert np.array_equal(d.state.to_host()["inv_depth"], kf.init_id.reshape(-1))
