"""Parameters and small shapes through the C ABI against the FP64 oracle:
Huber threshold and initialisation radius, the double-precision solve for
every surfel, the damped variant of the depth-only ablation, u8 storage with
another scale, the surfel-index map, and keyframes of a single surfel."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from scenegen import make_keyframe, spec_for_config
from tests.parity import assert_parity, check_parity, oracle_keyframe, oracle_state

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


# These scenes have 4 neighbour frames (the batch workload's lower end), where
# more 4x4 surfels are not determined at float resolution than with 8; the
# unstable fraction is bounded at 25 % here.
def _spec(**kw):
    base = dataclasses.replace(spec_for_config(1), width=192, height=144, n_rects=5, n_nbr=4,
                               seed=31, half_new=True)
    return dataclasses.replace(base, **kw)


def _run(ctx, kf, prm, storage="f32", **kw):
    sg, engine = _mods()
    d = engine.DeviceKeyframe.from_scene(ctx, kf, storage=storage, **kw)
    engine.update_plain(ctx, d, prm)
    torch.cuda.synchronize()
    return d, d.state.to_host()


def test_huber_threshold_and_init_radius(ctx):
    sg, _ = _mods()
    kf = make_keyframe(_spec(), device="cuda")
    print("case huber_k 0.01, beta_r 8", flush=True)
    d, dev = _run(ctx, kf, sg.params(iters=10, huber_k=0.01, beta_r=8.0))
    res = check_parity(d, dev, kf.init_id, kf.init_n, kf.is_new,
                       oracle.OracleParams(iters=10, huber_k=0.01, beta_r=8.0), label="huber beta")
    assert_parity(res, label="huber beta", max_unstable=0.17)          # measured 0.144


def test_double_precision_solve_for_every_surfel(ctx):
    sg, _ = _mods()
    kf = make_keyframe(_spec(seed=32), device="cuda")
    print("case kappa_fp64 = 1", flush=True)
    d, dev = _run(ctx, kf, sg.params(iters=10, kappa_fp64=1.0))
    solved = (dev["nvalid"] >= 3) & ((dev["flags"] & (oracle.SOLVE_FAIL | oracle.DEGENERATE)) == 0)
    assert np.all(dev["flags"][solved] & oracle.FP64_SOLVE)
    res = check_parity(d, dev, kf.init_id, kf.init_n, kf.is_new, oracle.OracleParams(iters=10),
                       label="fp64 everywhere")
    assert_parity(res, label="fp64 everywhere", max_unstable=0.19)     # measured 0.168


def test_damped_depth_only(ctx):
    sg, _ = _mods()
    kf = make_keyframe(_spec(seed=33, half_new=False), device="cuda")
    print("case LM + depth-only", flush=True)
    d, dev = _run(ctx, kf, sg.params(iters=10, depth_only=True, lm_lambda=1e-2))
    assert np.array_equal(dev["n"], kf.init_n.reshape(-1, 3))
    res = check_parity(d, dev, kf.init_id, kf.init_n, None,
                       oracle.OracleParams(iters=10, depth_only=True, lm_lambda=1e-2),
                       label="LM depth-only")
    assert_parity(res, label="LM depth-only", max_unstable=0.03)       # measured 0.009


def test_u8_with_another_scale(ctx):
    sg, _ = _mods()
    kf = make_keyframe(_spec(seed=34), device="cuda")
    # images scaled to [0, 0.5] so that codes of step 1/200 stay within 0..100
    kf = dataclasses.replace(kf, kf_image=kf.kf_image * 0.5, nbr_images=kf.nbr_images * 0.5)
    print("case u8 scale 1/200", flush=True)
    d, dev = _run(ctx, kf, sg.params(iters=10, huber_k=4.5 / 255.0), storage="u8", u8_scale=1 / 200)
    codes = d.nbr_imgs.cpu().numpy()
    assert codes.max() <= 101
    res = check_parity(d, dev, kf.init_id, kf.init_n, kf.is_new,
                       oracle.OracleParams(iters=10, huber_k=4.5 / 255.0), label="u8 1/200")
    # half the contrast doubles the relative weight of the noise, so more
    # surfels sit near the edge of what float resolution determines
    assert_parity(res, label="u8 1/200", min_stable=0.998, max_unstable=0.15)  # measured 0.128


def test_surfel_index_map_matches_oracle(ctx):
    sg, engine = _mods()
    kf = make_keyframe(_spec(seed=35), device="cuda")
    d = engine.DeviceKeyframe.from_scene(ctx, kf, index_map=True)
    engine.update_plain(ctx, d, sg.params(iters=6))
    torch.cuda.synchronize()
    dev = d.state.to_host()
    st = oracle_state(dev["inv_depth"], dev["n"], dev["flags"])
    idm, ind = oracle.render(oracle_keyframe(d), st)
    got = d.index_out.cpu().numpy()
    assert np.array_equal(got >= 0, ind >= 0)
    assert np.array_equal(got[got >= 0], ind[got >= 0])


@pytest.mark.parametrize("W,H,S,N", [(8, 8, 8, 2), (4, 4, 4, 3), (7, 5, 4, 2)])
def test_single_surfel_keyframes(ctx, W, H, S, N):
    sg, engine = _mods()
    spec = _spec(width=W, height=H, patch=S, n_nbr=N, n_rects=1, half_new=False, seed=36)
    kf = make_keyframe(spec, device="cuda")
    print(f"case single surfel {W}x{H} S{S} N{N}", flush=True)
    d, dev = _run(ctx, kf, sg.params(iters=5))
    assert dev["inv_depth"].size == (W // S) * (H // S) == 1
    res = check_parity(d, dev, kf.init_id, kf.init_n, None, oracle.OracleParams(iters=5),
                       label=f"single {W}x{H}")
    assert_parity(res, label=f"single {W}x{H}", max_unstable=0.0)      # measured 0
