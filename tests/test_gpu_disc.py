"""Disc surfels (Eq. 4) on the device, through the C ABI, against the oracle:
the Gauss-Newton update over disc pixels in every storage form and with the
damped variant, the depth-buffered render and its surfel-index map, the
empty-area search with placement and neighbour initialisation, the whole
keyframe step chained, batch == alone, edge cases and argument errors."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from scenegen import make_disc_surfels, make_keyframe, spec_for_config
from tests.parity import angle_deg, assert_parity, check_parity, oracle_keyframe, oracle_state

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


def _scene(width=320, height=240, n_nbr=4, seed=61, radius=10.0, **kw):
    spec = dataclasses.replace(spec_for_config(1), width=width, height=height, n_nbr=n_nbr,
                               n_rects=8, seed=seed, half_new=False)
    kf = make_keyframe(spec, device="cuda")
    return kf, make_disc_surfels(kf, radius=radius, **kw)


def _disc_of(dk):
    ux, uy = dk.centres()
    return (ux, uy, dk.radius)


def _state_equal(a: dict, b: dict):
    for k in ("inv_depth", "n", "flags", "cost", "nvalid"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storage", ["f32", "f16", "u8"])
def test_disc_gauss_newton_matches_oracle(ctx, storage):
    sg, engine = _mods()
    kf, discs = _scene()
    print(f"case disc GN 320x240 r10 N4 {storage} ({discs.ux.size} surfels)", flush=True)
    dk = engine.DiscKeyframe.from_scene(ctx, kf, discs, storage=storage)
    engine.disc_update(ctx, [dk], sg.params(iters=10))
    torch.cuda.synchronize()
    dev = dk.state_host()
    res = check_parity(dk, dev, discs.init_id, discs.init_n, None, oracle.OracleParams(iters=10),
                       label=f"disc {storage}", disc=_disc_of(dk))
    # probe-unstable measured: f32 0.072, f16 0.077, u8 0.069
    assert_parity(res, label=f"disc {storage}", max_unstable=0.10)
    assert np.all(dev["nvalid"][dev["flags"] == 0] > 0)


def test_disc_damped_depth_only_and_radius_five(ctx):
    sg, engine = _mods()
    kf, discs = _scene(seed=62, radius=5.0)
    for name, prm, oprm in (
            ("LM", sg.params(iters=8, lm_lambda=1e-3), oracle.OracleParams(iters=8, lm_lambda=1e-3)),
            ("depth-only", sg.params(iters=8, depth_only=True), oracle.OracleParams(iters=8, depth_only=True))):
        print(f"case disc r5 {name}", flush=True)
        dk = engine.DiscKeyframe.from_scene(ctx, kf, discs)
        engine.disc_update(ctx, [dk], prm)
        torch.cuda.synchronize()
        dev = dk.state_host()
        if name == "depth-only":
            assert np.array_equal(dev["n"], discs.init_n)
        res = check_parity(dk, dev, discs.init_id, discs.init_n, None, oprm, label=f"disc r5 {name}",
                           disc=_disc_of(dk))
        # 5 px discs have ~80 pixels: more of them sit at the edge of what
        # float resolution determines, as with the small tiles, and most of
        # the damped variant's acceptance tests end in near-ties
        # (probe-unstable measured: LM 0.233, depth-only 0.001)
        assert_parity(res, label=f"disc r5 {name}", max_unstable={"LM": 0.26, "depth-only": 0.03}[name],
                      max_reclassified={"LM": 0.08, "depth-only": 0.02}[name])


def test_disc_render_matches_oracle_exactly(ctx):
    """Both sides evaluate Eq. 3 in double in the printed order, so the depth
    test takes the same decisions: the surfel-index map is equal and the
    inverse depths are the oracle's doubles rounded to float."""
    sg, engine = _mods()
    kf, discs = _scene(seed=63)
    # extra surfels: centres beyond the border, and a coincident pair (a tie)
    ux = np.concatenate([discs.ux, np.float32([-4.5, 323.0, 150.0, 150.0])])
    uy = np.concatenate([discs.uy, np.float32([100.0, 7.25, 120.0, 120.0])])
    ids = np.concatenate([discs.init_id, np.float32([0.6, 0.7, 2.0, 2.0])])
    ns = np.concatenate([discs.init_n, np.float32([[0, 0, -1], [0.1, 0, -1], [0, 0.2, -1], [0, 0.2, -1]])])
    ns = (ns / np.linalg.norm(ns, axis=1, keepdims=True)).astype(np.float32)
    flags = np.zeros(ids.size, np.uint32)
    flags[5] = oracle.UNINIT
    flags[9] = oracle.DEGENERATE
    print("case disc render 320x240", flush=True)
    dk = engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0, ux, uy, ids, ns,
                             flags=flags)
    dk.render()
    torch.cuda.synchronize()
    okf = oracle_keyframe(dk)
    st = oracle_state(ids, ns, flags)
    idm, ind = oracle.disc_render(okf, st, ux.astype(np.float64), uy.astype(np.float64), 10.0)
    got_i = dk.index_out.cpu().numpy()
    got_d = dk.inv_depth_out.cpu().numpy()
    assert np.array_equal(got_i, ind)
    assert np.array_equal(got_d, idm.astype(np.float32))
    assert not np.any(got_i == 5) and not np.any(got_i == 9)
    assert np.any(got_i == ids.size - 2) and not np.any(got_i == ids.size - 1)
    assert np.any(got_i == -1) and (got_i >= 0).mean() > 0.8


def test_disc_place_matches_oracle_and_respects_capacity(ctx):
    sg, engine = _mods()
    kf, discs = _scene(seed=64, n_holes=4, hole_frac=(0.2, 0.3))
    print("case disc placement 320x240", flush=True)
    m = discs.ux.size
    for room in (1000, 5):
        dk = engine.DiscKeyframe.from_scene(ctx, kf, discs, capacity=m + room)
        dk.render()
        imap = dk.index_out.cpu().numpy()
        placed, found = dk.place(alpha=1.0, beta=2.0)
        torch.cuda.synchronize()
        xs, ys, o_found = oracle.disc_search(imap, 10.0, 1.0, discs.spacing)
        assert found == o_found and found > 5
        assert placed == min(found, room)
        ux, uy = dk.centres()
        assert np.array_equal(ux[m:], xs[:placed].astype(np.float32))
        assert np.array_equal(uy[m:], ys[:placed].astype(np.float32))
        dev = dk.state_host()
        st = oracle_state(np.concatenate([discs.init_id, np.zeros(placed, np.float32)]),
                          np.concatenate([discs.init_n, np.tile(np.float32([0, 0, -1]), (placed, 1))]))
        oracle.disc_init(oracle_keyframe(dk), st, ux.astype(np.float64), uy.astype(np.float64), imap, m,
                         10.0, 2.0)
        new = np.arange(m, m + placed)
        assert np.array_equal(dev["flags"][new], st["flags"][new].astype(np.uint32))
        ok = st["flags"][new] == 0
        assert ok.sum() >= 1
        rel = np.abs(dev["inv_depth"][new][ok] / st["inv_depth"][new][ok] - 1)
        on = np.stack([st["nx"], st["ny"], st["nz"]], 1)[new][ok]
        assert rel.max() < 1e-5 and angle_deg(dev["n"][new][ok], on).max() < 1e-3
        assert np.all(dev["inv_depth"][new][~ok] == 0) and np.all(dev["cost"][new] == 0)
        # old surfels are untouched
        assert np.array_equal(dev["inv_depth"][:m], discs.init_id)


def test_disc_keyframe_step_chained(ctx):
    """render -> search and placement -> Gauss-Newton over old and new
    surfels -> render, each stage against the oracle from the device's input
    to that stage."""
    sg, engine = _mods()
    kf, discs = _scene(640, 480, 8, seed=65)
    print("case disc step 640x480 r10 N8", flush=True)
    dk = engine.DiscKeyframe.from_scene(ctx, kf, discs, capacity=discs.ux.size + 600, storage="f16")
    dk.render()
    placed, found = dk.place()
    start = dk.state_host()
    engine.disc_update(ctx, [dk], sg.params(iters=6))
    dk.render()
    torch.cuda.synchronize()
    assert placed == found and placed > 10
    dev = dk.state_host()
    res = check_parity(dk, dev, start["inv_depth"], start["n"], None, oracle.OracleParams(iters=6),
                       label="disc step", disc=_disc_of(dk), init_flags=start["flags"])
    assert_parity(res, label="disc step", max_unstable=0.10)       # measured 0.078
    ux, uy = dk.centres()
    idm, ind = oracle.disc_render(oracle_keyframe(dk), oracle_state(dev["inv_depth"], dev["n"], dev["flags"]),
                                  ux.astype(np.float64), uy.astype(np.float64), 10.0)
    assert np.array_equal(dk.index_out.cpu().numpy(), ind)
    # the rims of the holes are filled (their middles, farther than beta r
    # from any measurement, stay uninitialised): fewer empty pixels
    before = oracle.disc_render(oracle_keyframe(dk), oracle_state(discs.init_id, discs.init_n),
                                discs.ux.astype(np.float64), discs.uy.astype(np.float64), 10.0)[1]
    assert (ind < 0).sum() < (before < 0).sum()


def test_disc_batch_equals_alone_and_empty_cases(ctx):
    sg, engine = _mods()
    scenes = [_scene(seed=66 + i, n_nbr=3 + i) for i in range(3)]
    print("case disc batch of 3 == alone", flush=True)
    prm = sg.params(iters=5)
    alone = []
    for kf, discs in scenes:
        dk = engine.DiscKeyframe.from_scene(ctx, kf, discs, storage="u8")
        engine.disc_update(ctx, [dk], prm)
        torch.cuda.synchronize()
        alone.append(dk.state_host())
    dks = [engine.DiscKeyframe.from_scene(ctx, kf, discs, storage="u8") for kf, discs in scenes]
    engine.disc_update(ctx, dks, prm)
    torch.cuda.synchronize()
    for dk, ref in zip(dks, alone):
        _state_equal(dk.state_host(), ref)
    # no surfels: render gives no measurement, every candidate qualifies and
    # none can be initialised, the update is a no-op
    kf, discs = scenes[0]
    empty = engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0,
                                np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                                np.zeros((0, 3), np.float32), capacity=2000)
    engine.disc_update(ctx, [empty], prm)
    empty.render()
    assert np.all(empty.index_out.cpu().numpy() == -1) and np.all(empty.inv_depth_out.cpu().numpy() == 0)
    placed, found = empty.place()
    n_lat = len(range(7, 320, 14)) * len(range(7, 240, 14))
    assert placed == found == n_lat
    assert np.all(empty.state_host()["flags"] == oracle.UNINIT)


def test_disc_batch_in_xcd_shares_equals_alone(ctx):
    """Ten keyframes (2-7 neighbours, one without surfels) run in one launch
    with the work items in one share per XCD: every keyframe's result equals
    its update alone, bitwise."""
    sg, engine = _mods()
    scenes = [_scene(seed=90 + i, n_nbr=2 + i % 6) for i in range(10)]
    print("case disc batch of 10 in XCD shares == alone", flush=True)
    prm = sg.params(iters=4)

    def make(i):
        kf, discs = scenes[i]
        if i == 4:
            z = np.zeros(0, np.float32)
            return engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0, z, z, z,
                                       np.zeros((0, 3), np.float32), capacity=16, storage="f16")
        return engine.DiscKeyframe.from_scene(ctx, kf, discs, storage="f16")

    alone = []
    for i in range(len(scenes)):
        dk = make(i)
        engine.disc_update(ctx, [dk], prm)
        torch.cuda.synchronize()
        alone.append(dk.state_host())
    dks = [make(i) for i in range(len(scenes))]
    engine.disc_update(ctx, dks, prm)
    torch.cuda.synchronize()
    for dk, ref in zip(dks, alone):
        _state_equal(dk.state_host(), ref)
    assert sum(dk.count for dk in dks) > 3000


def test_disc_argument_errors(ctx):
    sg, engine = _mods()
    L = sg.lib()
    kf, discs = _scene(seed=70)
    dk = engine.DiscKeyframe.from_scene(ctx, kf, discs, capacity=discs.ux.size + 10)
    print("case disc argument errors", flush=True)
    prm = sg.params(iters=3)
    rneed = sg.sgn_disc_render_workspace_bytes(1, dk.item())
    pneed = sg.sgn_disc_place_workspace_bytes(1, dk.item(), 14)
    wp, wb = ctx.workspace(max(rneed, pneed))
    for r in (0.0, -1.0, 12.5, float("nan")):
        it = dk.item()
        it.radius = r
        assert L.sgn_disc_optimize(ctx.handle, sg.disc_array([it]), 1, prm) == sg.SGN_E_INVALID
        assert L.sgn_disc_render(ctx.handle, it, dk.inv_depth_out.data_ptr(), None, wp, wb) == sg.SGN_E_INVALID
    it = dk.item()
    it.ux = None
    assert L.sgn_disc_optimize(ctx.handle, sg.disc_array([it]), 1, prm) == sg.SGN_E_INVALID
    it = dk.item()
    it.count = -1
    assert L.sgn_disc_optimize(ctx.handle, sg.disc_array([it]), 1, prm) == sg.SGN_E_INVALID
    ok_pp = sg.sgn_disc_place_params(1.0, 2.0, 14)
    cnt = dk.counts.data_ptr()
    imap = dk.index_out.data_ptr()
    assert L.sgn_disc_place(ctx.handle, dk.item(), imap, discs.ux.size - 1, ok_pp, cnt, wp, wb) == sg.SGN_E_INVALID
    for pp in (sg.sgn_disc_place_params(0.0, 2.0, 14), sg.sgn_disc_place_params(1.0, 4.5, 14),
               sg.sgn_disc_place_params(1.0, 2.0, 0)):
        assert L.sgn_disc_place(ctx.handle, dk.item(), imap, dk.capacity, pp, cnt, wp, wb) == sg.SGN_E_INVALID
    assert L.sgn_disc_place(ctx.handle, dk.item(), None, dk.capacity, ok_pp, cnt, wp, wb) == sg.SGN_E_INVALID
    assert L.sgn_disc_render(ctx.handle, dk.item(), None, None, wp, wb) == sg.SGN_E_INVALID
    # undersized or missing workspaces
    assert L.sgn_disc_render(ctx.handle, dk.item(), dk.inv_depth_out.data_ptr(), None, wp,
                             rneed - 1) == sg.SGN_E_INVALID
    assert "workspace" in sg.sgn_last_error()
    assert L.sgn_disc_place(ctx.handle, dk.item(), imap, dk.capacity, ok_pp, cnt, None, pneed) == sg.SGN_E_INVALID
    assert L.sgn_disc_place(ctx.handle, dk.item(), imap, dk.capacity, ok_pp, cnt, wp, pneed - 1) == sg.SGN_E_INVALID
    # nothing was enqueued: the state is untouched
    torch.cuda.synchronize()
    assert np.array_equal(dk.state_host()["inv_depth"], discs.init_id)


def _as_keyframe_of(kf, j):
    """Neighbour frame j of kf as a keyframe: its image, with the old keyframe
    and the other neighbour frames as its neighbours (poses composed:
    X_i = R_i R_j^T (X_j - t_j) + t_i)."""
    Rj, tj = kf.R[j], kf.t[j]
    imgs = [kf.kf_image] + [kf.nbr_images[i] for i in range(kf.n_nbr) if i != j]
    Rs = [Rj.T] + [kf.R[i] @ Rj.T for i in range(kf.n_nbr) if i != j]
    ts = [-Rj.T @ tj] + [kf.t[i] - kf.R[i] @ Rj.T @ tj for i in range(kf.n_nbr) if i != j]
    return kf.nbr_images[j], torch.stack(imgs), np.stack(Rs), np.stack(ts)


def test_disc_transfer_matches_oracle_exactly(ctx):
    sg, engine = _mods()
    kf, discs = _scene(seed=71)
    print("case disc transfer 320x240", flush=True)
    src = engine.DiscKeyframe.from_scene(ctx, kf, discs)
    engine.disc_update(ctx, [src], sg.params(iters=5))
    img1, nb1, R1, t1 = _as_keyframe_of(kf, 0)
    for cap in (src.count + 10, 50):
        dst = engine.DiscKeyframe(ctx, img1, nb1, R1, t1, kf.K, 10.0, np.zeros(0, np.float32),
                                  np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros((0, 3), np.float32),
                                  capacity=cap)
        sidx = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        written, landed = dst.transfer_from(src, kf.R[0], kf.t[0], src_index=sidx)
        torch.cuda.synchronize()
        h = src.state_host()
        ux, uy = src.centres()
        st = oracle_state(h["inv_depth"], h["n"], h["flags"])
        st["last_update"][:] = h["last_update"]
        out, (ox, oy), oidx, o_landed = oracle.disc_transfer(kf.K, kf.K, (320, 240), kf.R[0], kf.t[0], st,
                                                             ux.astype(np.float64), uy.astype(np.float64),
                                                             capacity=cap)
        assert landed == o_landed and written == min(cap, landed) and landed > 250
        assert np.array_equal(sidx.cpu().numpy()[:written], oidx)
        dh = dst.state_host()
        dx, dy = dst.centres()
        assert np.array_equal(dx, ox.astype(np.float32)) and np.array_equal(dy, oy.astype(np.float32))
        assert np.array_equal(dh["inv_depth"], out["inv_depth"].astype(np.float32))
        assert np.array_equal(dh["n"], np.stack([out["nx"], out["ny"], out["nz"]], 1).astype(np.float32))
        assert np.all(dh["flags"] == 0) and np.array_equal(dh["last_update"], out["last_update"])


def test_disc_transfer_many_surfels_matches_oracle_exactly(ctx):
    """More sources than one pass of the transfer workgroup (9,500, over
    4 x 1024 per pass), unusable ones among them (degenerate, uninitialised,
    zero or negative inverse depth); room for all, and room that runs out
    inside the first and inside the second pass: the written set, its order
    and its values equal the oracle's exactly."""
    sg, engine = _mods()
    kf, _ = _scene(width=1280, height=720, seed=79)
    print("case disc transfer 1280x720, 9500 synthetic sources", flush=True)
    rng = np.random.default_rng(79)
    m = 9500
    ux = rng.uniform(0.0, 1279.0, m).astype(np.float32)
    uy = rng.uniform(0.0, 719.0, m).astype(np.float32)
    ids = rng.uniform(0.2, 1.0, m).astype(np.float32)
    ids[rng.choice(m, 60, replace=False)] = 0.0
    ids[rng.choice(m, 60, replace=False)] = -0.5
    g = rng.normal(size=(m, 3)) * [0.3, 0.3, 1.0]
    g[:, 2] = -np.abs(g[:, 2])
    ns = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    flags = np.zeros(m, np.uint32)
    flags[rng.choice(m, 300, replace=False)] |= oracle.DEGENERATE
    flags[rng.choice(m, 300, replace=False)] |= oracle.UNINIT
    src = engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0, ux, uy, ids, ns,
                              flags=flags)
    src.state.last_update.copy_(torch.as_tensor(rng.integers(1, 1000, m).astype(np.int32), device="cuda"))
    img1, nb1, R1, t1 = _as_keyframe_of(kf, 0)
    h = src.state_host()
    st = oracle_state(h["inv_depth"], h["n"], h["flags"])
    st["last_update"][:] = h["last_update"]
    for cap in (m + 10, 2500, 6000):
        dst = engine.DiscKeyframe(ctx, img1, nb1, R1, t1, kf.K, 10.0, np.zeros(0, np.float32),
                                  np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros((0, 3), np.float32),
                                  capacity=cap)
        sidx = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        written, landed = dst.transfer_from(src, kf.R[0], kf.t[0], src_index=sidx)
        torch.cuda.synchronize()
        out, (ox, oy), oidx, o_landed = oracle.disc_transfer(kf.K, kf.K, (1280, 720), kf.R[0], kf.t[0], st,
                                                             ux.astype(np.float64), uy.astype(np.float64),
                                                             capacity=cap)
        assert landed == o_landed and written == min(cap, landed) and landed > 6000, (cap, landed, o_landed)
        assert np.array_equal(sidx.cpu().numpy()[:written], oidx)
        dh = dst.state_host()
        dx, dy = dst.centres()
        assert np.array_equal(dx, ox.astype(np.float32)) and np.array_equal(dy, oy.astype(np.float32))
        assert np.array_equal(dh["inv_depth"], out["inv_depth"].astype(np.float32))
        assert np.array_equal(dh["n"], np.stack([out["nx"], out["ny"], out["nz"]], 1).astype(np.float32))
        assert np.all(dh["flags"] == 0) and np.array_equal(dh["last_update"], out["last_update"])


def test_disc_transfer_batch_equals_one_by_one(ctx):
    """Batched Eq. 10 for discs (three pairs in one launch, one with less
    room than it needs, one without a source-index output) equals the calls
    one by one: counts, centres, state and source indices, bitwise."""
    sg, engine = _mods()
    print("case disc transfer batch of three pairs", flush=True)
    srcs, dsts_ref, dsts_got, poses, caps = [], [], [], [], []
    for k in range(3):
        kf, discs = _scene(seed=73 + k)
        src = engine.DiscKeyframe.from_scene(ctx, kf, discs)
        engine.disc_update(ctx, [src], sg.params(iters=3))
        img1, nb1, R1, t1 = _as_keyframe_of(kf, k)
        cap = 40 if k == 1 else src.count + 10
        z = np.zeros(0, np.float32)
        mk = lambda: engine.DiscKeyframe(ctx, img1, nb1, R1, t1, kf.K, 10.0, z, z, z,
                                         np.zeros((0, 3), np.float32), capacity=cap)
        srcs.append(src)
        dsts_ref.append(mk())
        dsts_got.append(mk())
        poses.append((kf.R[k], kf.t[k]))
        caps.append(cap)
    ref_idx = [torch.full((c,), -2, dtype=torch.int32, device="cuda") for c in caps]
    ref_counts = [d.transfer_from(s, R, t, src_index=i)
                  for d, s, (R, t), i in zip(dsts_ref, srcs, poses, ref_idx)]
    got_idx = [torch.full((c,), -2, dtype=torch.int32, device="cuda") for c in caps]
    sg.sgn_disc_transfer_batch(ctx.handle, [s.item() for s in srcs], [sg.pose_of(R, t) for R, t in poses],
                               [d.item() for d in dsts_got], caps, [d.counts.data_ptr() for d in dsts_got],
                               [i.data_ptr() if k != 2 else 0 for k, i in enumerate(got_idx)])
    torch.cuda.synchronize()
    for k, (d_ref, d_got) in enumerate(zip(dsts_ref, dsts_got)):
        written, landed = (int(v) for v in d_got.counts.cpu().tolist())
        assert (written, landed) == ref_counts[k]
        d_got.count = written
        assert np.array_equal(np.stack(d_got.centres()), np.stack(d_ref.centres()))
        _state_equal(d_got.state_host(), d_ref.state_host())
        if k != 2:
            assert np.array_equal(got_idx[k].cpu().numpy(), ref_idx[k].cpu().numpy())
        else:
            assert np.all(got_idx[k].cpu().numpy() == -2)
    assert ref_counts[1][0] == 40 and ref_counts[1][1] > 40


def test_disc_two_keyframes_chained(ctx):
    """Keyframe 0 optimised, its surfels moved into keyframe 1 (a neighbour
    frame, Eq. 10), rendered there, the empty areas filled, and keyframe 1
    optimised: every stage against the oracle from the device's input."""
    sg, engine = _mods()
    kf, discs = _scene(640, 480, 6, seed=72)
    print("case disc two keyframes 640x480", flush=True)
    k0 = engine.DiscKeyframe.from_scene(ctx, kf, discs, storage="f16")
    engine.disc_update(ctx, [k0], sg.params(iters=8))
    img1, nb1, R1, t1 = _as_keyframe_of(kf, 2)
    k1 = engine.DiscKeyframe(ctx, img1, nb1, R1, t1, kf.K, 10.0, np.zeros(0, np.float32),
                             np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros((0, 3), np.float32),
                             capacity=k0.count + 800, storage="f16")
    written, landed = k1.transfer_from(k0, kf.R[2], kf.t[2])
    assert written == landed and written > 0.9 * k0.count
    k1.render()
    placed, found = k1.place()
    start = k1.state_host()
    engine.disc_update(ctx, [k1], sg.params(iters=8))
    k1.render()
    torch.cuda.synchronize()
    assert placed == found
    dev = k1.state_host()
    res = check_parity(k1, dev, start["inv_depth"], start["n"], None, oracle.OracleParams(iters=8),
                       label="disc keyframe 1", disc=_disc_of(k1), init_flags=start["flags"])
    assert_parity(res, label="disc keyframe 1", max_unstable=0.10)  # measured 0.078
    ux, uy = k1.centres()
    idm, ind = oracle.disc_render(oracle_keyframe(k1), oracle_state(dev["inv_depth"], dev["n"], dev["flags"]),
                                  ux.astype(np.float64), uy.astype(np.float64), 10.0)
    assert np.array_equal(k1.index_out.cpu().numpy(), ind)
    assert (ind >= 0).mean() > 0.8


def test_disc_place_batch_equals_one_by_one(ctx):
    """Batched placement (three launches for several keyframes: one without
    surfels, whose whole lattice qualifies, and one without room) equals
    per-keyframe placement: counts, centres and state, bitwise."""
    sg, engine = _mods()
    print("case disc place batch", flush=True)

    def build():
        dks = []
        for i, (w, h) in enumerate([(320, 240), (200, 130), (320, 240), (320, 240)]):
            kf, discs = _scene(w, h, 3, seed=90 + i, n_holes=4, hole_frac=(0.2, 0.3))
            if i == 2:
                z = np.zeros(0, np.float32)
                dks.append(engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0,
                                               z, z, z, np.zeros((0, 3), np.float32), capacity=500))
            else:
                room = 0 if i == 3 else 300
                dks.append(engine.DiscKeyframe.from_scene(ctx, kf, discs, capacity=discs.ux.size + room))
        for d in dks:
            d.render()
        return dks

    ref = build()
    ref_counts = [d.place(alpha=1.0, beta=2.0) for d in ref]
    got = build()
    got_counts = engine.disc_place(ctx, got, 1.0, 2.0)
    assert got_counts == ref_counts
    assert ref_counts[0][0] > 0 and ref_counts[2][0] > 100
    assert ref_counts[3][0] == 0 and ref_counts[3][1] > 0
    for a, b in zip(ref, got):
        assert a.count == b.count
        (ua, va), (ub, vb) = a.centres(), b.centres()
        assert np.array_equal(ua, ub) and np.array_equal(va, vb)
        _state_equal(a.state_host(), b.state_host())


def test_disc_render_batch_equals_one_by_one(ctx):
    """The batched render (one pass over several keyframes, an empty one in
    the middle, one without an index output) equals per-keyframe renders."""
    sg, engine = _mods()
    print("case disc render batch", flush=True)
    dks = []
    for i, (w, h) in enumerate([(320, 240), (200, 130), (320, 240), (160, 120)]):
        kf, discs = _scene(w, h, 3, seed=80 + i)
        if i == 2:
            dks.append(engine.DiscKeyframe(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, 10.0,
                                           np.zeros(0, np.float32), np.zeros(0, np.float32),
                                           np.zeros(0, np.float32), np.zeros((0, 3), np.float32)))
        else:
            dks.append(engine.DiscKeyframe.from_scene(ctx, kf, discs))
    ref = []
    for d in dks:
        d.render()
        torch.cuda.synchronize()
        ref.append((d.inv_depth_out.cpu().numpy().copy(), d.index_out.cpu().numpy().copy()))
        d.inv_depth_out.fill_(7.0)
        d.index_out.fill_(7)
    items = sg.disc_array([d.item() for d in dks])
    sg.sgn_disc_render_batch(ctx.handle, items, len(dks), [d.inv_depth_out.data_ptr() for d in dks],
                             [d.index_out.data_ptr() if i != 1 else 0 for i, d in enumerate(dks)],
                             ctx.workspace(sg.sgn_disc_render_workspace_bytes(len(dks), items)))
    torch.cuda.synchronize()
    for i, (d, (rd, ri)) in enumerate(zip(dks, ref)):
        assert np.array_equal(d.inv_depth_out.cpu().numpy(), rd)
        if i != 1:
            assert np.array_equal(d.index_out.cpu().numpy(), ri)
        else:
            assert np.all(d.index_out.cpu().numpy() == 7)        # not written
    assert np.all(ref[2][1] == -1)
