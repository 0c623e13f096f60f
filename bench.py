"""Benchmark of the surfel Gauss-Newton hot path on one MI355X.

A step is one pass of the whole path over one batch: neighbour-plane
initialisation of the new surfels, the fused Gauss-Newton iterations of
every surfel of every keyframe, and the per-pixel inverse-depth render, for
the 64-keyframe mixed-resolution batch (320x240 / 640x480 / 1280x720, 4-12
neighbour frames each, 4x4 surfels, 15 iterations) with images stored as
FP16.  Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line: metric, value (surfel-frame GN updates per second),
the roofline of the fused GN kernel (timed with HIP events on its own
stream), and the FP64 oracle timed on a bounded sample on the host cores.
Beside the metric it reports the other image storages, the plain
single-keyframe form, the depth-only ablation against ground truth, the disc
surfels of Eq. 4 on the same keyframes (radius 10 px: Gauss-Newton kernel and
the whole keyframe step with the empty-area search), and serving latency.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "surfel·frame GN updates/s (% roofline) + p50/p99 keyframe latency, served vs plain"
UNIT = "surfel-frame updates/s"

# The reported roofline: the method's FP32 flops per sample (one pixel of one
# surfel against one neighbour frame in one iteration; warp, divide,
# bilinear value and gradient, residual, Huber weight, chain factor and
# accumulation; an FMA counts 2) against MI355X's published FP32 vector peak.
FLOPS_PER_SAMPLE = 50
FP32_PEAK_TFLOPS = 157.3
# Secondary view, issue slots: the same inventory counted as VALU lane
# operations (an FMA, a compare or a convert counts 1): 44 per sample, against
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operation issues per second.
OPS_PER_SAMPLE = 44
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the first launches of a process run slower while the clock ramps up
    # (about five steps of the batch); ten warm-up steps take 50 ms
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storage", default="f16", choices=["f32", "f16", "u8"])
    ap.add_argument("--keyframes", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip timing the GN kernel with the other image storages")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the depth-only vs full comparison against ground truth")
    ap.add_argument("--no-disc", action="store_true",
                    help="skip the disc-surfel leg (Eq. 4 support, 10 px radius)")
    ap.add_argument("--disc-steps", type=int, default=10)
    ap.add_argument("--no-transfer", action="store_true",
                    help="skip the reference-frame change leg (Eq. 10 with re-gridding)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default plan instead of the autotuned one")
    ap.add_argument("--plan", default="",
                    help="GN mapping TXxTY:K[:P[:X]] (surfels per group, groups per work item, "
                         "persistent grid 0/1, XCD queues or shares 0/1; P and X default to 1), "
                         "e.g. 2x4:2 or 4x4:1:0:1")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of "
                         "known traffic for scaling the HBM counters)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the Poisson serving trace (0: skip the serving leg)")
    ap.add_argument("--serve-sweep", default="500,1000,2000,3000",
                    help="offered loads (req/s) of the shorter serving traces after the 200 req/s one")
    ap.add_argument("--serve-load-seconds", type=float, default=2.0,
                    help="length of each of those traces (0: skip them)")
    return ap.parse_args()


def disc_pixel_counts(ux, uy, radius, width, height):
    """Pixels of each disc inside the image (|u - u_s| < r): the samples per
    surfel and frame of the disc workload."""
    import numpy as np
    R = int(np.ceil(radius)) + 1
    off = np.arange(-R, R + 1)
    out = np.zeros(ux.size, np.int64)
    for dy in off:
        for dx in off:
            x = np.floor(ux.astype(np.float64)) + dx
            y = np.floor(uy.astype(np.float64)) + dy
            d2 = (x - ux) ** 2 + (y - uy) ** 2
            out += ((d2 < radius * radius) & (x >= 0) & (y >= 0) & (x < width) & (y < height))
    return out


def time_transfer(run, n_surfels, written, bytes_per_surfel, what, reps=5):
    """Median of `reps` timed runs (HIP events on the context's stream, which
    is torch's current stream) after one warm-up run; algorithmic bytes:
    each source surfel read and each destination entry written once."""
    import numpy as np
    import torch
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms))
    gbs = n_surfels * bytes_per_surfel / (t * 1e-3) / 1e9
    return {"workload": what, "surfels": int(n_surfels), "written": written(), "ms": t,
            "surfels_per_s": n_surfels / (t * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_surfel": bytes_per_surfel}}


def transfer_leg(ctx, kfs, dks):
    """Eq. 10 with re-gridding: every keyframe's surfels into the tiles of the
    keyframe seen from its first neighbour's pose (same intrinsics, size and
    tile edge), one call per keyframe."""
    import numpy as np
    import torch

    from paper_1910_01997_amd import surfgn as sg
    m = [d.n_surfels for d in dks]
    dsts = [sg.SurfelState.from_arrays(np.zeros(n, np.float32), np.tile(np.float32([0, 0, -1]), (n, 1)))
            for n in m]
    is_new = [torch.zeros(n, dtype=torch.uint8, device="cuda") for n in m]
    src_idx = [torch.empty(n, dtype=torch.int32, device="cuda") for n in m]
    grids = [sg.grid_of(k.K, k.width, k.height, k.patch) for k in kfs]
    poses = [sg.pose_of(k.R[0], k.t[0]) for k in kfs]

    srcs = [d.state.c for d in dks]
    dcs = [t.c for t in dsts]
    new_ptrs = [t.data_ptr() for t in is_new]
    idx_ptrs = [t.data_ptr() for t in src_idx]

    ws = ctx.workspace(sg.sgn_transfer_workspace_bytes(grids))
    # the call's argument arrays, built once (a C caller holds them as arrays)
    a_grids, a_srcs, a_poses = sg.c_array(sg.sgn_grid, grids), sg.c_array(sg.sgn_surfels, srcs), \
        sg.c_array(sg.sgn_pose, poses)
    a_dsts, a_new, a_idx = sg.c_array(sg.sgn_surfels, dcs), sg.c_array(C.c_void_p, new_ptrs), \
        sg.c_array(C.c_void_p, idx_ptrs)

    def run():
        sg.sgn_transfer_surfels_batch(ctx.handle, a_grids, a_srcs, a_poses, a_grids, a_dsts, a_new, a_idx, ws)

    # bytes per surfel: the source state read (id, normal, flags: 20 B), the
    # destination tile written (state 32 B, is_new 1 B, source index 4 B)
    return time_transfer(run, sum(m), lambda: int(sum(int((t == 0).sum()) for t in is_new)),
                         bytes_per_surfel=20 + 37,
                         what=f"{len(dks)} keyframes of 4x4 surfels, each into the tiles of the view of "
                              f"its first neighbour (Eq. 10 and re-gridding), one batched call")


def disc_leg(ctx, kfs, storage, iters, steps, with_ablation):
    """Disc surfels (Eq. 4) on the batch's keyframes: radius 10 px (the
    paper's evaluation setting) on the 14 px lattice with three holes per
    keyframe.  Times the batched disc Gauss-Newton kernel and the whole
    keyframe step (render, empty-area search and placement, Gauss-Newton,
    render)."""
    import numpy as np
    import torch

    from paper_1910_01997_amd import engine
    from paper_1910_01997_amd import surfgn as sg
    from scenegen import make_disc_surfels

    radius = 10.0
    t0 = time.time()
    sets = [make_disc_surfels(k, radius=radius) for k in kfs]
    dks = [engine.DiscKeyframe.from_scene(ctx, k, d, capacity=d.ux.size + d.ux.size // 4 + 64,
                                          storage=storage) for k, d in zip(kfs, sets)]
    torch.cuda.synchronize()
    log(f"disc leg: {sum(d.count for d in dks)} disc surfels on {len(dks)} keyframes "
        f"({time.time() - t0:.1f}s)")
    fields = ("inv_depth", "nx", "ny", "nz", "flags", "cost", "nvalid", "last_update")
    snaps = [([getattr(d.state, f).clone() for f in fields], d.ux.clone(), d.uy.clone(), d.count)
             for d in dks]

    def restore():
        for d, (st, ux, uy, m) in zip(dks, snaps):
            for f, t in zip(fields, st):
                getattr(d.state, f).copy_(t)
            d.ux.copy_(ux)
            d.uy.copy_(uy)
            d.count = m

    prm = sg.params(iters=iters)
    pp = sg.sgn_disc_place_params(1.0, 2.0, sets[0].spacing)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]

    def step():
        # one descriptor array for the step (its counts refreshed after the
        # placement), like a caller that keeps its keyframes resident
        items = engine.disc_items(dks)
        ev[0].record()
        engine.disc_render(ctx, dks, items)
        ev[1].record()
        engine.disc_place(ctx, dks, pp.alpha, pp.beta, pp.spacing, wait=False, items=items)
        ev[2].record()
        counts = torch.stack([d.counts for d in dks]).cpu().numpy()
        for d, c in zip(dks, counts):
            d.count += int(c[0])
        engine.refresh_counts(items, dks)
        engine.disc_update(ctx, dks, prm, items)
        ev[3].record()
        engine.disc_render(ctx, dks, items)
        ev[4].record()
        return counts

    restore()
    step()
    torch.cuda.synchronize()
    wall, phases, gn = [], [], []
    for _ in range(steps):
        restore()
        torch.cuda.synchronize()
        tw = time.perf_counter()
        counts = step()
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - tw)
        gn.append(sg.sgn_last_kernel_ms(ctx.handle))
        phases.append([ev[i].elapsed_time(ev[i + 1]) for i in range(4)])
    ph = np.median(np.array(phases), axis=0)
    gn_ms = float(np.median(gn))
    n_old = sum(s.ux.size for s in sets)
    n_new = int(counts[:, 0].sum())
    # algorithmic samples: initialised surfels (new ones without neighbours
    # carry id 0 and give none) x their disc pixels x frames x iterations
    samples, sframes = 0, 0
    for d in dks:
        h = d.state_host()
        ux, uy = d.centres()
        use = (h["flags"] & sg.FLAG_UNINIT) == 0
        npx = disc_pixel_counts(ux[use], uy[use], radius, d.width, d.height)
        samples += int(npx.sum()) * d.img.n_nbr * iters
        sframes += int(use.sum()) * d.img.n_nbr * iters
    achieved = samples * FLOPS_PER_SAMPLE / (gn_ms * 1e-3) / 1e12
    step_ms = float(np.median(wall)) * 1e3
    out = {
        "workload": f"{len(dks)} keyframes of the batch, disc surfels of radius {radius:g} px on a "
                    f"{sets[0].spacing} px lattice with 3 holes each, {iters} GN iterations, "
                    f"{storage} image storage; step = render, empty-area search and placement "
                    f"(alpha 1, beta 2), Gauss-Newton over old and new surfels, render",
        "surfels": n_old, "placed": n_new, "qualifying": int(counts[:, 1].sum()),
        "gn_ms": gn_ms, "step_ms": step_ms,
        "phase_ms": {"render": float(ph[0]), "place": float(ph[1]), "gn_with_table": float(ph[2]),
                     "render_after": float(ph[3])},
        "surfel_frame_per_s_gn": sframes / (gn_ms * 1e-3),
        "surfel_frame_per_s_step": sframes / (step_ms * 1e-3),
        "samples_per_s": samples / (gn_ms * 1e-3),
        "samples_per_surfel_frame": samples / max(1, sframes),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "flops_per_sample": FLOPS_PER_SAMPLE, "kernel": "disc_gn_kernel"},
    }
    log(f"disc leg: step {step_ms:.3f} ms (render {ph[0]:.3f}, place {ph[1]:.3f}, GN {ph[2]:.3f}, "
        f"render {ph[3]:.3f}); GN kernel {gn_ms:.3f} ms, {samples / (gn_ms * 1e-3):.4e} samples/s, "
        f"flop frac {achieved / FP32_PEAK_TFLOPS:.3f}; placed {n_new}")
    # Eq. 10 for discs: every keyframe's surfels into the keyframe seen from
    # its first neighbour's pose (same intrinsics and size), one call each
    tstates, tux, tuy, tcnt = [], [], [], []
    for d in dks:
        n = max(1, d.count)
        tstates.append(sg.SurfelState.from_arrays(np.zeros(n, np.float32),
                                                  np.tile(np.float32([0, 0, -1]), (n, 1))))
        tux.append(torch.empty(n, dtype=torch.float32, device="cuda"))
        tuy.append(torch.empty(n, dtype=torch.float32, device="cuda"))
        tcnt.append(torch.zeros(2, dtype=torch.int32, device="cuda"))
    tposes = [sg.pose_of(k.R[0], k.t[0]) for k in kfs]

    tsrc = [d.item() for d in dks]
    tdst = [sg.sgn_disc_item(d.img.view.c, tstates[i].c, tux[i].data_ptr(), tuy[i].data_ptr(), 0,
                             float(radius)) for i, d in enumerate(dks)]
    tcap = [t.numel() for t in tux]
    tcnt_ptrs = [t.data_ptr() for t in tcnt]

    # the call's argument arrays, built once (a C caller holds them as arrays)
    a_src, a_poses, a_dst = sg.c_array(sg.sgn_disc_item, tsrc), sg.c_array(sg.sgn_pose, tposes), \
        sg.c_array(sg.sgn_disc_item, tdst)
    a_cap, a_cnt = sg.c_array(C.c_int32, tcap), sg.c_array(C.c_void_p, tcnt_ptrs)

    def transfer():
        sg.sgn_disc_transfer_batch(ctx.handle, a_src, a_poses, a_dst, a_cap, a_cnt)

    out["transfer"] = time_transfer(transfer, sum(d.count for d in dks),
                                    lambda: int(torch.stack(tcnt)[:, 0].sum()),
                                    bytes_per_surfel=20 + 8 + 40,
                                    what=f"{len(dks)} keyframes of disc surfels, each into the view of "
                                         f"its first neighbour (Eq. 10, a disc stays a disc), one batched "
                                         f"call")
    log(f"disc transfer: {out['transfer']}")
    if with_ablation:
        # full vs depth-only against the true planes, on the original discs
        # that see one plane
        def errors():
            rel, ang = [], []
            for d, sset in zip(dks, sets):
                h = d.state_host()
                m = sset.ux.size
                bad = (sg.FLAG_DEGENERATE | sg.FLAG_FEW_SAMPLES | sg.FLAG_SOLVE_FAIL |
                       sg.FLAG_REJECTED | sg.FLAG_UNINIT)
                ok = sset.pure & ((h["flags"][:m] & bad) == 0)
                rel.append(np.abs(h["inv_depth"][:m][ok] / sset.gt_id[ok] - 1))
                g = h["n"][:m][ok].astype(np.float64)
                cr = np.linalg.norm(np.cross(g, sset.gt_n[ok]), axis=1)
                ang.append(np.degrees(np.arctan2(cr, np.abs((g * sset.gt_n[ok]).sum(1)))))
            rel, ang = np.concatenate(rel), np.concatenate(ang)
            return {"surfels": int(rel.size), "depth_rel_err_p50": float(np.median(rel)),
                    "depth_rel_err_p90": float(np.percentile(rel, 90)),
                    "normal_err_deg_p50": float(np.median(ang)),
                    "normal_err_deg_p90": float(np.percentile(ang, 90))}
        abl = {}
        for name, p in (("full", prm), ("depth_only", sg.params(iters=iters, depth_only=True))):
            restore()
            engine.disc_update(ctx, dks, p)
            torch.cuda.synchronize()
            abl[name] = errors()
        out["ablation"] = abl
        log(f"disc ablation: {abl}")
    restore()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(keyframes and streams would shard across GPUs with no exchange). "
              "Run with --gpus 1.", file=sys.stderr, flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1910_01997_amd import engine
    from paper_1910_01997_amd import surfgn as sg
    from scenegen import make_keyframe, spec_for_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    info = sg.sgn_device_info(0)
    log("device", info)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 18          # float32 elements
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy_mib} MiB read + {args.calibrate_copy_mib} MiB written")
        del a, b
    ctx = sg.Context(0)
    iters = 15
    t0 = time.time()
    kfs = [make_keyframe(spec_for_config(2, i), device="cuda") for i in range(args.keyframes)]
    dks = [engine.DeviceKeyframe.from_scene(ctx, k, storage=args.storage) for k in kfs]
    torch.cuda.synchronize()
    log(f"generated {len(dks)} keyframes in {time.time() - t0:.1f}s")
    pool = engine.StatePool(dks)
    init_state = pool.snapshot()
    prm = sg.params(iters=iters)
    surfel_frames = sum(d.n_surfels * d.n_nbr for d in dks) * iters
    samples = sum(d.n_surfels * d.n_nbr * d.patch * d.patch for d in dks) * iters
    plan = None
    if args.plan:
        fields = args.plan.split(":")
        tx, ty = (int(v) for v in fields[0].split("x"))
        pers = int(fields[2]) if len(fields) > 2 else 1
        xq = int(fields[3]) if len(fields) > 3 else 1
        plan = sg.plan(tx, ty, pers, 0, 0, xq, groups=int(fields[1]))
    elif not args.no_autotune:
        # the mapping the autotuner picks for this batch (every tile layout,
        # groups per item, persistent grid or not, XCD queues or shares or not)
        items = sg.batch_array([d.item(render=False, init=False) for d in dks])
        plan = engine.autotune(ctx, items, len(dks), prm)
        log("autotuned plan", plan.as_dict())

    def restore():
        pool.restore(init_state)

    # the batch descriptors point at fixed device buffers: built once, like a
    # caller that keeps its keyframes resident
    step_items = sg.batch_array([d.item() for d in dks])

    def step():
        restore()
        sg.sgn_optimize_batch(ctx.handle, step_items, len(dks), prm, plan)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Each step waits for its GN kernel's end event before the host builds the
    # next one.  Without that wait the host runs several steps ahead, and
    # graph launches queued that far ahead stalled the stream for a few
    # steps (measured: GN windows of 8-16 ms among 4.8 ms ones); the wait
    # costs about 0.03 ms per step.
    kernel_ms = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        kernel_ms.append(sg.sgn_last_kernel_ms(ctx.handle))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = surfel_frames / (ms_per_step * 1e-3)
    gn_ms = float(np.mean(kernel_ms))
    flops = samples * FLOPS_PER_SAMPLE / (gn_ms * 1e-3) / 1e12
    hbm_bytes = compulsory_bytes(dks, iters)
    hbm_gbs = hbm_bytes / (gn_ms * 1e-3) / 1e9
    # the device's results of the timed launches, for the error report
    form_results = {args.storage: form_snapshot(dks, kfs)}
    log(f"steps {args.steps}: {ms_per_step:.3f} ms/step, GN kernel {gn_ms:.3f} ms "
        f"(min {min(kernel_ms):.3f}), {value:.4e} surfel-frame/s, {samples / (gn_ms * 1e-3):.4e} samples/s")

    ablation = None
    if not args.no_ablation:
        # the paper's controlled comparison (depth-only vs full surfel
        # optimisation) on the batch's synthetic scenes: error of the
        # converged surfels against the ground-truth planes, on surfels whose
        # tile lies on one plane
        def gt_errors(dk_list, kf_list=None):
            rel, ang = [], []
            for d, k in zip(dk_list, kf_list if kf_list is not None else kfs):
                st = d.state.to_host()
                S = k.patch
                gh, gw = k.gt_id.shape
                pid = k.kf_plane_id[:gh * S, :gw * S].reshape(gh, S, gw, S)
                pure = (pid == pid[:, :1, :, :1]).all(axis=(1, 3)).reshape(-1)
                bad = (sg.FLAG_DEGENERATE | sg.FLAG_FEW_SAMPLES | sg.FLAG_SOLVE_FAIL |
                       sg.FLAG_REJECTED | sg.FLAG_UNINIT)
                ok = pure & ((st["flags"] & bad) == 0)
                gid = k.gt_id.reshape(-1)
                gn = k.gt_n.reshape(-1, 3)
                rel.append(np.abs(st["inv_depth"][ok] / gid[ok] - 1))
                g = st["n"][ok].astype(np.float64)
                cr = np.linalg.norm(np.cross(g, gn[ok]), axis=1)
                ang.append(np.degrees(np.arctan2(cr, np.abs((g * gn[ok]).sum(1)))))
            rel, ang = np.concatenate(rel), np.concatenate(ang)
            return {"surfels": int(rel.size), "depth_rel_err_p50": float(np.median(rel)),
                    "depth_rel_err_p90": float(np.percentile(rel, 90)),
                    "normal_err_deg_p50": float(np.median(ang)),
                    "normal_err_deg_p90": float(np.percentile(ang, 90))}
        restore()
        engine.update_batch(ctx, dks, prm, plan)
        torch.cuda.synchronize()
        ablation = {"full": gt_errors(dks)}
        restore()
        engine.update_batch(ctx, dks, sg.params(iters=iters, depth_only=True), plan)
        dms = sg.sgn_last_kernel_ms(ctx.handle)
        torch.cuda.synchronize()
        ablation["depth_only"] = gt_errors(dks)
        ablation["depth_only"]["gn_ms"] = dms
        restore()
        engine.update_batch(ctx, dks, sg.params(iters=iters, lm_lambda=1e-2), plan)
        lms = sg.sgn_last_kernel_ms(ctx.handle)
        torch.cuda.synchronize()
        ablation["damped_full"] = gt_errors(dks)
        ablation["damped_full"]["gn_ms"] = lms
        ablation["initial"] = {"depth_rel_err_p50": float(np.median(np.concatenate(
            [np.abs(np.asarray(k.init_id, np.float64).reshape(-1) / k.gt_id.reshape(-1) - 1)
             for k in kfs])))}
        # the same comparison with 8x8 and 16x16 surfels (16 keyframes of the
        # batch's scene recipe): four and sixteen times the pixels, twice and
        # four times the span per surfel
        import dataclasses
        for S in (8, 16):
            kfS = [make_keyframe(dataclasses.replace(spec_for_config(2, i), patch=S), device="cuda")
                   for i in range(16)]
            dkS = [engine.DeviceKeyframe.from_scene(ctx, k, storage=args.storage) for k in kfS]
            poolS = engine.StatePool(dkS)
            initS = poolS.snapshot()
            leg = ablation[f"surfels_{S}x{S}"] = {}
            for name, pS in (("full", sg.params(iters=iters)),
                             ("depth_only", sg.params(iters=iters, depth_only=True)),
                             ("damped_full", sg.params(iters=iters, lm_lambda=1e-2))):
                poolS.restore(initS)
                engine.update_batch(ctx, dkS, pS)
                leg[name] = {"gn_ms": sg.sgn_last_kernel_ms(ctx.handle)}
                torch.cuda.synchronize()
                leg[name].update(gt_errors(dkS, kfS))
            del kfS, dkS, poolS, initS
        log(f"ablation: {ablation}")
        restore()

    forms = None
    if not args.no_precision_forms:
        # the same batch with the other image storages: GN kernel time, the
        # fraction of surfels solved in double, and (in the oracle leg) the
        # error against the oracle
        forms = {}
        for st_name in ("f32", "f16", "u8"):
            if st_name == args.storage:
                forms[st_name] = form_entry(gn_ms, samples, hbm_bytes, form_results[st_name])
                continue
            odks = [engine.DeviceKeyframe.from_scene(ctx, k, storage=st_name) for k in kfs]
            opool = engine.StatePool(odks)
            oinit = opool.snapshot()
            oms = []
            for rep in range(4):
                opool.restore(oinit)
                engine.update_batch(ctx, odks, prm, plan)
                oms.append(sg.sgn_last_kernel_ms(ctx.handle))
            o_ms = float(np.mean(oms[1:]))
            torch.cuda.synchronize()
            form_results[st_name] = form_snapshot(odks, kfs)
            forms[st_name] = form_entry(o_ms, samples, compulsory_bytes(odks, iters), form_results[st_name])
            log(f"{st_name} storage: GN kernel {o_ms:.3f} ms")
            del odks, opool, oinit
        torch.cuda.synchronize()

    discs = None
    transfer = None
    if not args.no_transfer:
        transfer = transfer_leg(ctx, kfs, dks)
        log(f"tile transfer: {transfer}")
        restore()
    if not args.no_disc:
        discs = disc_leg(ctx, kfs, args.storage, iters, args.disc_steps, not args.no_ablation)
        torch.cuda.synchronize()

    plain = None
    if not args.no_plain:
        # the plain single-keyframe form on the same batch, one keyframe at a
        # time, with the plan that suits a single keyframe best: one group of
        # four surfels per wavefront, one wavefront per work item
        plain_plan = sg.plan(2, 2, 0, 0, 0, 0, groups=1)
        restore()
        torch.cuda.synchronize()
        for d in dks[:4]:
            engine.update_plain(ctx, d, prm, plain_plan)
        torch.cuda.synchronize()
        best_s = None
        for _ in range(2):
            restore()
            torch.cuda.synchronize()
            tp = time.perf_counter()
            for d in dks:
                engine.update_plain(ctx, d, prm, plain_plan)
            torch.cuda.synchronize()
            t_s = time.perf_counter() - tp
            best_s = t_s if best_s is None else min(best_s, t_s)
        plain_s = best_s
        plain = {"value": surfel_frames / plain_s, "ms_per_batch": plain_s * 1e3,
                 "form": "per-keyframe calls: init + GN launch (2x2 tiles, one group per "
                         "wavefront, one wavefront per item) + render"}
        log(f"plain form: {plain_s * 1e3:.3f} ms per batch, {surfel_frames / plain_s:.4e} surfel-frame/s")

    traffic = None
    prof = os.path.join(ROOT, "profiles", "gn_kernel_traffic.json")
    if os.path.exists(prof):
        try:
            from paper_1910_01997_amd import build as hb
            rec = json.load(open(prof))
            if rec.get("kernel_source_sha256") == hb.kernel_source_hash() and \
                    rec.get("storage") == args.storage and rec.get("keyframes") == args.keyframes and \
                    same_plan(rec.get("plan"), plan):
                traffic = rec.get("hbm_bytes_per_launch")
        except Exception as e:  # a stale or unreadable summary gives null
            log("traffic summary unusable:", e)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(dks, kfs, iters, args.cpu_seconds)
        errors = form_errors(form_results, kfs, iters)
        cpu["device_error"] = errors
        if forms is not None:
            for k, v in errors.items():
                if k in forms:
                    forms[k]["error_vs_oracle"] = v
    ctx.close()
    n_kf = len(dks)
    n_surfels = int(sum(d.n_surfels for d in dks))
    del dks, kfs, pool, init_state
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    serving = None
    if args.serve_seconds > 0:
        from paper_1910_01997_amd import serve
        # the workload's 200 req/s trace, then shorter traces at higher
        # offered loads on the same resident streams (where continuous
        # batching has several requests to merge, up to saturation)
        sweep = tuple(float(r) for r in args.serve_sweep.split(",") if r) if args.serve_load_seconds > 0 else ()
        serving = serve.serving_benchmark(n_streams=32, rate=200.0, duration=args.serve_seconds + 2.0,
                                          warmup=2.0, storage=args.storage, iters=iters, log=log,
                                          sweep=sweep, sweep_duration=args.serve_load_seconds)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batch of {n_kf} keyframes, mixed 320x240/640x480/1280x720, 4-12 "
                        f"neighbour frames, 4x4 surfels, {iters} GN iterations, "
                        f"{args.storage} image storage, half the surfels initialised from neighbours",
            "keyframes": n_kf, "surfels": n_surfels,
            "surfel_frames_per_step": int(surfel_frames), "samples_per_step": int(samples),
            "image_storage": args.storage, "iterations": iters,
            "plan": plan.as_dict() if plan is not None else "default",
        },
        "roofline": {
            "bound": "alu",
            "achieved": flops,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops / FP32_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "gn_kernel",
            "kernel_ms": gn_ms,
            "flops_per_sample": FLOPS_PER_SAMPLE,
            "samples_per_launch": int(samples),
            "hbm_view": {"achieved_gbs": hbm_gbs, "peak_gbs": HBM_PEAK_GBS,
                         "frac": hbm_gbs / HBM_PEAK_GBS, "bytes_per_launch": int(hbm_bytes),
                         "definition": "every image once and the surfel state read and written, "
                                       "per iteration"},
            "valu_issue_view": issue_view(samples, gn_ms, plan),
        },
        "cpu_baseline": cpu,
        "plain_form": plain,
        "precision_forms": forms,
        "disc_surfels": discs,
        "transfer": transfer,
        "ablation": ablation,
        "serving": serving,
        "device": {"name": info["name"], "arch": info["arch"], "cus": info["compute_units"]},
    }
    print(json.dumps(out), flush=True)


def compulsory_bytes(dks, iters):
    """HBM bytes a launch cannot avoid when nothing stays cached across
    iterations: per iteration every image once (keyframe and neighbours) and
    each surfel's state read and written (32 bytes)."""
    per_it = sum((d.n_nbr + 1) * d.width * d.height * d.kf_img.element_size() + 32 * d.n_surfels
                 for d in dks)
    return per_it * iters


def same_plan(rec_plan, plan):
    """Whether a profile's plan (dict) is the plan the bench ran (None: the
    library's default, 4x4 tiles, one group, one wavefront per item, XCD
    shares)."""
    if not rec_plan:
        return False
    run = plan.as_dict() if plan is not None else {"tiles_x": 4, "tiles_y": 4, "groups": 1, "persistent": 0,
                                                  "xcd_queues": 1}
    return all(int(rec_plan.get(k, -1)) == int(run.get(k, -2))
               for k in ("tiles_x", "tiles_y", "groups", "persistent", "xcd_queues"))


def issue_view(samples, gn_ms, plan=None):
    """VALU issue slots: the 44 lane operations per sample against the issue
    peak, and beside it what the counters measured for this kernel build (the
    summary under profiles/ is used only when its source hash matches)."""
    rate = samples / (gn_ms * 1e-3)
    out = {"ops_per_sample": OPS_PER_SAMPLE, "achieved_tops": rate * OPS_PER_SAMPLE / 1e12,
           "peak_tops": VALU_PEAK_TOPS, "frac": rate * OPS_PER_SAMPLE / 1e12 / VALU_PEAK_TOPS,
           "measured_valu_insts_per_wave_sample": None, "measured_issue_frac": None}
    prof = os.path.join(ROOT, "profiles", "gn_kernel_counters.json")
    if os.path.exists(prof):
        try:
            from paper_1910_01997_amd import build as hb
            rec = json.load(open(prof))
            if rec.get("kernel_source_sha256") == hb.kernel_source_hash() and same_plan(rec.get("plan"), plan):
                per = rec["valu_insts_per_wave_sample"]
                out["measured_valu_insts_per_wave_sample"] = per
                out["measured_issue_frac"] = rate * per / 1e12 / VALU_PEAK_TOPS
        except Exception as e:  # a stale or unreadable summary gives null
            log("counter summary unusable:", e)
    return out


# keyframes of the batch whose surfels the error report samples
ERROR_KEYFRAMES = (0, 21, 42, 63)
ERROR_SURFELS = 2000


def form_snapshot(dks, kfs):
    """Host copy of the device's results for the error report: the states of
    the sampled keyframes (with the images they sampled, exactly) and the
    fraction of all surfels whose 3x3 system was solved in double."""
    from paper_1910_01997_amd import surfgn as sg
    fp64 = 0
    total = 0
    for d in dks:
        fl = d.state.flags.cpu().numpy()
        fp64 += int(((fl & sg.FLAG_FP64_SOLVE) != 0).sum())
        total += fl.size
    sample = {}
    for j in ERROR_KEYFRAMES:
        if j < len(dks):
            d = dks[j]
            sample[j] = {"state": d.state.to_host(), "images": d.dequantized_images(),
                         "K": d.K, "R": d.R, "t": d.t, "patch": d.patch}
    return {"fp64_solve_frac": fp64 / max(1, total), "sample": sample}


def form_entry(ms, samples, hbm_bytes, res):
    return {"gn_ms": ms, "flop_frac": samples * FLOPS_PER_SAMPLE / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
            "hbm_frac": hbm_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "fp64_solve_frac": res["fp64_solve_frac"]}


class _HostKeyframe:
    def __init__(self, rec, images=None):
        self.K, self.R, self.t, self.patch = rec["K"], rec["R"], rec["t"], rec["patch"]
        self._img = images if images is not None else rec["images"]

    def dequantized_images(self):
        return self._img


def form_errors(form_results, kfs, iters):
    """Device results against the oracle per image storage, on ERROR_SURFELS
    random surfels of each of ERROR_KEYFRAMES: the parity bar's figures
    (within tolerance over all sampled surfels and over the stable ones, the
    probe's unstable fraction, surfels reclassified by the targeted probe,
    unstable surfels above the cost bound) with the oracle on the exact
    images the kernel sampled; and, for f16 / u8, the error against the
    oracle run on the float32 images (the data-quantisation effect)."""
    import numpy as np

    import oracle
    from tests.parity import check_parity, compare, run_oracle_k, oracle_keyframe

    rng = np.random.default_rng(777)
    out = {}
    prm = oracle.OracleParams(iters=iters)
    for name, res in form_results.items():
        agg = {"surfels": 0, "within_all": 0, "stable": 0, "within_stable": 0, "probe_unstable": 0,
               "reclassified": 0, "cost_violations": 0, "edge": 0}
        rel, ang, qrel, qang, qwithin = [], [], [], [], []
        for j, rec in res["sample"].items():
            k = kfs[j]
            n = rec["state"]["inv_depth"].size
            sub = np.sort(rng.choice(n, size=min(ERROR_SURFELS, n), replace=False))
            hk = _HostKeyframe(rec)
            r = check_parity(hk, rec["state"], k.init_id, k.init_n, k.is_new, prm, subset=sub,
                             label=f"bench {name} kf{j}")
            c, uns, _ = r
            agg["surfels"] += sub.size
            agg["within_all"] += int(c["within"].sum())
            agg["stable"] += int((~uns).sum())
            agg["within_stable"] += int(c["within"][~uns].sum())
            agg["probe_unstable"] += int(round(r.probe_unstable * sub.size))
            agg["reclassified"] += r.reclassified
            agg["cost_violations"] += r.cost_violations
            agg["edge"] += r.edge
            rel.append(c["rel"])
            ang.append(c["ang"])
            if name != "f32":
                # the same starting state on the float32 images
                f32 = (k.kf_image.double().cpu().numpy(), k.nbr_images.double().cpu().numpy())
                okf = oracle_keyframe(_HostKeyframe(rec, images=f32))
                st = run_oracle_k(okf, k.init_id, k.init_n, k.is_new, prm, subset=sub)
                q = compare(rec["state"], st, idx=sub)
                qrel.append(q["rel"])
                qang.append(q["ang"])
                qwithin.append(q["within"])
        rel, ang = np.concatenate(rel), np.concatenate(ang)
        e = {"surfels": agg["surfels"], "keyframes": list(res["sample"].keys()),
             "within_tolerance_all": agg["within_all"] / agg["surfels"],
             "within_tolerance_stable": agg["within_stable"] / max(1, agg["stable"]),
             "probe_unstable_frac": agg["probe_unstable"] / agg["surfels"],
             "reclassified": agg["reclassified"], "cost_bound_violations": agg["cost_violations"],
             "valid_window_edge": agg["edge"],
             "rel_p50": float(np.percentile(rel, 50)), "rel_p99": float(np.percentile(rel, 99)),
             "rel_max": float(rel.max()), "angle_deg_p50": float(np.percentile(ang, 50)),
             "angle_deg_p99": float(np.percentile(ang, 99)), "angle_deg_max": float(ang.max()),
             "fp64_solve_frac": res["fp64_solve_frac"]}
        if qrel:
            qrel, qang, qwithin = np.concatenate(qrel), np.concatenate(qang), np.concatenate(qwithin)
            e["vs_float32_image_oracle"] = {
                "within_tolerance_all": float(qwithin.mean()),
                "rel_p50": float(np.percentile(qrel, 50)), "rel_p99": float(np.percentile(qrel, 99)),
                "angle_deg_p50": float(np.percentile(qang, 50)),
                "angle_deg_p99": float(np.percentile(qang, 99))}
        out[name] = e
        log(f"error vs oracle, {name}: {e}")
    return out


def _oracle_rate(dks, kfs, iters, budget_s, rng):
    """Oracle surfel-frame updates per second on random surfels of every
    keyframe (random keyframe order), about budget_s seconds of work: the
    first keyframe's rate sizes the per-keyframe sample."""
    import numpy as np

    import oracle

    done_sf = 0
    spent = 0.0
    used = []
    quota = None            # surfel-frame updates per keyframe
    for j in rng.permutation(len(dks)):
        d, k = dks[j], kfs[j]
        kimg, nimg = d.dequantized_images()
        okf = oracle.OracleKeyframe(d.K, kimg, nimg, d.R, d.t, d.patch)
        st = oracle.new_state(np.asarray(k.init_id, np.float32).astype(np.float64),
                              np.asarray(k.init_n, np.float32).astype(np.float64))
        prm = oracle.OracleParams(iters=iters)
        m = d.n_surfels
        take = 2048 if quota is None else int(quota // (d.n_nbr * iters))
        take = max(256, min(m, take))
        sub = np.sort(rng.choice(m, size=take, replace=False)).astype(np.int32)
        t = time.perf_counter()
        oracle.init_from_neighbours(okf, st, k.is_new, prm, subset=sub)
        oracle.optimize(okf, st, prm, subset=sub)
        dt = time.perf_counter() - t
        spent += dt
        done_sf += take * d.n_nbr * iters
        used.append(f"kf{j}:{take}/{m}")
        if quota is None:
            rate = take * d.n_nbr * iters / max(dt, 1e-6)
            quota = max(0.0, budget_s - spent) * rate / max(1, len(dks) - 1)
        if spent >= 1.5 * budget_s:
            break
    return done_sf / spent, done_sf, spent, used


def cpu_baseline(dks, kfs, iters, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same batch,
    timed on all host threads (the reported value) and on one thread (a
    quarter of the budget)."""
    import os as _os

    import numpy as np

    import oracle

    threads = oracle.max_threads()
    rng = np.random.default_rng(12345)
    value, done_sf, spent, used = _oracle_rate(dks, kfs, iters, budget_s, rng)
    oracle.set_threads(1)
    try:
        v1, sf1, sp1, used1 = _oracle_rate(dks, kfs, iters, budget_s / 4, np.random.default_rng(54321))
    finally:
        oracle.set_threads(threads)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": value, "unit": UNIT, "cores": int(threads), "kind": "oracle",
            "sample": f"{len(used)} keyframes of the batch, random surfels of each sized to a "
                      f"{budget_s:.0f} s budget ({done_sf} surfel-frame updates, {spent:.1f} s); "
                      + ",".join(used[:8]),
            "single_thread": {"value": v1, "cores": 1,
                              "sample": f"{len(used1)} keyframes, {sf1} surfel-frame updates, {sp1:.1f} s"},
            "host": {"cpu_model": cpu_model, "nproc": _os.cpu_count()}}


if __name__ == "__main__":
    main()
