"""Element-by-element comparison of device results with the FP64 oracle."""
from __future__ import annotations

import os

import numpy as np

import oracle

# Tolerance of the FP32 form: |delta id| / id <= 1e-4 and normal angle <= 0.01 deg.
REL_TOL = 1e-4
ANGLE_TOL_DEG = 0.01
# flag bits compared between the two sides (the device-only FP64_SOLVE bit is not)
CMP_FLAGS = (oracle.DEGENERATE | oracle.FEW_SAMPLES | oracle.SOLVE_FAIL | oracle.REJECTED |
             oracle.UNINIT)


def angle_deg(n1, n2):
    n1 = np.asarray(n1, np.float64).reshape(-1, 3)
    n2 = np.asarray(n2, np.float64).reshape(-1, 3)
    c = np.linalg.norm(np.cross(n1, n2), axis=1)
    d = np.abs((n1 * n2).sum(1))
    return np.degrees(np.arctan2(c, d))


def oracle_keyframe(dk):
    kf, nb = dk.dequantized_images()
    return oracle.OracleKeyframe(dk.K, kf, nb, dk.R, dk.t, getattr(dk, "patch", 1))


def oracle_state(init_id, init_n, flags=None):
    """The device's float32 starting state, exactly, in double."""
    return oracle.new_state(np.asarray(init_id, np.float32).astype(np.float64),
                            np.asarray(init_n, np.float32).astype(np.float64), flags)


def run_oracle(dk, init_id, init_n, is_new, params: "oracle.OracleParams", subset=None, disc=None,
               init_flags=None):
    """Oracle run from the device's starting state (with its flags, if
    given).  disc = (ux, uy, radius) selects disc surfels (Eq. 4) with those
    centres; is_new is then unused.  Returns (oracle keyframe, final state)."""
    ok = oracle_keyframe(dk)
    return ok, run_oracle_k(ok, init_id, init_n, is_new, params, subset, disc, init_flags)


def run_oracle_k(ok, init_id, init_n, is_new, params: "oracle.OracleParams", subset=None, disc=None,
                 init_flags=None):
    """run_oracle on a prepared oracle keyframe; returns the final state."""
    st = oracle_state(init_id, init_n, init_flags)
    if disc is not None:
        ux, uy, radius = disc
        oracle.disc_optimize(ok, st, np.asarray(ux, np.float32).astype(np.float64),
                             np.asarray(uy, np.float32).astype(np.float64),
                             float(np.float32(radius)), params, subset=subset)
        return st
    if is_new is not None and np.any(is_new):
        if subset is not None:
            # the initialisation reads only non-new surfels, so a subset's
            # starting state is computed exactly by initialising that subset
            oracle.init_from_neighbours(ok, st, is_new, params, subset=subset)
        else:
            oracle.init_from_neighbours(ok, st, is_new, params)
    oracle.optimize(ok, st, params, subset=subset)
    return st


def compare(dev: dict, st: dict, idx=None):
    """Per-surfel errors of device state `dev` (SurfelState.to_host()) against
    oracle state `st`, on indices idx (default: all)."""
    if idx is None:
        idx = np.arange(st["inv_depth"].shape[0])
    idx = np.asarray(idx)
    g_id = dev["inv_depth"][idx].astype(np.float64)
    o_id = st["inv_depth"][idx]
    g_n = dev["n"][idx].astype(np.float64)
    o_n = np.stack([st["nx"][idx], st["ny"][idx], st["nz"][idx]], 1)
    diff = np.abs(g_id - o_id)
    rel = np.where(diff == 0, 0.0, diff / np.maximum(np.abs(o_id), np.finfo(np.float64).tiny))
    ang = angle_deg(g_n, o_n)
    gf = dev["flags"][idx] & CMP_FLAGS
    of = st["flags"][idx].astype(np.uint32) & CMP_FLAGS
    same_flags = gf == of
    ok = (rel <= REL_TOL) & (ang <= ANGLE_TOL_DEG)
    return {
        "idx": idx, "rel": rel, "ang": ang, "same_flags": same_flags, "within": ok,
        "kappa": st["kappa"][idx], "nvalid_dev": dev["nvalid"][idx], "nvalid_or": st["nvalid"][idx],
        "cost_dev": dev["cost"][idx], "cost_or": st["cost"][idx],
    }


# Conditioning probe.  The device computes in float: its warped coordinates,
# samples, normal equations, cost sums and updates carry relative errors of a
# few float ulps, which the condition of each Gauss-Newton step (and, in the
# damped variant, a near-tie in the acceptance test) then amplifies.  The
# probe reruns the oracle with that kind of noise injected (PROBE_EPS,
# relative, on every entry of J^T W J and J^T W r, on the state after every
# accepted step and on the damped variant's acceptance threshold; about 30
# float ulps) under several seeds.  A surfel whose probed results leave the
# tolerance of the unprobed one is not determined to the tolerance at float
# resolution ("unstable").
#
# The bar (assert_parity):
#  1. the probe's unstable fraction is bounded per test by the measured
#     fraction plus a small margin (it depends on the oracle alone);
#  2. every stable surfel is within the tolerance with equal flags (all but
#     a fraction 1 - min_stable, or `slack` surfels in small cases).  A stable
#     surfel that the device leaves out of tolerance is first probed harder,
#     alone (TARGET_TIERS: many more seeds at PROBE_EPS, then at a noise of
#     1e-5, the error bound of a float sum of a few hundred terms): only if
#     the oracle itself moves it out of tolerance under that noise is it
#     unstable after all ("reclassified"; their number is bounded too);
#  3. every unstable surfel ends with a Huber cost (evaluated by the oracle
#     at the device's final state) at most (1 + COST_REL_TOL) times the worst
#     of the oracle's own outcomes for it (unprobed, probed, and, where the
#     device looks worse, the targeted tiers as well), all but `slack` (or
#     one in MAX_COST_VIOLATIONS of the compared surfels in large cases).
# Surfels at the edge of the valid sampling window (reading R16) are a class
# of their own: where a warped sample passes within MARGIN_PX of the window's
# edge on the oracle's path, or the two sides end with different valid-sample
# counts, float position error decides which samples exist, so the cost
# functions themselves differ.  They are counted (bounded by max_edge) and
# kept out of the tolerance and cost checks.
# Reported beside it: the within-tolerance fraction over all compared
# surfels, which no classification touches.
PROBE_EPS = 2e-6
PROBE_SEEDS = (1, 2, 3, 4, 5)
# small cases (at most SMALL_CASE surfels compared) afford more probe runs,
# which catch more of the surfels that are unstable only now and then
SMALL_CASE = 5000
PROBE_SEEDS_SMALL = tuple(range(1, 11))
TARGET_TIERS = ((PROBE_EPS, tuple(range(101, 301))), (1e-5, tuple(range(301, 501))))
COST_REL_TOL = 1e-3
# warped samples closer than this to the edge of the valid window (pixels):
# ten times the float position error of the warp in anchor-local coordinates
MARGIN_PX = 1e-4
MAX_EDGE = 0.03
# reclassified surfels allowed, as a fraction of the compared ones
MAX_RECLASSIFIED = 0.02
# unstable surfels above the cost bound allowed, as a fraction of the compared
# ones (measured: 5 in 500,000 surfel results, see the design notes)
MAX_COST_VIOLATIONS = 1e-4


def as_dev(st: dict) -> dict:
    return {"inv_depth": st["inv_depth"], "n": np.stack([st["nx"], st["ny"], st["nz"]], 1),
            "flags": st["flags"], "nvalid": st["nvalid"], "cost": st["cost"]}


def _probe_runs(okf, init_id, init_n, is_new, params, base, idx, seeds, disc=None, init_flags=None,
                eps=PROBE_EPS):
    """Probe runs on surfels idx: returns (moved mask over idx, final states)."""
    import dataclasses
    moved = np.zeros(idx.size, bool)
    runs = []
    for seed in seeds:
        p = dataclasses.replace(params, perturb=eps, perturb_seed=seed, perturb_parts=0)
        st = run_oracle_k(okf, init_id, init_n, is_new, p, subset=idx, disc=disc, init_flags=init_flags)
        c = compare(as_dev(st), base, idx=idx)
        moved |= ~c["within"] | ~c["same_flags"]
        runs.append(st)
    return moved, runs


def unstable_set(dk, init_id, init_n, is_new, params, base, subset=None, disc=None, init_flags=None):
    """Surfels whose oracle result is not stable under the conditioning
    probe (mask over all surfels), and the probe runs' final states."""
    okf = oracle_keyframe(dk)
    n = base["inv_depth"].shape[0]
    idx = np.arange(n) if subset is None else np.asarray(subset)
    seeds = PROBE_SEEDS if idx.size > SMALL_CASE else PROBE_SEEDS_SMALL
    moved, runs = _probe_runs(okf, init_id, init_n, is_new, params, base, idx, seeds, disc, init_flags)
    bad = np.zeros(n, bool)
    bad[idx] = moved
    return bad, runs


def final_costs(okf, states: dict, idx, huber_k=9.0 / 255.0, disc=None):
    """Oracle Huber cost at each listed surfel's state (id, n)."""
    idx = np.asarray(idx)
    if idx.size == 0:
        return np.zeros(0)
    cost, _ = oracle.costs_at(okf, states["inv_depth"], states["n"], idx, huber_k, disc=disc)
    return cost


class ParityResult(tuple):
    """(compare dict, unstable mask over the compared indices, per-surfel
    cost ratios of the unstable surfels to their worst oracle outcome) plus
    the statistics the bar and the reports use."""
    probe_unstable: float = 0.0   # fraction flagged by the fixed probe seeds
    reclassified: int = 0         # stable surfels the targeted probe moved
    reclassified_tiers: tuple = ()  # of them, per targeted tier
    edge: int = 0                 # surfels of the valid-window edge class
    cost_violations: int = 0      # unstable surfels above (1 + COST_REL_TOL) x worst outcome
    mean_ratio: float = 1.0       # device mean cost / worst oracle run's mean cost (unstable)
    within_all: float = 1.0       # within tolerance over every compared surfel
    within_stable: float = 1.0


def check_parity(dk, dev: dict, init_id, init_n, is_new, params, subset=None, label="", disc=None,
                 init_flags=None):
    """Oracle base run + conditioning probe (+ targeted probes where the
    device disagrees); returns a ParityResult.  disc = (ux, uy, radius) for
    disc surfels; init_flags: the starting flags."""
    okf = oracle_keyframe(dk)
    base = run_oracle_k(okf, init_id, init_n, is_new, params, subset=subset, disc=disc,
                        init_flags=init_flags)
    idx = np.arange(base["inv_depth"].shape[0]) if subset is None else np.asarray(subset)
    c = compare(dev, base, idx=idx)
    seeds = PROBE_SEEDS if idx.size > SMALL_CASE else PROBE_SEEDS_SMALL
    uns, runs = _probe_runs(okf, init_id, init_n, is_new, params, base, idx, seeds, disc, init_flags)
    probe_frac = float(uns.mean()) if uns.size else 0.0
    # the valid-window edge class (R16)
    edge = (base["margin"][idx] < MARGIN_PX) | (c["nvalid_dev"] != c["nvalid_or"])
    uns &= ~edge
    # per-surfel reference runs: (states, mask over idx of the surfels they cover)
    refs = [(base, np.ones(idx.size, bool))] + [(st, np.ones(idx.size, bool)) for st in runs]
    # stable surfels the device leaves out of tolerance: probe them harder,
    # tier by tier
    sus = ~uns & ~edge & (~c["within"] | ~c["same_flags"])
    reclass = [0] * len(TARGET_TIERS)
    searched = np.zeros((len(TARGET_TIERS), idx.size), bool)
    for t, (eps, tseeds) in enumerate(TARGET_TIERS):
        if not sus.any():
            break
        moved, extra = _probe_runs(okf, init_id, init_n, is_new, params, base, idx[sus], tseeds,
                                   disc, init_flags, eps=eps)
        searched[t] |= sus
        pos = np.flatnonzero(sus)
        uns[pos[moved]] = True
        reclass[t] = int(moved.sum())
        refs += [(st, sus.copy()) for st in extra]
        sus[pos[moved]] = False
    # unstable surfels: the device's final cost against the oracle's outcomes
    ratios = np.zeros(0)
    viol = 0
    mean_ratio = 1.0
    dev_n = np.asarray(dev["n"], np.float64)
    dev_states = {"inv_depth": np.asarray(dev["inv_depth"], np.float64), "n": dev_n}
    hk = params.huber_k
    if uns.any():
        ui = np.flatnonzero(uns)
        cg = final_costs(okf, dev_states, idx[ui], hk, disc=disc)

        def worst_of(refs_):
            w = np.full(ui.size, -np.inf)
            for st, cover in refs_:
                m = cover[ui]
                if m.any():
                    w[m] = np.maximum(w[m], final_costs(okf, as_dev(st), idx[ui[m]], hk, disc=disc))
            return w

        worst = worst_of(refs)
        over = cg > worst * (1.0 + COST_REL_TOL) + 1e-15
        # where the device looks worse than every outcome so far, search
        # harder for an oracle outcome as bad, tier by tier (tiers already
        # run for a surfel are not repeated)
        for t, (eps, tseeds) in enumerate(TARGET_TIERS):
            need = over & ~searched[t][ui]
            if not need.any():
                continue
            sel = np.zeros(idx.size, bool)
            sel[ui[need]] = True
            _, extra = _probe_runs(okf, init_id, init_n, is_new, params, base, idx[sel], tseeds,
                                   disc, init_flags, eps=eps)
            worst = np.maximum(worst, worst_of([(st, sel) for st in extra]))
            over = cg > worst * (1.0 + COST_REL_TOL) + 1e-15
        ratios = cg / np.maximum(worst, 1e-300)
        viol = int(over.sum())
        for i in np.flatnonzero(over)[:8]:
            g = idx[ui[i]]
            print(f"  above the cost bound: surfel {g} ratio {ratios[i]:.5f} nvalid {c['nvalid_dev'][ui[i]]}/"
                  f"{c['nvalid_or'][ui[i]]} margin {base['margin'][g]:.3g} kappa {base['kappa'][g]:.3g} "
                  f"rel {c['rel'][ui[i]]:.3g} angle {c['ang'][ui[i]]:.3g}", flush=True)
        run_means = [final_costs(okf, as_dev(st), idx[ui], hk, disc=disc).mean() for st in [base] + runs]
        mean_ratio = float(cg.mean() / max(max(run_means), 1e-30))
    stable = ~uns & ~edge
    res = ParityResult((c, uns | edge, ratios))
    res.edge = int(edge.sum())
    res.probe_unstable = probe_frac
    res.reclassified = sum(reclass)
    res.reclassified_tiers = tuple(reclass)
    res.cost_violations = viol
    res.mean_ratio = mean_ratio
    res.within_all = float(c["within"].mean()) if idx.size else 1.0
    res.within_stable = float(c["within"][stable].mean()) if stable.any() else 1.0
    print(f"{label} {summary(c)} | edge {res.edge} probe-unstable {probe_frac:.4f} "
          f"reclassified {sum(reclass)} {tuple(reclass)} "
          f"within-all {res.within_all:.5f} within-stable {res.within_stable:.5f} "
          f"({int((~c['within'][stable]).sum())} out) unstable cost: max ratio "
          f"{ratios.max() if ratios.size else 1.0:.5f}, over (1+{COST_REL_TOL:g}) {viol}, "
          f"mean ratio {mean_ratio:.4f}", flush=True)
    dump = os.environ.get("PARITY_DUMP_DIR")
    if dump:
        os.makedirs(dump, exist_ok=True)
        name = "".join(ch if ch.isalnum() else "_" for ch in label) or "case"
        np.savez_compressed(os.path.join(dump, f"parity_{name}.npz"), idx=idx, uns=uns,
                            within=c["within"], rel=c["rel"], ang=c["ang"],
                            dev_id=dev["inv_depth"], dev_n=dev["n"], dev_flags=dev["flags"],
                            dev_cost=dev["cost"], or_id=base["inv_depth"], or_flags=base["flags"],
                            or_n=np.stack([base["nx"], base["ny"], base["nz"]], 1),
                            or_kappa=base["kappa"], or_margin=base["margin"], ratios=ratios)
        if os.environ.get("PARITY_DUMP_INPUTS"):
            # the oracle's inputs as well, for replaying the case offline
            # (images as float32: exact for f32 and f16 storage)
            import dataclasses
            kimg, nimg = dk.dequantized_images()
            extra = {} if disc is None else {"disc_ux": np.asarray(disc[0]), "disc_uy": np.asarray(disc[1]),
                                             "disc_r": np.float64(disc[2])}
            np.savez_compressed(os.path.join(dump, f"inputs_{name}.npz"),
                                kf=np.asarray(kimg, np.float32), nbr=np.asarray(nimg, np.float32),
                                K=np.asarray(dk.K, np.float64), R=np.asarray(dk.R), t=np.asarray(dk.t),
                                patch=np.int64(getattr(dk, "patch", 1)), init_id=np.asarray(init_id),
                                init_n=np.asarray(init_n),
                                is_new=np.zeros(0, np.uint8) if is_new is None else np.asarray(is_new),
                                init_flags=np.zeros(0, np.uint32) if init_flags is None else np.asarray(init_flags),
                                subset=np.zeros(0, np.int64) if subset is None else np.asarray(subset),
                                params=np.array([str(dataclasses.asdict(params))]), **extra)
    return res


def assert_parity(res, label="", min_stable=0.999, max_unstable=0.15, slack=1,
                  max_reclassified=MAX_RECLASSIFIED, max_edge=MAX_EDGE):
    """The parity bar (see the probe's description above): a bounded probe
    unstable fraction, stable surfels within tolerance and with equal flags
    (all but a fraction 1 - min_stable of them, or `slack` surfels), a bounded
    number of reclassified surfels, and each unstable surfel's final cost
    within (1 + COST_REL_TOL) of the oracle's worst float-level outcome (all
    but `slack`)."""
    c, uns, ratios = res
    stable = ~uns
    n_st = int(stable.sum())
    assert res.edge <= max(slack, int(max_edge * uns.size)), f"{label}: {res.edge} surfels at the valid-window edge"
    allowed = max(slack, int(np.floor((1.0 - min_stable) * n_st + 1e-9)))
    assert res.probe_unstable <= max_unstable, f"{label}: unstable fraction {res.probe_unstable:.4f}"
    assert int((~c["same_flags"][stable]).sum()) <= allowed, f"{label}: flag mismatches"
    n_out = int((~c["within"][stable]).sum())
    assert n_out <= allowed, f"{label}: {n_out} stable surfels out of tolerance (allowed {allowed}); {summary(c)}"
    n = max(1, uns.size)
    assert res.reclassified <= max(slack, int(max_reclassified * n)), \
        f"{label}: {res.reclassified} surfels reclassified by the targeted probe"
    assert res.cost_violations <= max(slack, int(MAX_COST_VIOLATIONS * n)), \
        f"{label}: {res.cost_violations} unstable surfels above (1 + {COST_REL_TOL}) x the worst oracle outcome"


def assert_render(dk, dev: dict, got):
    """The device's rendered inverse-depth map `got` against the oracle's
    render of the device's own final state."""
    st = oracle_state(dev["inv_depth"], dev["n"], dev["flags"])
    idm, ind = oracle.render(oracle_keyframe(dk), st)
    got = np.asarray(got, np.float64)
    both = (idm > 0) & (got > 0)
    assert (both == (idm > 0)).mean() > 0.9999
    assert (both == (got > 0)).mean() > 0.9999
    # float error of id_u = id_s (1 + sigma), sigma = n.(r_u - r_s) / (n.r_s):
    # a few ulps of id_s, amplified by |r_s| / |n.r_s| for planes seen edge-on
    gw = dk.grid[0]
    i = ind[both]
    S = dk.patch
    fx, fy, cx, cy = dk.K
    rsx = (S * (i % gw) + (S - 1) / 2 - cx) / fx
    rsy = (S * (i // gw) + (S - 1) / 2 - cy) / fy
    n = dev["n"][i].astype(np.float64)
    c = np.abs(n[:, 0] * rsx + n[:, 1] * rsy + n[:, 2])
    amp = np.sqrt(rsx ** 2 + rsy ** 2 + 1) / c
    tol = 2e-6 * (np.abs(idm[both]) + dev["inv_depth"][i]) * np.maximum(1.0, amp)
    assert np.all(np.abs(got[both] - idm[both]) <= tol)


def summary(c: dict) -> str:
    n = c["idx"].size
    return (f"n={n} within={c['within'].mean():.5f} flags_equal={c['same_flags'].mean():.5f} "
            f"rel max={c['rel'].max():.3g} p99={np.percentile(c['rel'], 99):.3g} "
            f"ang max={c['ang'].max():.3g} p99={np.percentile(c['ang'], 99):.3g} "
            f"nvalid_equal={(c['nvalid_dev'] == c['nvalid_or']).mean():.5f}")
