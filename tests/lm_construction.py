"""A keyframe on which one damped Gauss-Newton step changes the mean Huber
cost by a chosen relative amount (numpy only; calls neither the oracle nor
the device library).

The neighbour frames see the keyframe shifted sideways (R = I, t = (1/32, 0,
0), fx = 64, so a pixel at inverse depth id lands at x + 2 id), rows are
constant, and the neighbour image is piecewise linear in x.  Surfel 1 (the
4 x 4 tile at columns 4..7) is fronto-parallel at id = 0.625, so its pixels
sample the neighbours at x + 1.25 with residual -1/128 on a slope of 1/128.
The depth-only step moves every sample by 1/(1 + lambda) pixel: columns 4-6
land on the same slope (residual about zero), column 7 crosses into a cell
whose slope s9 is chosen so that the mean cost over the 48 valid samples
changes by the factor 1 + eps.  Every image value except the knot f(10) and
every warp quantity is a dyadic rational, so float arithmetic reproduces the
construction up to the rounding of f(10) and of the damped division.
"""
from __future__ import annotations

import math

import numpy as np

W, H, S = 32, 8, 4
K = (64.0, 64.0, 16.0, 4.0)
N_FRAMES = 3
ID0 = 0.625
SURFEL = 1                      # tile (1, 0): columns 4..7, rows 0..3
SLOPE = 1.0 / 128.0


def build(eps: float, lam: float):
    """Images, poses and starting state for a cost ratio of 1 + eps after one
    depth-only step damped by lam.  Returns a dict with kf (H, W), nbrs
    (N, H, W), R (N, 3, 3), t (N, 3), init_id (gw*gh), init_n (gw*gh, 3) and
    the expected candidate inverse depth of SURFEL."""
    mu = 1.0 / (1.0 + lam)                      # sample shift of the damped step (pixels)
    r0 = -SLOPE
    # residual of columns 4-6 after the step, then column 7's for the ratio
    r_near = r0 + SLOPE * mu
    r7 = math.sqrt((1.0 + eps) * 4.0 * r0 * r0 - 3.0 * r_near * r_near)
    # column 7 samples at 8.25 + mu, in cell [9, 10); its residual there is
    # f(9) - g(7) + s9 (mu - 0.75) = -0.25/128 + s9 (mu - 0.75)
    s9 = (r7 + 0.25 * SLOPE) / (mu - 0.75)
    f = np.full(W, 0.5)
    for k in range(5, 10):
        f[k] = 0.5 + (k - 5) * SLOPE
    f[10:] = f[9] + s9
    g = np.full(W, 0.5)
    for x in range(4, 8):
        g[x] = 0.5 + (x - 2.75) * SLOPE      # f(x + 1.25) - r0
    kf = np.tile(g, (H, 1))
    nbrs = np.tile(f, (N_FRAMES, H, 1))
    R = np.tile(np.eye(3), (N_FRAMES, 1, 1))
    t = np.tile([1.0 / 32.0, 0.0, 0.0], (N_FRAMES, 1))
    gw, gh = W // S, H // S
    init_id = np.full(gw * gh, ID0)
    init_n = np.tile([0.0, 0.0, -1.0], (gw * gh, 1))
    return {"kf": kf, "nbrs": nbrs, "R": R, "t": t, "init_id": init_id, "init_n": init_n,
            "candidate_id": ID0 + 0.5 * mu, "r0": r0, "r_near": r_near, "r7": r7}


def huber(r, k=9.0 / 255.0):
    a = abs(r)
    return 0.5 * r * r if a <= k else k * a - 0.5 * k * k


def mean_cost_ratio(case) -> float:
    """The candidate's mean Huber cost over the current one, evaluated from
    the construction's residuals (every sample stays valid)."""
    c0 = 4 * huber(case["r0"])
    c1 = 3 * huber(case["r_near"]) + huber(case["r7"])
    return c1 / c0
