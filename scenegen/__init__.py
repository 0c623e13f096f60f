"""Seeded synthetic piecewise-planar scenes: the inputs shared by the oracle
and the HIP path.

This package draws scene parameters and renders images; it holds none of the
surfel method's arithmetic (no plane-induced warp, no bilinear sampling, no
residuals, Jacobians or solves).  Every random number is drawn here and handed
to both sides as plain arrays.
"""
from .scene import (  # noqa: F401
    Keyframe,
    SceneSpec,
    make_keyframe,
    make_config,
    spec_for_config,
    batch_specs,
    stream_specs,
    rotation_about,
)
from .discs import DiscSet, lattice, make_disc_surfels  # noqa: F401,E402
