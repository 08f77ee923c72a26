"""Seeded synthetic inputs for the StereoVAE hot path.

Draws random stereo pairs shaped like driving scenes (planar Voronoi disparity
cells, forward-warped right view), network weights and reparameterisation
noise.  It holds none of the matching or refinement arithmetic, so both the
CPU oracle's tests and the GPU path's tests and bench can take their inputs
from here without sharing any of the method's code.
"""
from .stereo import (  # noqa: F401
    PRESETS,
    StereoPair,
    gen_pair,
    gen_shift_pair,
    gen_preset,
    he_init_params,
    gen_eps,
)
