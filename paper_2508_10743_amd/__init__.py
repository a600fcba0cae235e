"""DARC hot path for MI355X (gfx950): HIP kernels behind a C ABI (libdarc.so).

DARC is the coordinate-descent groupwise atlas construction of "An Efficient
Model-Driven Groupwise Approach for Atlas Construction" (arXiv 2508.10743).
The Python layer (:mod:`.darc`) only marshals torch tensors into the C ABI
declared in ``include/darc.h``.
"""

from .darc import (  # noqa: F401
    Cohort,
    DarcError,
    SweepParams,
    adam_step,
    atlas_update,
    center,
    diffusion,
    exp_svf,
    exp_svf_bwd,
    gauss_smooth,
    lib,
    sim_grad,
    warp3d,
    warp3d_bwd,
)
