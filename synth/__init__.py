"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates *inputs only*: scan trajectories (per-view source /
detector-centre / pixel-step vectors), random ellipsoid-and-cube phantoms,
their exact analytic line integrals, and the counting noise that turns line
integrals into measured data.  It contains none of the reconstruction
method's arithmetic (no projector, no back-projector, no filter, no solver).
"""

from .geometry import (  # noqa: F401
    CONFIGS, ScanConfig, trajectory, perturb_geometry, volume_axes, evaluation_mask, masked_rel_error,
    PAPER_SHAPED, PAPER_SHAPED_NZ, PAPER_SHAPED_Z_RANGE, helix_trajectory,
)
from .phantom import (  # noqa: F401
    Phantom,
    random_phantom,
    voxelize,
    line_integrals,
    add_noise,
    make_dataset,
    crop,
    line_integrals_clipped,
    crop_dataset,
)
