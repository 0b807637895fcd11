"""Seeded synthetic inputs for the data-parallel volume renderer and its oracle.

This package builds *inputs only*: scalar volumes (anisotropic Gaussian blobs,
per-voxel white noise, value-noise fBm), 256-entry RGBA transfer-function
tables sampled from control points, pinhole cameras, k-d brick partitions with
ghost layers, and synthetic partial RGBA+depth frames.  It holds none of the
rendering or compositing arithmetic, so both the CPU oracle and the GPU path
consume exactly the bytes it produces.

The paper renders scientific datasets (DNS turbulence, thunderstorm,
aircraft Q-criterion; Introduction, Fig. 3, Fig. 8).  None of them is
available, so these generators stand in for them: smooth features, large
transparent regions, turbulence-like noise, non-cubic shapes and FP16 storage.
"""

from .volume import (  # noqa: F401
    BlobSet, make_blobs, perturb_blobs, blobs_field, white_noise, fbm_field, make_volume_small,
    make_volume_large,
)
from .scene import (  # noqa: F401
    Camera, Brick, make_tf, orbit_camera, fibonacci_cameras, kd_split,
    even_split, brick_ghosts, extract_brick, pixel_subset,
)
from .frames import synthetic_frames  # noqa: F401
from .configs import CONFIGS, Config, get_config  # noqa: F401
