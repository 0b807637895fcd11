"""FP64 CPU oracle for data-parallel brick volume rendering and sort-last compositing.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only the test suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the GPU path (no kernels, headers,
tables or helpers); the two meet only through the seeded inputs of ``synth``.

What it computes, and where the paper fixes it:

* Sort-last compositing of one RGBA-z fragment per pixel per rank, sorted by
  depth and merged front to back (paper section 2.1, Data Parallel Rendering;
  section 5.1.1, Compositing: every fragment carries RGBA *and* depth, so no
  fixed compositing order is needed).  ``composite.py``.
* The per-rank local render that produces those fragments.  The paper leaves it
  to "any device that computes colour and depth" (section 5.1.2, Rendering), so
  its definition here is a reading: fixed-step emission-absorption quadrature on
  an eye-anchored sample lattice, trilinear sampling with clamp-to-edge at the
  global domain, a 1D RGBA transfer function, per-brick ray/box clipping,
  early ray termination and depth = brick entry distance.  ``render.py``.
* Macrocell value ranges and transfer-function majorants used by empty-space
  skipping, from their plain definitions (exact min/max; table coordinates in
  FP64).  ``macrocell.py``.
* Gradients of an L2 image loss with respect to the density grid and the
  transfer-function table.  ``grad.py``.
* An independent loop-based brute-force renderer for tiny inputs.  ``brute.py``.
* Iso-surface fragments: an opaque, shaded iso-surface of the trilinear field
  found on the same sample lattice and mixed with the emission-absorption march
  (the paper renders iso-surfaces through the same pipeline: Fig. 1c, Fig. 3c,
  Fig. 4).  ``iso.py``.
* Data-parallel volumetric path tracing (delta tracking, next-event estimation
  with ratio-tracked shadow rays, isotropic scattering; the rays a rank cannot
  finish are forwarded to the rank holding the content they meet next: sections
  2.2 and 5.2, Fig. 7), with the counter-based generator Philox4x32-10 restated
  from its published definition.  ``path.py``, ``rng.py``.
* Deep (multi-fragment) partial frames of ranks with non-convex data and their
  per-pixel merge (section 5.1.1 allows several fragments per pixel; section 2.1
  and Fig. 6 on non-convex partitions).  ``deep.py``.

Pins (tests marked ``not gpu``): closed-form transmittance of a constant volume,
O(dt^2) convergence to the analytic integral of an affine field, brute force on
tiny grids, the split invariant (one brick == k bricks with ghosts, composited),
composite closed forms and permutation invariance, iso-surface closed forms on
trilinear-exact fields, second-order convergence of the hit point, the split
invariant with the surface, deep frames of interleaved
(non-convex) partitions reproducing the unsplit image, numpy min/max for macrocell
ranges, finite differences and torch.autograd (FP64) for gradients.
"""

from .render import (  # noqa: F401
    RenderParams, camera_basis, camera_rays, clip_box, trilinear, tf_lookup,
    march_rays, march_rays_thresholds, render_brick, render_brick_thresholds, render_image,
)
from .composite import composite  # noqa: F401
from .deep import FID_RANK, composite_deep, deep_frame  # noqa: F401
from .path import PathParams, render_path, trace_paths  # noqa: F401
from .iso import IsoParams, iso_class_ambiguous, iso_classes, march_rays_iso, render_brick_iso, render_image_iso, trilinear_grad  # noqa: F401
from .macrocell import (  # noqa: F401
    entry_decision_ambiguous, entry_range, macrocell_grid, macrocell_ranges, majorants, tf_coord,
)
from .grad import loss_and_grad, forward_image  # noqa: F401
