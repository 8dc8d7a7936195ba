"""FP64 CPU oracle for the SkipGS training hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the HIP path; both are fed
from the seeded input generators, which hold none of the method's arithmetic.

The oracle is a plain, slow statement of what the method computes:

* ``render``  - 3D Gaussian density and covariance factorisation (Sec. 3,
  Eqs. 1-2), EWA projection (Eq. 3), front-to-back compositing, in depth
  order, of the Gaussians that cover a pixel (Eqs. 4-5), SH colour, tile
  binning as the order-defining step.
* ``loss``    - the photometric loss (1-lambda) L1 + lambda (1 - SSIM), Eq. 6.
* ``gate``    - SkipGS backward gating, Algorithm 1 with Eqs. 7-13.
* ``adam``    - the Adam update the optimiser applies when backward runs.
* ``grad``    - gradients of the above as the exact derivative of the
  discrete-decision forward (torch autograd in float64).

Readings of points the paper leaves open are module-level constants and
arguments; each is documented where it is used.
"""
from . import render, loss, gate, adam, grad  # noqa: F401
