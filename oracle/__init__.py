"""FP64 CPU oracle for the log-polar hyperbolic Radon transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library.

Two oracles live here, both written from the paper (Nikitin, Andersson,
Carlsson, Duchkov, "Fast hyperbolic Radon transform represented as
convolutions in log-polar coordinates"):

* `direct`   - the definition, eq. (1) (label Rhdef): summation over
               hyperbolas with cubic interpolation in time (Section 5), and
               its exact transpose.
* `logpolar` - the discrete log-polar method of Sections 2-4, step by step in
               the paper's order (resampling with the 1/(2 sqrt y) weight,
               B-spline smearing, FFT convolution with the kernel spectrum,
               B-spline interpolation back to (tau, q)), and its transpose.

Supporting modules: `geometry` (rescaling, sector placement, coordinate maps,
lattice sizing), `bspline` (cubic cardinal B-spline), `kernel` (the spectrum of
zeta by quadrature), `ista` (soft-thresholding iterations of Section 3),
`demultiple` (Radon-domain multiple attenuation of Section 6), `split`
(the transform cut into parts in time and slowness, Sections 4 and 5).
All arithmetic is float64.  Readings of points where the paper is silent or
garbled are stated in each function's docstring.

Every function is pinned by a test against something other than itself
(tests/test_oracle_*.py): closed forms, invariants, brute force on tiny grids
or an independent computation, each chosen so that a plausible slip fails
it.  The kernel multiplier's B-spline division along each axis is pinned by
a narrow Gaussian's closed form on the C2 grid, and the trapezoid end
weights of the smear weight (first and last trace, last time sample) by the
lattice mass against an adaptive quadrature and by a Gaussian on the last
trace against direct summation.  Quantities with no paper value to check
against (reconstruction SNR of the iterations, the quality of multiple
attenuation) are reported, not pinned.
"""
from . import bspline, geometry, kernel, logpolar, direct, ista, demultiple, split  # noqa: F401
