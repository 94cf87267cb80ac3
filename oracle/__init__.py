"""FP64 CPU oracle for sketched Tucker-ALS (Ma & Solomonik, arXiv 2104.01101).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only the test-suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import it.
The product path (the C-ABI library and its Python binding) never calls it,
and it shares no code with that path: the counter-based random generator, the
hashes, the sketches, the solves and the drivers are all written out here
independently, from the paper and from the published generator definition.

Modules
-------
rng      SplitMix64 keyed-counter generator (Steele, Lea & Flood 2014).
sketch   CountSketch / TensorSketch (Sec. 3.1), leverage-score sampling
         (Sec. 3.2), the composite sketch of the range finder (Sec. 5).
solve    rank-constrained least squares (Sec. 4 theorems; Alg. 5).
tucker   Init-RRF (Alg. 3), Sketch-Tucker-ALS (Alg. 4), HOOI (Alg. 1), fit.
cp       CP-ALS (Alg. 2) on the Tucker core, CP-Sketch-Tucker (Alg. 6).
adjoint  sketched mode-n residual and its gradients.

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
from . import rng, sketch, solve, tucker, cp, adjoint  # noqa: F401
