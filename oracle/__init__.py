"""FP64 CPU oracle for the per-frame Gauss-Newton solvers (test infrastructure).

This package is test infrastructure only: tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library never
does, and the oracle imports nothing from the product.

It is a plain, slow, readable restatement of what the solvers compute:

* ``graph``     -- deformation-graph construction (farthest-point nodes,
                   4-nearest-node binding, 8-nearest-node edges).
* ``image``     -- silhouette contour, exact Euclidean distance transform,
                   Gaussian blur, cubic-convolution sampling.
* ``decisions`` -- the once-per-frame integer decisions (depth-buffer
                   visibility, contour vertices, silhouette direction signs),
                   taken in float32 by a fixed recipe so they can be matched
                   bit for bit.
* ``nonrigid``  -- residuals, explicit sparse Jacobian, normal equations,
                   Cholesky or Jacobi-PCG solve, Gauss-Newton loop (float64).
* ``vertex``    -- the paper's own per-vertex non-rigid stage: data terms,
                   spatial smoothness, edge length, velocity and acceleration
                   priors with Table 1 material weights; Gauss-Newton (float64).
* ``so3``       -- rotation exponential / logarithm.

Every result the paper pins only qualitatively is pinned in ``tests/`` by
finite differences, closed forms, invariants and brute force.
"""
