"""FP64 CPU oracle for LocalPower -- test infrastructure, not part of the product.

Plain, slow, obviously correct NumPy float64 code written from the paper
(Algorithm 1 "LocalPower", the OPT and sign-fixing alignments of Section 3, the
projection distance of Definition 1, and the operational update rule of the
appendix).  It shares no code with the HIP library and never imports it.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import,
call or execute anything in this package.

Pins (checked by the CPU test-suite against mathematics, not against itself):
  * localpower with p = 1 equals an independent distributed power iteration;
  * identical partitions reduce LocalPower to single-node power iteration;
  * sign-fixing equals the brute-force minimum over all 2^k sign matrices;
  * OPT satisfies the closed form of the Procrustes lemma and undoes
    injected rotations exactly;
  * the cyclic Jacobi eigensolver equals LAPACK and the truth on tiny d;
  * Ritz values at convergence equal the top eigenvalues of M;
  * the rank-r iterate converges at lambda_{r+1} / lambda_k (subspace iteration);
  * eta has a closed form on axis-aligned partitions;
  * the OPT residual error equals a brute-force minimum over rotations and
    2 sin(theta_max / 2);
  * orth is the thin QR with a positive diagonal R (upper-triangular Q^T Y,
    Q R = Y, equal to plain Gram-Schmidt), also where LAPACK's own R has
    negative diagonal entries;
  * the orthonormalised Gaussian start meets the initial-angle bound of the
    appendix (Lemma "initial") at the stated rates.
Qualitative behaviours (error floors growing with p, decay reaching DPI
precision, vanilla instability) are checked as trends only: parity unpinned
for the exact values of p > 1 runs on large workloads, which only the
oracle-vs-GPU comparison covers.
"""

from .localpower import (  # noqa: F401
    partition_setup,
    orth,
    local_multiply,
    sign_fix,
    opt_matrix,
    localpower,
    dpi,
    power_iteration,
    sin_theta,
    projection_distance,
    ritz,
    eta,
    residual_error,
)
from .jacobi import jacobi_eig  # noqa: F401
from .truth import top_k  # noqa: F401
