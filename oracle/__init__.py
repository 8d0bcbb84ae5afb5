"""CPU oracle for the Wilson-Dirac operator and the CG solve on D^dagger D.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls into it, links against it or shares code with it; it exists to prove
the GPU results right.

Everything here is plain NumPy in complex128 (float64), written to be read
against the paper rather than to be fast:

* ``gamma``     -- the chiral Euclidean gamma matrices and the spin
                   projectors P^{+-mu} = 1 +- gamma_mu of eq. (1);
* ``wilson``    -- D of eq. (1) with full 4x4 spin matrices and np.roll
                   neighbours, its adjoint, D^dagger D, and a dense matrix of
                   D filled by explicit site loops;
* ``freefield`` -- the closed forms for U = 1 (momentum-space operator and
                   an FFT solve of D^dagger D);
* ``solvers``   -- textbook CG on D^dagger D and an emulation of the mixed
                   precision "Residual Guided CG" of Algorithm 1;
* ``force``     -- the gradient of a real loss with respect to the links
                   (projected spinor outer products);
* ``lowprec``   -- the storage formats of the low-precision inner solve
                   (binary32, and binary16 / bfloat16 with a per-site scale),
                   as roundings of float64 values;
* ``evenodd``   -- the even-odd (Schur complement) form of D x = b: the
                   even-site operator D_hat = A - K_eo K_oe / A, the reduced
                   source, the odd-site reconstruction and the solve.

Conventions: canonical arrays as in ``synth`` (links ``[T,Z,Y,X,4,3,3]``,
spinors ``[T,Z,Y,X,4,3]``, direction mu = 0..3 <-> x,y,z,t), periodic
boundaries in all four directions.

Every oracle function is pinned by tests in ``tests/test_oracle_*.py``
against something other than itself: a dense matrix built by brute force,
closed forms of the free field and of pure-gauge links, gamma-5 hermiticity,
gauge and translation covariance, dense linear solves, and finite
differences of the operator.  None is "parity unpinned".
"""

from . import gamma, wilson, freefield, solvers, force, lowprec, evenodd  # noqa: F401
