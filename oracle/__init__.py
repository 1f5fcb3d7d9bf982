"""CPU FP64 oracle for the weakly singular Burton-Miller (WSBM) Nystrom system.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute anything in this package; only the tests, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
it has its own geometry, its own kernel formulas (SciPy/AMOS Hankel functions,
or mpmath for brute force) and its own dense LU (LAPACK via SciPy).

Contents (each function cites the passage of the paper it follows):
  geometry  -- nodes, outward normals, trapezoidal weights, curvature (Sec. II)
  wsbm      -- layer-potential entries S, D, D*, N_k0-N_k1 with the one-point
               corrected diagonal; the 2x2 block system of Eq. (3)/(5); the
               plane-wave right-hand side; far field; dense LU solve
  mie       -- closed forms for a dielectric circle: separation-of-variables
               (Mie) solution and the eigenvalues of each layer potential
  brute     -- the same entries evaluated with mpmath at 30 digits (tiny N)
  shape     -- the backscatter intensity of a Fourier-parametrised boundary and
               its derivative with respect to the coefficients, by Richardson
               central differences of J or of the pieces of the adjoint identity
  idecomp   -- the interpolative decomposition that picks a box's skeleton
               (Sec. III): Householder QR with column pivoting, relative rank
               rule, interpolation matrix from one triangular solve

Readings where the paper is silent (fundamental solution, normal-derivative
definitions, the meaning of q, the one-point correction constants, the
multi-scatterer coupling) are listed in the module docstrings; every one of
them is pinned by a closed form in tests/test_oracle_pins.py; the shape
derivative's readings are in oracle/shape.py, pinned in
tests/test_oracle_shape_pins.py; the ID's in oracle/idecomp.py, pinned in
tests/test_oracle_id_pins.py.
"""
