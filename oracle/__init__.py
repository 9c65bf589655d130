"""CPU oracle for the C* Pfaffian-sign hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 implementations of what the GPU path computes, written from
the paper's definitions and shared with the GPU code in nothing but the seeded
input generators.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything from here; the product path never does.

Modules:
  dirac     -- ctypes wrapper of dirac_oracle.c (the operator D, Q = g5 D)
  dense     -- dense D and Q, eigenvalues, Kramers pairing, inertia
  pfaffian  -- Pfaffian of a complex antisymmetric matrix (pivoted reduction),
               brute-force expansion for tiny matrices
  sign      -- W_sgn from dense inertia and from the Pfaffian, step A of the paper
  lanczos   -- eigenvalues of Q by Lanczos on Q^2, for lattices too large for dense work
  evenodd   -- even-odd blocks of D, the Schur complement D_hat and the factor W_eo
  nn        -- forward/backward of the gauge-covariant preconditioner network
"""
