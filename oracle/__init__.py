"""CPU oracle for the DACP central-eigenvalue path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 implementations written from the paper (Guan & Zhang,
"Dual application of Chebyshev polynomial for efficiently computing thousands
of central eigenvalues in many-spin systems").  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import this package; the
product library never calls it and shares no code with it.

Modules:
  hamiltonian    -- Pauli-term Hamiltonian, dense element formula, matrix-free apply
  _native        -- own Householder + implicit QL and cyclic Jacobi (C, OpenMP)
  jordan_wigner  -- closed-form spectrum of the open transverse-field Ising chain
  chebyshev      -- T_k closed form, filter recurrence, evolution basis
  subspace       -- S, P projection and the App. C generalised eigen-solve
  spectral       -- Lanczos bound, kernel-polynomial moments, window choice
  philox         -- Philox4x32-10 + Box-Muller start states
  central        -- the plain definition: dense full diagonalisation + selection
  mlp            -- the learned window's regression network: forward, backward, Adam
  acceptance     -- the acceptance rule for computed Ritz pairs (quadratic residual bound)
  levels         -- gap ratios of consecutive level spacings
"""
