"""CPU oracle for the factorized on-the-fly CI hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library
computes, written from the method's definitions (the M-scheme basis of
proton x neutron Slater determinants, second-quantised operator action on
bit strings, the one- plus two-body Hamiltonian, Lanczos with full
reorthogonalisation) in float64.

Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import or run anything in this package. The GPU library never calls
it, and the two share no code: the oracle takes plain numpy arrays and never
imports the library package.

Modules:
  fermion      -- creation/annihilation on bit strings and the fermion phase
  basis        -- m-states, Slater determinants, sectors, basis index
  hamiltonian  -- direct operator action: dense H, matvec, jumps, densities
  lanczos      -- float64 Lanczos with full reorthogonalisation, tridiagonal eig
  fast         -- ctypes front-end of cmatvec.c (same definitions, in C with
                  OpenMP) for workloads too large for the Python loops
"""
