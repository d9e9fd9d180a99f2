"""fotci: factorized on-the-fly configuration interaction on MI355X (gfx950).

The Hamiltonian-times-vector product of the factorized M-scheme CI method,
with its setup (basis, jumps), adjoint and Lanczos driver, as hand-written
HIP kernels behind a C-ABI shared library (libfotci.so). This package holds
the thin ctypes binding (``fotci``) and the seeded input recipes
(``inputs``). Importing the package does not load the library; the binding
loads it on first use and raises if it has not been built.
"""
__all__ = ["inputs"]
