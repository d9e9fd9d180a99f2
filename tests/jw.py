"""Jordan-Wigner Fock-space matrices: an independent construction for pins.

Fermion operators on n modes as sparse 2^n x 2^n matrices built from Kronecker
products (a_i = 1 x ... x 1 x sigma^- x Z x ... x Z, with a sign string over
the modes of lower index). Fock index bit i = occupation of mode i. This
shares nothing with the bit-string phase code of the oracle; it is used only
to pin it.
"""
import numpy as np
import scipy.sparse as sp

_I = sp.identity(2, format="csr")
_Z = sp.csr_matrix(np.diag([1.0, -1.0]))
_LOWER = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))   # |0><1|


def annihilators(n):
    """List of a_i (i = 0..n-1) as CSR matrices on the 2^n Fock space.

    Kronecker order puts mode n-1 as the most significant factor, so that the
    Fock index has bit i = occupation of mode i.
    """
    ops = []
    for i in range(n):
        m = sp.identity(1, format="csr")
        for k in reversed(range(n)):      # most significant factor first
            if k > i:
                f = _I
            elif k == i:
                f = _LOWER
            else:
                f = _Z
            m = sp.kron(m, f, format="csr")
        ops.append(m)
    return ops


def element(op, row, col):
    return float(op[row, col])
