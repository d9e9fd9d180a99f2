"""Angular-momentum observables in the forms the library takes.

``j_squared(two_j)`` gives J^2 = (J_p + J_n)^2 of the valence nucleons as a
one- plus two-body operator in J-coupled form (App. A, eq. hamdef): the
one-body part is j(j+1) on every m-state of an orbit, and the two-body part
2 j_1 . j_2 = J^2 - j_1^2 - j_2^2 is diagonal in normalised pair states of good
J, V_J(ab,ab) = J(J+1) - j_a(j_a+1) - j_b(j_b+1) (like-particle pairs a <= b,
even J only when a == b; proton-neutron pairs for every a, b). Decoupled with
``fotci.decouple_tbme`` and applied with apply_H it gives <psi|J^2|psi>.
"""
import numpy as np


def j_squared(two_j):
    """(eps, pp, nn, pn): single-particle energies per orbit and J-coupled
    element lists (a, b, c, d, two_J, V) of J^2."""
    n = len(two_j)
    jj = [0.25 * tj * (tj + 2) for tj in two_j]   # j(j+1) from 2j
    like, pn = [], []
    for a in range(n):
        for b in range(n):
            for tJ in range(abs(two_j[a] - two_j[b]), two_j[a] + two_j[b] + 1, 2):
                v = 0.25 * tJ * (tJ + 2) - jj[a] - jj[b]
                pn.append((a, b, a, b, tJ, v))
                if a < b or (a == b and tJ % 4 == 0):
                    like.append((a, b, a, b, tJ, v))
    return np.array(jj), like, list(like), pn
