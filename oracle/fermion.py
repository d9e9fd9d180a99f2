"""Fermion operators acting on occupation bit strings.

Follows the occupation representation of a Slater determinant as a bit string
(Ch. 2, "Representation of the basis"): single-particle state i is bit i of an
integer mask. Creation and annihilation carry the anticommutation sign
(-1)^(number of occupied states with a lower index). This is the consistent
reading of the chapter's examples (creators are ordered by ascending index);
with it, annihilating the second state of the paper's string 110101 gives
-100101, and the two-body example keeps its overall minus sign.
"""


def phase_below(mask, i):
    """(-1)^(number of occupied states with index < i)."""
    return -1 if bin(mask & ((1 << i) - 1)).count("1") & 1 else 1


def annihilate(mask, i):
    """a_i |mask>  ->  (sign, new_mask), or None if state i is empty."""
    if not (mask >> i) & 1:
        return None
    return phase_below(mask, i), mask & ~(1 << i)


def create(mask, i):
    """a+_i |mask>  ->  (sign, new_mask), or None if state i is occupied."""
    if (mask >> i) & 1:
        return None
    return phase_below(mask, i), mask | (1 << i)


def apply_ops(mask, ops):
    """Apply a product of operators to |mask>, rightmost first.

    ``ops`` is a sequence of ('+', i) / ('-', i) read left to right as
    written, e.g. [('+', a), ('+', b), ('-', d), ('-', c)] for
    a+_a a+_b a_d a_c. Returns (sign, new_mask) or None.
    """
    sign = 1
    for kind, i in reversed(ops):
        r = create(mask, i) if kind == "+" else annihilate(mask, i)
        if r is None:
            return None
        s, mask = r
        sign *= s
    return sign, mask


def from_string(bits):
    """Paper-style bit string (leftmost character = state 1) -> mask."""
    return sum(1 << k for k, ch in enumerate(bits) if ch == "1")


def to_string(mask, n):
    return "".join("1" if (mask >> k) & 1 else "0" for k in range(n))
