"""Angular-momentum coupling for J-coupled two-body matrix elements.

Test infrastructure like the rest of ``oracle/``: plain and slow.

- ``clebsch_gordan``: Racah's closed form for (j1 m1, j2 m2 | J M) with exact
  rational arithmetic (Fractions of integer factorials), converted to float at
  the end. All angular momenta are passed doubled (2j, 2m).
- ``pair_state``: the normalised J-coupled two-particle state of App. A
  ("The Hamiltonian and other operators in second quantization", eq. Adagger
  and the normalised pair operator), (1/zeta_ab) sum CG a+_{m_a} b+_{m_b}|0>,
  expanded on ordered two-particle bit strings by direct fermion operator
  action (``fermion.apply_ops``).
- ``decouple``: m-scheme matrices V_pp, V_nn, V_pn (the layouts the library
  takes) from J-coupled elements, as <ab|V|cd> = sum_J sum_M <ab|ab;JM>
  V_J(ab,cd) <cd;JM|cd> with the pair states above (eq. hamdef: V_J is the
  matrix element between normalised two-body states of good J; for a
  proton-neutron pair the state is the product of distinguishable particles,
  with no zeta factor).
- ``j_squared_direct``: J^2 = (J_p + J_n)^2 as an interaction built from the
  single-particle j_z, j_+ and j_- matrices and normal ordering, with no
  coupling coefficients at all.
- ``j_squared_coupled``: the same operator written as J-coupled elements,
  V_J(ab,ab) = J(J+1) - j_a(j_a+1) - j_b(j_b+1), single-particle energy
  j(j+1).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .basis import m_states
from .fermion import apply_ops


def _fact(n):
    if n < 0:
        raise ValueError
    return math.factorial(n)


def clebsch_gordan(tj1, tm1, tj2, tm2, tJ, tM):
    """(j1 m1, j2 m2 | J M) for doubled arguments (Racah's formula)."""
    if tm1 + tm2 != tM:
        return 0.0
    if tJ < abs(tj1 - tj2) or tJ > tj1 + tj2 or (tj1 + tj2 + tJ) % 2:
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    # integer arguments
    a = (tJ + tj1 - tj2) // 2
    b = (tJ - tj1 + tj2) // 2
    c = (tj1 + tj2 - tJ) // 2
    d = (tj1 + tj2 + tJ) // 2 + 1
    pre = Fraction((tJ + 1) * _fact(a) * _fact(b) * _fact(c), _fact(d))
    pre *= (_fact((tJ + tM) // 2) * _fact((tJ - tM) // 2) * _fact((tj1 - tm1) // 2) * _fact((tj1 + tm1) // 2)
            * _fact((tj2 - tm2) // 2) * _fact((tj2 + tm2) // 2))
    s = Fraction(0)
    for k in range(0, c + (tj1 + tj2) + 1):
        args = [k, c - k, (tj1 - tm1) // 2 - k, (tj2 + tm2) // 2 - k,
                (tJ - tj2 + tm1) // 2 + k, (tJ - tj1 - tm2) // 2 + k]
        if min(args) < 0:
            continue
        den = 1
        for x in args:
            den *= _fact(x)
        s += Fraction((-1) ** k, den)
    return float(s) * math.sqrt(float(pre))


def _orbit_states(ms, orb):
    return [i for i, m in enumerate(ms) if m[0] == orb]


def pair_state(ms, a, b, tJ, tM, same_species=True):
    """Normalised |ab; J M> as {(i, k): amplitude} over ordered m-state pairs.

    same_species: {(i, k): amp} with i < k on one species' bit strings (the
    state a+_i a+_k |0>); otherwise (i proton m-state, k neutron m-state) for
    the product p+_i n+_k |0>."""
    zeta = math.sqrt(2.0) if (same_species and a == b) else 1.0
    out = {}
    for i in _orbit_states(ms, a):
        for k in _orbit_states(ms, b):
            cg = clebsch_gordan(ms[i][1], ms[i][2], ms[k][1], ms[k][2], tJ, tM)
            if cg == 0.0:
                continue
            if not same_species:
                out[(i, k)] = out.get((i, k), 0.0) + cg
                continue
            res = apply_ops(0, [("+", i), ("+", k)])   # a+_i a+_k |0>, rightmost first
            if res is None:
                continue
            sign, mask = res
            lo, hi = min(i, k), max(i, k)
            # the ordered state a+_lo a+_hi |0>
            ref = apply_ops(0, [("+", lo), ("+", hi)])
            amp = sign * ref[0] * cg / zeta
            out[(lo, hi)] = out.get((lo, hi), 0.0) + amp
    return out


def _pairs(ns):
    return [(a, b) for a in range(ns) for b in range(a + 1, ns)]


def decouple(two_j, pp=(), nn=(), pn=(), parity=None):
    """m-scheme (v_pp, v_nn, v_pn) from J-coupled elements.

    pp, nn: iterables of (a, b, c, d, two_J, V) with orbit indices a <= b,
    c <= d; pn: (a, b, c, d, two_J, V) with a, c proton orbits and b, d
    neutron orbits. Each (ab, cd) is given once; (cd, ab) is implied."""
    ms = m_states(two_j, parity)
    ns = len(ms)
    pl = _pairs(ns)
    pidx = {p: k for k, p in enumerate(pl)}
    npairs = len(pl)
    out = dict(v_pp=np.zeros((npairs, npairs)), v_nn=np.zeros((npairs, npairs)), v_pn=np.zeros((ns * ns, ns * ns)))

    def add(key, elems, same):
        for (a, b, c, d, tJ, v) in elems:
            for tM in range(-tJ, tJ + 1, 2):
                bra = pair_state(ms, a, b, tJ, tM, same)
                ket = pair_state(ms, c, d, tJ, tM, same)
                for (i, k), x in bra.items():
                    r = pidx[(i, k)] if same else i * ns + k
                    for (p, q), z in ket.items():
                        col = pidx[(p, q)] if same else p * ns + q
                        out[key][r, col] += x * v * z
                        if (a, b) != (c, d):
                            out[key][col, r] += x * v * z

    add("v_pp", pp, True)
    add("v_nn", nn, True)
    add("v_pn", pn, False)
    return out


def _jmats(ms):
    ns = len(ms)
    jz = np.zeros((ns, ns))
    jp = np.zeros((ns, ns))
    for i, (o, tj, tm, _) in enumerate(ms):
        jz[i, i] = tm / 2.0
        for k, (o2, tj2, tm2, _) in enumerate(ms):
            if o2 == o and tm2 == tm - 2:   # j+ |m-1> = sqrt(j(j+1) - (m-1)m) |m>
                j, m = tj / 2.0, tm2 / 2.0
                jp[i, k] = math.sqrt(j * (j + 1) - m * (m + 1))
    return jz, jp, jp.T.copy()


def j_squared_direct(two_j, parity=None):
    """J^2 of all nucleons as an interaction dict (eps per orbit, v_pp, v_nn, v_pn)."""
    ms = m_states(two_j, parity)
    ns = len(ms)
    jz, jp, jm = _jmats(ms)
    pl = _pairs(ns)
    npairs = len(pl)
    # coefficient of a+_al a+_be a_de a_ga (unrestricted) in sum_{A,B} O_A O_B
    def w(al, be, ga, de):
        return jz[al, ga] * jz[be, de] + 0.5 * (jp[al, ga] * jm[be, de] + jm[al, ga] * jp[be, de])
    v = np.zeros((npairs, npairs))
    for r, (al, be) in enumerate(pl):
        for c, (ga, de) in enumerate(pl):
            v[r, c] = w(al, be, ga, de) - w(be, al, ga, de) - w(al, be, de, ga) + w(be, al, de, ga)
    vpn = np.zeros((ns * ns, ns * ns))
    for al in range(ns):
        for be in range(ns):
            for ga in range(ns):
                for de in range(ns):
                    vpn[al * ns + be, ga * ns + de] = (2 * jz[al, ga] * jz[be, de] + jp[al, ga] * jm[be, de]
                                                       + jm[al, ga] * jp[be, de])
    eps = np.array([(tj / 2.0) * (tj / 2.0 + 1) for tj in two_j])
    return dict(eps_p=eps, eps_n=eps.copy(), v_pp=v, v_nn=v.copy(), v_pn=vpn)


def j_squared_coupled(two_j):
    """J^2 as J-coupled elements: (eps, pp, nn, pn) lists for ``decouple``."""
    n = len(two_j)
    jj = [(tj / 2.0) * (tj / 2.0 + 1) for tj in two_j]
    pp = []
    pn = []
    for a in range(n):
        for b in range(n):
            for tJ in range(abs(two_j[a] - two_j[b]), two_j[a] + two_j[b] + 1, 2):
                J = tJ / 2.0
                val = J * (J + 1) - jj[a] - jj[b]
                pn.append((a, b, a, b, tJ, val))
                if a < b or (a == b and (tJ // 2) % 2 == 0):
                    pp.append((a, b, a, b, tJ, val))
    return np.array(jj), pp, list(pp), pn
