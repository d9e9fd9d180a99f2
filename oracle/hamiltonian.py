"""Direct second-quantised action of the one- plus two-body Hamiltonian.

The Hamiltonian is the M-scheme form of the paper's standard one- plus
two-body operator (App. A, "The Hamiltonian and other operators in second
quantization", eq. hamdef), with the proton-neutron part written on product
states (Ch. 2, "Representation of the Hamiltonian": pp and nn forces act on
one species with the other a spectator, pn forces act on both):

  H = sum_i eps_p[orb i] n_i(p) + sum_i eps_n[orb i] n_i(n)
    + sum_{a<b, c<d} V_pp[(ab),(cd)] p+_a p+_b p_d p_c
    + sum_{a<b, c<d} V_nn[(ab),(cd)] n+_a n+_b n_d n_c
    + sum_{a,b,c,d}  V_pn[(a b),(c d)] (p+_a p_c)(n+_b n_d)

Every function here builds its result by applying these operator strings to
bit strings with ``fermion.apply_ops`` -- no jump tables, no factorisation --
so it can be checked against the paper by eye.

Jumps (Ch. 2, "Representation of the Hamiltonian"; Ch. 8, "Opbundles and
optypes") are the nonzero results of one species' operator strings on that
species' SDs, recorded as (src SD, dst SD, phase, label) in canonical
(dst, src, label) order.
"""
from __future__ import annotations

import numpy as np

from .fermion import apply_ops


def pair_list(ns):
    return [(a, b) for a in range(ns) for b in range(a + 1, ns)]


def _eps_mstate(b, inter, sp):
    key = "eps_%s_mstate" % sp
    if key in inter:
        return np.asarray(inter[key], dtype=np.float64)
    eps = np.asarray(inter["eps_%s" % sp], dtype=np.float64)
    return np.array([eps[m[0]] for m in b.ms])


def _occ(mask, ns):
    return [i for i in range(ns) if (mask >> i) & 1]


def _two_body_allowed(ms):
    """For each pair (c<d): list of (row pair index, a, b) conserving 2M and parity."""
    pl = pair_list(len(ms))
    key = [(ms[a][2] + ms[b][2], ms[a][3] * ms[b][3]) for a, b in pl]
    by_key = {}
    for r, k in enumerate(key):
        by_key.setdefault(k, []).append(r)
    return pl, {c: [(r, pl[r][0], pl[r][1]) for r in by_key[key[c]]] for c in range(len(pl))}


def column(b, inter, pmask, nmask):
    """H|pmask,nmask> as a list of ((pmask', nmask'), amplitude) terms."""
    ms = b.ms
    ns = len(ms)
    ep, en = _eps_mstate(b, inter, "p"), _eps_mstate(b, inter, "n")
    pocc, nocc = _occ(pmask, ns), _occ(nmask, ns)
    out = [((pmask, nmask), float(sum(ep[i] for i in pocc) + sum(en[i] for i in nocc)))]
    pl = pair_list(ns)
    pidx = {p: k for k, p in enumerate(pl)}
    for sp, occ, v in (("p", pocc, inter["v_pp"]), ("n", nocc, inter["v_nn"])):
        mask = pmask if sp == "p" else nmask
        for i1 in range(len(occ)):
            for i2 in range(i1 + 1, len(occ)):
                c, d = occ[i1], occ[i2]
                col = pidx[(c, d)]
                for r in np.nonzero(v[:, col])[0]:
                    a, bb = pl[r]
                    res = apply_ops(mask, [("+", a), ("+", bb), ("-", d), ("-", c)])
                    if res is None:
                        continue
                    s, m2 = res
                    tgt = (m2, nmask) if sp == "p" else (pmask, m2)
                    out.append((tgt, s * float(v[r, col])))
    vpn = inter["v_pn"]
    for c in pocc:
        for d in nocc:
            col = c * ns + d
            for row in np.nonzero(vpn[:, col])[0]:
                a, bb = divmod(int(row), ns)
                rp = apply_ops(pmask, [("+", a), ("-", c)])
                if rp is None:
                    continue
                rn = apply_ops(nmask, [("+", bb), ("-", d)])
                if rn is None:
                    continue
                out.append(((rp[1], rn[1]), rp[0] * rn[0] * float(vpn[row, col])))
    return out


def dense_h(b, inter):
    """The full H matrix in the basis, H[t, s] = <t|H|s>."""
    h = np.zeros((b.dim, b.dim))
    for s, (pm, nm) in enumerate(b.states()):
        for (tp, tn), amp in column(b, inter, pm, nm):
            t = b.index(tp, tn)
            if t is None:
                raise AssertionError("H left the basis: M or parity not conserved")
            h[t, s] += amp
    return h


def apply_h(b, inter, x):
    """y = H x by direct action (column by column)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(b.dim)
    for s, (pm, nm) in enumerate(b.states()):
        if x[s] == 0.0:
            continue
        for (tp, tn), amp in column(b, inter, pm, nm):
            y[b.index(tp, tn)] += amp * x[s]
    return y


def densities(b, g, x):
    """Label-wise contractions <g|O_label|x> for every operator string of H.

    Returns dict with
      d_eps_p[orbit] = <g| sum_{i in orbit} n_i(p) |x>   (same for n),
      d_v_pp[(ab),(cd)] = <g| p+_a p+_b p_d p_c |x>     (same for nn),
      d_v_pn[(a b),(c d)] = <g| (p+_a p_c)(n+_b n_d) |x>,
    i.e. the derivative of <g|H|x> with respect to each array entry of the
    interaction (unsymmetrised: (r,c) and (c,r) are separate entries).
    """
    ms = b.ms
    ns = len(ms)
    n_orb = 1 + max(m[0] for m in ms)
    pl, allowed = _two_body_allowed(ms)
    npairs = len(pl)
    pidx = {p: k for k, p in enumerate(pl)}
    out = dict(d_eps_p=np.zeros(n_orb), d_eps_n=np.zeros(n_orb),
               d_v_pp=np.zeros((npairs, npairs)), d_v_nn=np.zeros((npairs, npairs)),
               d_v_pn=np.zeros((ns * ns, ns * ns)))
    g = np.asarray(g, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    for s, (pm, nm) in enumerate(b.states()):
        xs = x[s]
        if xs == 0.0:
            continue
        pocc, nocc = _occ(pm, ns), _occ(nm, ns)
        gs = g[s]
        for i in pocc:
            out["d_eps_p"][ms[i][0]] += gs * xs
        for i in nocc:
            out["d_eps_n"][ms[i][0]] += gs * xs
        for sp, occ, key in (("p", pocc, "d_v_pp"), ("n", nocc, "d_v_nn")):
            mask = pm if sp == "p" else nm
            for i1 in range(len(occ)):
                for i2 in range(i1 + 1, len(occ)):
                    c, d = occ[i1], occ[i2]
                    col = pidx[(c, d)]
                    for (r, a, bb) in allowed[col]:
                        res = apply_ops(mask, [("+", a), ("+", bb), ("-", d), ("-", c)])
                        if res is None:
                            continue
                        t = b.index(res[1], nm) if sp == "p" else b.index(pm, res[1])
                        out[key][r, col] += res[0] * g[t] * xs
        for c in pocc:
            for d in nocc:
                for a in range(ns):
                    rp = apply_ops(pm, [("+", a), ("-", c)])
                    if rp is None:
                        continue
                    for bb in range(ns):
                        if ms[a][2] + ms[bb][2] != ms[c][2] + ms[d][2]:
                            continue
                        if ms[a][3] * ms[bb][3] != ms[c][3] * ms[d][3]:
                            continue
                        rn = apply_ops(nm, [("+", bb), ("-", d)])
                        if rn is None:
                            continue
                        t = b.index(rp[1], rn[1])
                        out["d_v_pn"][a * ns + bb, c * ns + d] += rp[0] * rn[0] * g[t] * xs
    return out


def one_body_densities(b, g, x):
    """M-scheme one-body transition densities between two vectors of basis b:

      rho_p[a, c] = <g| p+_a p_c |x>,   rho_n[a, c] = <g| n+_a n_c |x>

    (Ch. 5, "One-body density matrices": the proton-neutron densities from
    which the J-reduced ones are coupled). An operator that changes Jz or
    parity leads out of the basis, so only entries with m_a = m_c and equal
    parities can be nonzero. For g = x = psi (unit norm) the diagonal holds
    the occupations of the m-states (Ch. 4, "Single-particle occupations").
    """
    ms = b.ms
    ns = len(ms)
    rho = dict(p=np.zeros((ns, ns)), n=np.zeros((ns, ns)))
    g = np.asarray(g, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    for s, (pm, nm) in enumerate(b.states()):
        xs = x[s]
        if xs == 0.0:
            continue
        for sp, mask in (("p", pm), ("n", nm)):
            for c in _occ(mask, ns):
                for a in range(ns):
                    if ms[a][2] != ms[c][2] or ms[a][3] != ms[c][3]:
                        continue
                    res = apply_ops(mask, [("+", a), ("-", c)])
                    if res is None:
                        continue
                    t = b.index(res[1], nm) if sp == "p" else b.index(pm, res[1])
                    rho[sp][a, c] += res[0] * g[t] * xs
    return rho["p"], rho["n"]


def jumps(b, species, src_subset=None):
    """Jump lists of one species over its kept SDs (or only from ``src_subset``).

    Returns dict with 'two_body' and 'one_body', each an int64 array of rows
    (src, dst, phase, label) sorted by (dst, src, label):
      two-body label = row_pair * n_pairs + col_pair for p+_a p+_b p_d p_c,
        with (a<b) the row pair and (c<d) the column pair; every (a<b) that
        conserves 2M and parity is tried, the diagonal included.
      one-body label = a * ns + c for p+_a p_c, every a and c tried; the
        destination SD must belong to the kept SDs of the species.
    """
    ms = b.ms
    ns = len(ms)
    sds = b.p_sds if species == "p" else b.n_sds
    rank = {m: i for i, m in enumerate(sds)}
    pl, allowed = _two_body_allowed(ms)
    npairs = len(pl)
    pidx = {p: k for k, p in enumerate(pl)}
    two, one = [], []
    srcs = range(len(sds)) if src_subset is None else sorted(int(i) for i in src_subset)
    for src in srcs:
        mask = sds[src]
        occ = _occ(mask, ns)
        for i1 in range(len(occ)):
            for i2 in range(i1 + 1, len(occ)):
                c, d = occ[i1], occ[i2]
                col = pidx[(c, d)]
                for (r, a, bb) in allowed[col]:
                    res = apply_ops(mask, [("+", a), ("+", bb), ("-", d), ("-", c)])
                    if res is None:
                        continue
                    two.append((src, rank[res[1]], res[0], r * npairs + col))
        for c in occ:
            for a in range(ns):
                res = apply_ops(mask, [("+", a), ("-", c)])
                if res is None or res[1] not in rank:
                    continue
                one.append((src, rank[res[1]], res[0], a * ns + c))

    def canon(rows):
        arr = np.array(rows, dtype=np.int64).reshape(-1, 4)
        order = np.lexsort((arr[:, 3], arr[:, 0], arr[:, 1]))
        return arr[order]

    return dict(two_body=canon(two), one_body=canon(one))


def expectation(b, inter, x):
    """<x|H|x> / <x|x>."""
    y = apply_h(b, inter, x)
    return float(np.dot(x, y) / np.dot(x, x))
