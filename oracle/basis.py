"""M-scheme basis factorised into proton x neutron Slater determinants.

Written from Ch. 2, "Use of quantum numbers: factorization of the basis" and
Ch. 6, "Writing out the basis":

* Each basis state is a product of a proton SD and a neutron SD with
  M_p + M_n = M (and parity pi_p * pi_n = pi).
* SDs of one species are grouped into sectors of fixed (M, parity); every
  proton SD of a sector combines with every neutron SD of the conjugate
  sector, so a sector of the basis is the dense block np_s x nn_s.
* A species sector with no conjugate partner is dropped (the "missing"
  neutron SD of the 27Al example).
* basis index = pstart(ip) + nstart(jn) with the neutron index innermost.

Readings where the paper leaves the order open: m-states orbit by orbit, 2m
ascending; sectors by 2M ascending, parity +1 before -1; SDs inside a sector
by ascending mask value; neutron sectors ordered the same way.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field


def m_states(two_j, parity=None):
    """(orbit, 2j, 2m, parity) per single-particle m-state."""
    if parity is None:
        parity = [1] * len(two_j)
    out = []
    for o, (tj, p) in enumerate(zip(two_j, parity)):
        for tm in range(-tj, tj + 1, 2):
            out.append((o, tj, tm, p))
    return out


def sd_quantum_numbers(mask, ms):
    """(2M, parity) of a Slater determinant."""
    two_m, par = 0, 1
    for i, m in enumerate(ms):
        if (mask >> i) & 1:
            two_m += m[2]
            par *= m[3]
    return two_m, par


def all_sds(ms, n):
    """All n-particle masks of the species, ascending."""
    masks = [sum(1 << i for i in occ) for occ in itertools.combinations(range(len(ms)), n)]
    return sorted(masks)


def _sector_key(k):
    two_m, par = k
    return (two_m, 0 if par == 1 else 1)


@dataclass
class Basis:
    ms: list
    Z: int
    N: int
    two_M: int
    parity: int
    p_sds: list = field(default_factory=list)      # kept proton masks, sector-grouped
    n_sds: list = field(default_factory=list)      # kept neutron masks, sector-grouped
    p_sectors: list = field(default_factory=list)  # (2M, par, first, count)
    n_sectors: list = field(default_factory=list)
    sectors: list = field(default_factory=list)    # (2Mp, par_p, p_sector, n_sector, offset)
    pstart: list = field(default_factory=list)     # per kept proton SD
    nstart: list = field(default_factory=list)     # per kept neutron SD
    dim: int = 0

    def index(self, pmask, nmask):
        """Basis index of (proton mask, neutron mask), or None if not in the basis."""
        ip = self._p_rank.get(pmask)
        jn = self._n_rank.get(nmask)
        if ip is None or jn is None:
            return None
        if self._p_sec_of[ip] != self._conj_p[self._n_sec_of[jn]]:
            return None
        return self.pstart[ip] + self.nstart[jn]

    def states(self):
        """All (pmask, nmask) in basis order."""
        out = [None] * self.dim
        for (_, _, ps, ns_, off) in self.sectors:
            _, _, pf, pc = self.p_sectors[ps]
            _, _, nf, nc = self.n_sectors[ns_]
            for r in range(pc):
                for c in range(nc):
                    out[off + r * nc + c] = (self.p_sds[pf + r], self.n_sds[nf + c])
        return out


def build_basis(two_j, Z, N, two_M, parity=1, orbit_parity=None):
    """Build the factorised M-scheme basis (raises ValueError when empty/invalid)."""
    ms = m_states(two_j, orbit_parity)
    ns = len(ms)
    if Z < 0 or N < 0 or Z > ns or N > ns:
        raise ValueError("particle number out of range")
    groups = {}
    for sp, n in (("p", Z), ("n", N)):
        g = {}
        for m in all_sds(ms, n):
            g.setdefault(sd_quantum_numbers(m, ms), []).append(m)
        groups[sp] = g
    pkeys = sorted(groups["p"], key=_sector_key)
    kept = []
    for k in pkeys:
        conj = (two_M - k[0], parity * k[1])
        if conj in groups["n"]:
            kept.append((k, conj))
    if not kept:
        raise ValueError("empty basis")
    b = Basis(ms=ms, Z=Z, N=N, two_M=two_M, parity=parity)
    nkeys = sorted({c for _, c in kept}, key=_sector_key)
    n_sec_index = {}
    for k in nkeys:
        sds = groups["n"][k]
        n_sec_index[k] = len(b.n_sectors)
        b.n_sectors.append((k[0], k[1], len(b.n_sds), len(sds)))
        b.n_sds.extend(sds)
    b.nstart = [0] * len(b.n_sds)
    for (_, _, f, c) in b.n_sectors:
        for r in range(c):
            b.nstart[f + r] = r
    off = 0
    b.pstart = []
    conj_p = {}
    for (k, conj) in kept:
        sds = groups["p"][k]
        ps = len(b.p_sectors)
        b.p_sectors.append((k[0], k[1], len(b.p_sds), len(sds)))
        b.p_sds.extend(sds)
        nsec = n_sec_index[conj]
        nn = b.n_sectors[nsec][3]
        b.sectors.append((k[0], k[1], ps, nsec, off))
        conj_p[nsec] = ps
        for r in range(len(sds)):
            b.pstart.append(off + r * nn)
        off += len(sds) * nn
    b.dim = off
    b._p_rank = {m: i for i, m in enumerate(b.p_sds)}
    b._n_rank = {m: i for i, m in enumerate(b.n_sds)}
    b._p_sec_of = [0] * len(b.p_sds)
    for s, (_, _, f, c) in enumerate(b.p_sectors):
        for r in range(c):
            b._p_sec_of[f + r] = s
    b._n_sec_of = [0] * len(b.n_sds)
    for s, (_, _, f, c) in enumerate(b.n_sectors):
        for r in range(c):
            b._n_sec_of[f + r] = s
    b._conj_p = conj_p
    return b


def sector_table(b):
    """Per basis sector: (2Mp, par_p, p_first, np, n_first, nn, offset)."""
    rows = []
    for (tm, par, ps, nsec, off) in b.sectors:
        _, _, pf, pc = b.p_sectors[ps]
        _, _, nf, nc = b.n_sectors[nsec]
        rows.append((tm, par, pf, pc, nf, nc, off))
    return rows


def dimension_only(two_j, Z, N, two_M, parity=1, orbit_parity=None):
    """Sector counts and dimension without storing the basis (for large pins).

    Returns (per proton sector rows (2Mp, np, 2Mn, nn), n_psd, n_nsd, dim),
    counting SDs per (2M, parity) by enumeration.
    """
    ms = m_states(two_j, orbit_parity)
    counts = {}
    for sp, n in (("p", Z), ("n", N)):
        c = {}
        for occ in itertools.combinations(range(len(ms)), n):
            two_m = sum(ms[i][2] for i in occ)
            par = 1
            for i in occ:
                par *= ms[i][3]
            c[(two_m, par)] = c.get((two_m, par), 0) + 1
        counts[sp] = c
    rows, npsd, nnsd, dim = [], 0, 0, 0
    for k in sorted(counts["p"], key=_sector_key):
        conj = (two_M - k[0], parity * k[1])
        if conj not in counts["n"]:
            continue
        npc, nnc = counts["p"][k], counts["n"][conj]
        rows.append((k[0], npc, conj[0], nnc))
        npsd += npc
        nnsd += nnc
        dim += npc * nnc
    return rows, npsd, nnsd, dim
