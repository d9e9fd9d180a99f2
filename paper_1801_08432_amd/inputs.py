"""Seeded synthetic inputs for the factorized on-the-fly CI path.

This module holds input recipes only: single-particle spaces (lists of 2j and
parity per orbit), the five workload shapes, and seeded random single-particle
energies, m-scheme two-body matrix elements and vectors, laid out in the format
that ``fotci_set_interaction`` takes. It contains none of the method's
arithmetic (no operator action, no basis, no jumps), so that both the CPU oracle
and the GPU library can consume the same arrays.

Layout conventions of the interaction arrays (the library's input format):

* m-states of one species are numbered orbit by orbit in the given orbit order,
  2m ascending inside an orbit; m-state ``i`` is bit ``i`` of a Slater
  determinant mask.
* ``v_pp`` / ``v_nn`` are dense ``n_pairs x n_pairs`` arrays over pair states
  ``(a<b)`` enumerated lexicographically; entry ``[(ab),(cd)]`` multiplies
  ``a+_a a+_b a_d a_c`` (so it equals the antisymmetrised matrix element
  between normalised two-particle states |ab> and |cd>).
* ``v_pn`` is a dense ``(ns*ns) x (ns*ns)`` array; row ``a*ns+b`` pairs proton
  m-state ``a`` with neutron m-state ``b``; entry ``[(ab),(cd)]`` multiplies
  ``(p+_a p_c)(n+_b n_d)``.
* Entries that would change total Jz or parity are exactly zero; the arrays are
  exactly symmetric.

The random recipe (every independent element of V drawn i.i.d. N(0,1) MeV,
including the diagonal; single-particle energies U(-5,5) MeV per orbit) follows
the workloads described for the method's valence spaces.
"""
from __future__ import annotations

import numpy as np

SD_SHELL_LIKE = (1, 3, 5)       # 2j of the orbits: 12 m-states per species
PF_SHELL_LIKE = (1, 3, 5, 7)    # 20 m-states per species

# The five workloads: (space, Z, N, 2M, total parity, seed).
WORKLOADS = {
    "sd_2p2n": dict(two_j=SD_SHELL_LIKE, Z=2, N=2, two_M=0, parity=1, seed=1801084321),
    "sd_6p6n": dict(two_j=SD_SHELL_LIKE, Z=6, N=6, two_M=0, parity=1, seed=1801084322),
    "pf_4p4n": dict(two_j=PF_SHELL_LIKE, Z=4, N=4, two_M=0, parity=1, seed=1801084323),
    "pf_4p4n_grad": dict(two_j=PF_SHELL_LIKE, Z=4, N=4, two_M=0, parity=1, seed=1801084324),
    "pf_5p5n": dict(two_j=PF_SHELL_LIKE, Z=5, N=5, two_M=0, parity=1, seed=1801084325),
}


def orbit_parities(two_j, parity=None):
    """All orbits share one parity (+1) unless a list is given."""
    if parity is None:
        return tuple(1 for _ in two_j)
    return tuple(int(p) for p in parity)


def m_state_table(two_j, parity=None):
    """(orbit, 2j, 2m, parity) per m-state, in the input-format order."""
    par = orbit_parities(two_j, parity)
    out = []
    for o, (tj, p) in enumerate(zip(two_j, par)):
        for tm in range(-tj, tj + 1, 2):
            out.append((o, tj, tm, p))
    return out


def _pair_table(ms):
    ns = len(ms)
    return [(a, b) for a in range(ns) for b in range(a + 1, ns)]


def random_interaction(two_j, seed, parity=None, scale=1.0):
    """Seeded random Jz- and parity-conserving symmetric interaction.

    Draw order from ``numpy.random.default_rng(seed)``: eps_p (U(-5,5), one
    per orbit), eps_n, then V_pp, V_nn and V_pn, each as one
    ``standard_normal(count)`` call filled into the allowed upper-triangle
    entries (diagonal included) in row-major order and mirrored.
    Returns a dict of float64 arrays and the generator (for later draws).
    """
    rng = np.random.default_rng(seed)
    ms = m_state_table(two_j, parity)
    ns = len(ms)
    n_orb = len(two_j)
    eps_p = rng.uniform(-5.0, 5.0, n_orb)
    eps_n = rng.uniform(-5.0, 5.0, n_orb)

    tm = np.array([m[2] for m in ms])
    pi = np.array([m[3] for m in ms])
    pairs = _pair_table(ms)
    pm = np.array([tm[a] + tm[b] for a, b in pairs])
    pp = np.array([pi[a] * pi[b] for a, b in pairs])

    def sym_block(allowed):
        n = allowed.shape[0]
        iu = np.triu_indices(n)
        ok = allowed[iu]
        vals = rng.standard_normal(int(ok.sum())) * scale
        v = np.zeros((n, n))
        r, c = iu[0][ok], iu[1][ok]
        v[r, c] = vals
        v[c, r] = vals
        return v

    allowed_pair = (pm[:, None] == pm[None, :]) & (pp[:, None] == pp[None, :])
    v_pp = sym_block(allowed_pair)
    v_nn = sym_block(allowed_pair)

    # pn rows (a_p, b_n) -> index a*ns + b
    a_idx = np.repeat(np.arange(ns), ns)
    b_idx = np.tile(np.arange(ns), ns)
    qm = tm[a_idx] + tm[b_idx]
    qp = pi[a_idx] * pi[b_idx]
    allowed_pn = (qm[:, None] == qm[None, :]) & (qp[:, None] == qp[None, :])
    v_pn = sym_block(allowed_pn)
    return dict(eps_p=eps_p, eps_n=eps_n, v_pp=v_pp, v_nn=v_nn, v_pn=v_pn), rng


def workload(name):
    """The workload's shape parameters and its seeded interaction arrays."""
    w = dict(WORKLOADS[name])
    inter, rng = random_interaction(w["two_j"], w["seed"])
    w.update(inter)
    w["rng"] = rng
    return w


def random_vector(n, seed, dtype=np.float64):
    """Seeded N(0,1) vector of length n."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def random_jcoupled(two_j, seed, parity=None, scale=1.0):
    """Seeded random rotationally invariant interaction as J-coupled elements.

    For every 2J, one symmetric N(0,1) matrix over the allowed orbit pairs of
    each kind (like particles: a <= b, even J when a == b; proton-neutron: all
    (a, b)), parity-conserving pairs only; single-particle energies U(-5,5)
    per orbit. Draw order from ``numpy.random.default_rng(seed)``: eps_p,
    eps_n, then pp, nn, pn, each by ascending 2J, upper triangle row-major.
    Returns (eps_p, eps_n, pp, nn, pn), the element lists as
    (a, b, c, d, two_J, V) tuples with (ab) <= (cd) in list order.
    """
    rng = np.random.default_rng(seed)
    n = len(two_j)
    par = [1] * n if parity is None else list(parity)
    eps_p = rng.uniform(-5.0, 5.0, n)
    eps_n = rng.uniform(-5.0, 5.0, n)
    max_tJ = 2 * max(two_j)

    def draw(like):
        out = []
        for tJ in range(0, max_tJ + 1, 2):
            pl = []
            for a in range(n):
                for b in range(a if like else 0, n):
                    if not (abs(two_j[a] - two_j[b]) <= tJ <= two_j[a] + two_j[b]):
                        continue
                    if like and a == b and (tJ // 2) % 2:
                        continue
                    pl.append((a, b))
            for i in range(len(pl)):
                for k in range(i, len(pl)):
                    (a, b), (c, d) = pl[i], pl[k]
                    if par[a] * par[b] != par[c] * par[d]:
                        continue
                    out.append((a, b, c, d, tJ, float(rng.standard_normal()) * scale))
        return out

    pp = draw(True)
    nn = draw(True)
    pn = draw(False)
    return eps_p, eps_n, pp, nn, pn
