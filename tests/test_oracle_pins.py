"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: numbers the
paper prints (basis dimensions and sector tables), worked examples (phase
rule), closed forms (seniority pairing, sum rules, one-body spectra,
combinatorial counts), an independent Jordan-Wigner construction of the same
operators, and library eigensolvers.
"""
import itertools
import math
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

sys.path.insert(0, os.path.dirname(__file__))
import jw  # noqa: E402

from oracle import basis as ob  # noqa: E402
from oracle import fermion as fe  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402
from oracle import lanczos as ol  # noqa: E402
from oracle import fast as of  # noqa: E402
from paper_1801_08432_amd import inputs  # noqa: E402

SD = (5, 1, 3)          # 0d5/2, 1s1/2, 0d3/2
PF = (7, 3, 5, 1)       # 0f7/2, 1p3/2, 0f5/2, 1p1/2
P_SHELL = (1, 3)


def _load_golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- P3: phases
def test_phase_examples_from_the_paper():
    """Ch. 2 "Representation of the basis": annihilating state 2 of 110101 gives
    -100101; annihilating the empty state 2 of 100111 gives zero; the two-body
    example a+_3 a+_5 a_4 a_1 |1101011> carries an overall minus sign (its
    printed result has a stray digit; the 7-state result is 0110111)."""
    m = fe.from_string("110101")
    s, m2 = fe.annihilate(m, 1)
    assert s == -1 and fe.to_string(m2, 6) == "100101"
    assert fe.annihilate(fe.from_string("100111"), 1) is None
    m = fe.from_string("1101011")
    r = fe.apply_ops(m, [("+", 2), ("+", 4), ("-", 3), ("-", 0)])
    assert r is not None
    assert r[0] == -1 and fe.to_string(r[1], 7) == "0110111"
    # intermediate state of the example: -a+_3 a+_5 |0100011>
    r1 = fe.apply_ops(m, [("-", 3), ("-", 0)])
    assert r1[0] == -1 and fe.to_string(r1[1], 7) == "0100011"


# ------------------------------------------------- P4: anticommutation rules
def test_anticommutators_on_random_determinants():
    rng = np.random.default_rng(7)
    n = 10
    for _ in range(200):
        mask = int(rng.integers(0, 1 << n))
        i, j = (int(t) for t in rng.integers(0, n, 2))

        def act(ops):
            r = fe.apply_ops(mask, ops)
            return {} if r is None else {r[1]: r[0]}

        def add(d1, d2):
            out = dict(d1)
            for k, v in d2.items():
                out[k] = out.get(k, 0) + v
            return {k: v for k, v in out.items() if v != 0}

        # {a_i, a+_j} = delta_ij
        got = add(act([("-", i), ("+", j)]), act([("+", j), ("-", i)]))
        assert got == ({mask: 1} if i == j else {})
        # {a_i, a_j} = 0 and {a+_i, a+_j} = 0
        assert add(act([("-", i), ("-", j)]), act([("-", j), ("-", i)])) == {}
        assert add(act([("+", i), ("+", j)]), act([("+", j), ("+", i)])) == {}


def test_phase_matches_jordan_wigner():
    n = 8
    a = jw.annihilators(n)
    rng = np.random.default_rng(3)
    for _ in range(100):
        mask = int(rng.integers(0, 1 << n))
        ops = [(("+", "-")[int(rng.integers(0, 2))], int(rng.integers(0, n))) for _ in range(4)]
        mat = sp.identity(1 << n, format="csr")
        for kind, i in ops:
            mat = mat @ (a[i].T if kind == "+" else a[i])
        col = mat[:, [mask]].toarray().ravel()
        r = fe.apply_ops(mask, ops)
        if r is None:
            assert not np.any(col)
        else:
            expect = np.zeros(1 << n)
            expect[r[1]] = r[0]
            assert np.array_equal(col, expect)


# ------------------------------------------- P1: printed basis dimensions
def test_al27_sector_table():
    """Table al27 (Ch. 2): 27Al, sd shell, 5 protons + 6 neutrons, M = +1/2.

    The table's row M_p = -7/2 prints 2444 combined states; 51 x 47 = 2397,
    and the printed total 80,115 only adds up with 2397, so the fixture
    holds 2397."""
    rows = _load_golden("al27_sectors.txt")
    expect = {int(r[0]): (int(r[1]), int(r[2]), int(r[3]), int(r[4])) for r in rows}
    got_rows, npsd, nnsd, dim = ob.dimension_only(SD, 5, 6, 1)
    got = {tmp: (np_, tmn, nn, np_ * nn) for (tmp, np_, tmn, nn) in got_rows}
    assert got == expect
    assert len(got_rows) == 14
    assert (npsd, nnsd, dim) == (792, 923, 80115)
    # the lone M_n = -7 neutron SD has no conjugate proton sector
    b = ob.build_basis(SD, 5, 6, 1)
    assert len(ob.all_sds(b.ms, 6)) == 924 and len(b.n_sds) == 923


def test_printed_dimensions():
    """Dimensions printed in Ch. 2, Ch. 3 (Table timetable) and Ch. 6."""
    for (space, Z, N, two_M, dim, extra) in [
        (SD, 2, 2, 0, 640, (9, 66)),            # 20Ne, the .bas example: 9 sectors / 66 pSDs
        (SD, 4, 4, 0, 28503, None),             # 24Mg
        (SD, 6, 6, 0, 93710, None),             # 28Si (9.4e4 in Table jumps)
        (P_SHELL, 2, 2, 0, 51, None),           # 8Be, p shell
        (PF, 4, 4, 0, 1963461, None),           # 48Cr "2 M"
        (PF, 5, 6, 1, 44993824, None),          # 51Mn "44M"
    ]:
        rows, npsd, nnsd, d = ob.dimension_only(space, Z, N, two_M)
        assert d == dim, (Z, N, d)
        if extra:
            assert (len(rows), npsd) == extra


def test_fe56_and_zn60_printouts():
    """56Fe (pf, 6p10n, M=0): 27 sectors per species, 38,760 / 184,722 SDs,
    total 501,113,392 (Ch. 2 printout); 60Zn (10p10n): 2.3 billion."""
    rows, npsd, nnsd, dim = ob.dimension_only(PF, 6, 10, 0)
    assert (len(rows), npsd, nnsd, dim) == (27, 38760, 184722, 501113392)
    rows, npsd, nnsd, dim = ob.dimension_only(PF, 10, 10, 0)
    assert dim == 2292604744 and abs(npsd - 185000) < 1000


# ----------------------------------------------- P2: combinatorial counts
def _gf_counts(two_j, n):
    """Counts of n-particle SDs per 2M by a generating-function DP (no enumeration)."""
    ms = [tm for tj in two_j for tm in range(-tj, tj + 1, 2)]
    poly = {(0, 0): 1}                      # (particles, 2M) -> count
    for tm in ms:
        new = dict(poly)
        for (k, s), c in poly.items():
            if k < n:
                new[(k + 1, s + tm)] = new.get((k + 1, s + tm), 0) + c
        poly = new
    return {s: c for (k, s), c in poly.items() if k == n}


@pytest.mark.parametrize("space,Z,N,two_M", [(SD, 2, 2, 0), (SD, 6, 6, 0), (PF, 4, 4, 0),
                                              (PF, 5, 5, 0), (SD, 5, 6, 1), (PF, 3, 6, 3)])
def test_dimension_by_generating_function(space, Z, N, two_M):
    cp, cn = _gf_counts(space, Z), _gf_counts(space, N)
    dim = sum(c * cn.get(two_M - s, 0) for s, c in cp.items())
    rows, npsd, nnsd, d = ob.dimension_only(space, Z, N, two_M)
    assert d == dim
    ns = sum(tj + 1 for tj in space)
    assert sum(cp.values()) == math.comb(ns, Z)


def test_one_body_jumps_per_sd():
    """With every sector kept, each SD has n (N_s - n + 1) one-body jumps:
    n choices of c, and N_s - n empty states plus c itself for a."""
    b = ob.build_basis(SD, 3, 3, 0)
    ns = len(b.ms)
    for sp, n in (("p", 3), ("n", 3)):
        j = oh.jumps(b, sp)["one_body"]
        counts = np.bincount(j[:, 0], minlength=len(b.p_sds if sp == "p" else b.n_sds))
        assert np.all(counts == n * (ns - n + 1))


def test_basis_structure():
    b = ob.build_basis(PF, 3, 2, 1)
    states = b.states()
    assert len(states) == b.dim == len(set(states))
    for t, (pm, nm) in enumerate(states):
        assert b.index(pm, nm) == t
        m = ob.sd_quantum_numbers(pm, b.ms)[0] + ob.sd_quantum_numbers(nm, b.ms)[0]
        assert m == 1
    # neutron innermost, sectors contiguous, masks ascending within a sector
    for (tmp, par, pf, pc, nf, nc, off) in ob.sector_table(b):
        assert b.p_sds[pf:pf + pc] == sorted(b.p_sds[pf:pf + pc])
        assert b.n_sds[nf:nf + nc] == sorted(b.n_sds[nf:nf + nc])
        assert b.index(b.p_sds[pf], b.n_sds[nf + 1 if nc > 1 else nf]) == off + (1 if nc > 1 else 0)


# -------------------------- P10: Hamiltonian against Jordan-Wigner matrices
def _jw_hamiltonian(b, inter):
    """H restricted to the basis from per-species Jordan-Wigner matrices."""
    ns = len(b.ms)
    a = jw.annihilators(ns)
    ad = [m.T.tocsr() for m in a]
    states = b.states()
    pidx = np.array([s[0] for s in states])
    nidx = np.array([s[1] for s in states])
    orb = [m[0] for m in b.ms]
    eps_p = np.asarray(inter["eps_p"])[orb]
    eps_n = np.asarray(inter["eps_n"])[orb]
    dim = b.dim
    num = [ad[i] @ a[i] for i in range(ns)]
    Hp = sum(eps_p[i] * num[i] for i in range(ns)).tocsr()
    Hn = sum(eps_n[i] * num[i] for i in range(ns)).tocsr()
    pl = oh.pair_list(ns)
    for (vkey, target) in (("v_pp", "p"), ("v_nn", "n")):
        v = inter[vkey]
        acc = sp.csr_matrix((1 << ns, 1 << ns))
        for r, (aa, bb) in enumerate(pl):
            for c, (cc, dd) in enumerate(pl):
                if v[r, c] != 0.0:
                    acc += v[r, c] * (ad[aa] @ ad[bb] @ a[dd] @ a[cc])
        if target == "p":
            Hp = Hp + acc
        else:
            Hn = Hn + acc
    def sub(m, idx):
        return m.tocsr()[idx][:, idx].toarray()

    H = sub(Hp, pidx) * (nidx[:, None] == nidx[None, :])
    H = H + sub(Hn, nidx) * (pidx[:, None] == pidx[None, :])
    one = [[(ad[x] @ a[y]).tocsr() for y in range(ns)] for x in range(ns)]
    vpn = inter["v_pn"]
    for row, col in zip(*np.nonzero(vpn)):
        aa, bb = divmod(int(row), ns)
        cc, dd = divmod(int(col), ns)
        H = H + vpn[row, col] * sub(one[aa][cc], pidx) * sub(one[bb][dd], nidx)
    assert H.shape == (dim, dim)
    return H


@pytest.mark.parametrize("space,Z,N,two_M,seed", [(P_SHELL, 2, 2, 0, 11), (P_SHELL, 3, 2, 1, 12),
                                                   (inputs.SD_SHELL_LIKE, 2, 2, 0, 1801084321)])
def test_hamiltonian_matches_jordan_wigner(space, Z, N, two_M, seed):
    inter, _ = inputs.random_interaction(space, seed)
    b = ob.build_basis(space, Z, N, two_M)
    H = oh.dense_h(b, inter)
    Hj = _jw_hamiltonian(b, inter)
    assert np.max(np.abs(H - Hj)) < 1e-12
    assert np.max(np.abs(H - H.T)) < 1e-12   # P4/P9: Hermitian


# ------------------------------------------------- P5: two-particle blocks
def test_two_protons_block_is_v_pp():
    space = inputs.SD_SHELL_LIKE
    inter, _ = inputs.random_interaction(space, 5)
    for two_M in (0, 2, 4):
        b = ob.build_basis(space, 2, 0, two_M)
        H = oh.dense_h(b, inter)
        pl = oh.pair_list(len(b.ms))
        pos = {(1 << x) | (1 << y): k for k, (x, y) in enumerate(pl)}
        rows = [pos[pm] for pm, _ in b.states()]
        orb = [m[0] for m in b.ms]
        d = [inter["eps_p"][orb[pl[k][0]]] + inter["eps_p"][orb[pl[k][1]]] for k in rows]
        expect = inter["v_pp"][np.ix_(rows, rows)] + np.diag(d)
        assert np.array_equal(H, expect)


def test_one_proton_one_neutron_block_is_v_pn():
    space = inputs.SD_SHELL_LIKE
    inter, _ = inputs.random_interaction(space, 6)
    ns = 12
    for two_M in (0, 2):
        b = ob.build_basis(space, 1, 1, two_M)
        H = oh.dense_h(b, inter)
        rows = [(pm.bit_length() - 1) * ns + (nm.bit_length() - 1) for pm, nm in b.states()]
        orb = [m[0] for m in b.ms]
        d = [inter["eps_p"][orb[r // ns]] + inter["eps_n"][orb[r % ns]] for r in rows]
        expect = inter["v_pn"][np.ix_(rows, rows)] + np.diag(d)
        assert np.array_equal(H, expect)


# ----------------------------------------------- P6: one-body-only spectrum
def test_one_body_spectrum_is_sum_of_occupied_energies():
    space = inputs.SD_SHELL_LIKE
    rng = np.random.default_rng(9)
    b = ob.build_basis(space, 3, 2, 1)
    ns = len(b.ms)
    inter = dict(eps_p_mstate=rng.uniform(-5, 5, ns), eps_n_mstate=rng.uniform(-5, 5, ns),
                 v_pp=np.zeros((66, 66)), v_nn=np.zeros((66, 66)), v_pn=np.zeros((144, 144)))
    ev = np.linalg.eigvalsh(oh.dense_h(b, inter))
    expect = []
    for pm, nm in b.states():
        expect.append(sum(inter["eps_p_mstate"][i] for i in range(ns) if (pm >> i) & 1)
                      + sum(inter["eps_n_mstate"][i] for i in range(ns) if (nm >> i) & 1))
    assert np.allclose(np.sort(ev), np.sort(expect), atol=1e-12)


# -------------------------------------------------- P7: seniority pairing
def _pairing_interaction(two_j, G):
    ms = inputs.m_state_table((two_j,))
    ns = len(ms)
    pl = oh.pair_list(ns)
    v = np.zeros((len(pl), len(pl)))
    # pair (-m, m), m > 0: lower index first (2m ascending inside the orbit)
    pk = [k for k, (a, b) in enumerate(pl) if ms[a][2] == -ms[b][2] and ms[b][2] > 0]
    for r in pk:
        for c in pk:
            v[r, c] = -G
    return dict(eps_p=[0.0], eps_n=[0.0], v_pp=v, v_nn=np.zeros_like(v),
                v_pn=np.zeros((ns * ns, ns * ns)))


def _sd_count(two_j, v, two_M):
    ms = list(range(-two_j, two_j + 1, 2))
    return sum(1 for occ in itertools.combinations(ms, v) if sum(occ) == two_M) if v >= 0 else 0


@pytest.mark.parametrize("two_j,n,two_M", [(7, 4, 0), (7, 4, 2), (7, 3, 1), (7, 2, 0), (9, 4, 0), (9, 5, 1)])
def test_single_j_pairing_seniority_spectrum(two_j, n, two_M):
    """H = -G P+ P in one j shell: E(n,v) = -(G/4)(n-v)(2 Omega - n - v + 2),
    Omega = j + 1/2, multiplicity D_v(M) - D_{v-2}(M) (textbook seniority)."""
    G = 0.37
    b = ob.build_basis((two_j,), n, 0, two_M)
    ev = np.linalg.eigvalsh(oh.dense_h(b, _pairing_interaction(two_j, G)))
    omega = (two_j + 1) // 2
    expect = []
    for v in range(n % 2, min(n, 2 * omega - n) + 1, 2):
        mult = _sd_count(two_j, v, two_M) - _sd_count(two_j, v - 2, two_M)
        e = -(G / 4.0) * (n - v) * (2 * omega - n - v + 2)
        expect += [e] * mult
    assert len(expect) == b.dim
    assert np.allclose(np.sort(ev), np.sort(expect), atol=1e-12)


# -------------------------------------------------- P8: pair-number sum rules
def test_pair_number_sum_rules():
    space = inputs.SD_SHELL_LIKE
    ns = 12
    npairs = 66
    b = ob.build_basis(space, 3, 2, 1)
    inter = dict(eps_p=[0, 0, 0], eps_n=[0, 0, 0], v_pp=np.eye(npairs), v_nn=np.zeros((npairs, npairs)),
                 v_pn=np.zeros((ns * ns, ns * ns)))
    ev = np.linalg.eigvalsh(oh.dense_h(b, inter))
    assert np.allclose(ev, 3 * 2 / 2, atol=1e-12)
    inter["v_pp"] = np.zeros((npairs, npairs))
    inter["v_pn"] = np.eye(ns * ns)
    ev = np.linalg.eigvalsh(oh.dense_h(b, inter))
    assert np.allclose(ev, 3 * 2, atol=1e-12)
    # the same through the C oracle, on a larger case, applied to random vectors
    b = ob.build_basis(space, 4, 4, 0)
    prep = of.Prepared(b)
    x = np.random.default_rng(1).standard_normal(b.dim)
    inter["v_pn"] = np.zeros((ns * ns, ns * ns))
    inter["v_pp"] = np.eye(npairs)
    inter["v_nn"] = np.eye(npairs)
    assert np.allclose(of.apply_h(prep, inter, x), (6 + 6) * x, rtol=1e-13)
    inter["v_pp"] = np.zeros((npairs, npairs))
    inter["v_nn"] = np.zeros((npairs, npairs))
    inter["v_pn"] = np.eye(ns * ns)
    assert np.allclose(of.apply_h(prep, inter, x), 16 * x, rtol=1e-13)


# -------------------------- jumps against Jordan-Wigner matrix elements
def test_jumps_against_jordan_wigner():
    space = inputs.SD_SHELL_LIKE
    b = ob.build_basis(space, 3, 2, 1)
    ns = len(b.ms)
    a = jw.annihilators(ns)
    ad = [m.T.tocsr() for m in a]
    pl = oh.pair_list(ns)
    npairs = len(pl)
    for sp, sds in (("p", b.p_sds), ("n", b.n_sds)):
        j = oh.jumps(b, sp)
        kept = set(sds)
        # two-body: every record equals the Jordan-Wigner matrix element, and
        # every nonzero element between same-sector SDs appears
        seen = set()
        for src, dst, ph, lab in j["two_body"]:
            r, c = divmod(int(lab), npairs)
            (x, y), (u, w) = pl[r], pl[c]
            assert ob.sd_quantum_numbers(sds[dst], b.ms) == ob.sd_quantum_numbers(sds[src], b.ms)
            op = ad[x] @ ad[y] @ a[w] @ a[u]
            assert op[sds[dst], sds[src]] == ph
            seen.add((int(src), int(lab)))
        rng = np.random.default_rng(4)
        for src in rng.choice(len(sds), 6, replace=False):
            for r, (x, y) in enumerate(pl):
                for c, (u, w) in enumerate(pl):
                    if b.ms[x][2] + b.ms[y][2] != b.ms[u][2] + b.ms[w][2]:
                        continue
                    col = (ad[x] @ ad[y] @ a[w] @ a[u])[:, [sds[src]]].toarray().ravel()
                    nz = np.nonzero(col)[0]
                    assert (len(nz) > 0) == ((int(src), r * npairs + c) in seen)
        # one-body
        for src, dst, ph, lab in j["one_body"]:
            x, u = divmod(int(lab), ns)
            assert (ad[x] @ a[u])[sds[dst], sds[src]] == ph
            assert sds[dst] in kept
        # canonical order
        for key in ("two_body", "one_body"):
            arr = j[key]
            keys = list(zip(arr[:, 1], arr[:, 0], arr[:, 3]))
            assert keys == sorted(keys) and len(set(keys)) == len(keys)


# ----------------------------------------- C oracle == Python oracle
@pytest.mark.parametrize("space,Z,N,two_M,seed", [(inputs.SD_SHELL_LIKE, 2, 2, 0, 1801084321),
                                                   (inputs.PF_SHELL_LIKE, 2, 1, 1, 77)])
def test_c_oracle_matches_python_oracle(space, Z, N, two_M, seed):
    inter, rng = inputs.random_interaction(space, seed)
    b = ob.build_basis(space, Z, N, two_M)
    H = oh.dense_h(b, inter)
    prep = of.Prepared(b)
    x = rng.standard_normal(b.dim)
    g = rng.standard_normal(b.dim)
    y = of.apply_h(prep, inter, x)
    assert np.max(np.abs(y - H @ x)) <= 1e-12 * np.max(np.abs(H @ x))
    # a row window
    y2 = of.apply_h(prep, inter, x, rows=(3, b.dim - 2))
    assert np.array_equal(y2, y[3:b.dim - 2])
    dp = oh.densities(b, g, x)
    dc = of.densities(prep, g, x)
    for k in dp:
        assert np.allclose(dp[k], dc[k], rtol=1e-12, atol=1e-12), k


# ------------------------------------------ P12: Euler identity (linearity)
def test_euler_identity_for_densities():
    space = inputs.SD_SHELL_LIKE
    inter, rng = inputs.random_interaction(space, 21)
    b = ob.build_basis(space, 2, 2, 0)
    x = rng.standard_normal(b.dim)
    g = rng.standard_normal(b.dim)
    d = oh.densities(b, g, x)
    lhs = (np.dot(d["d_eps_p"], inter["eps_p"]) + np.dot(d["d_eps_n"], inter["eps_n"])
           + np.sum(d["d_v_pp"] * inter["v_pp"]) + np.sum(d["d_v_nn"] * inter["v_nn"])
           + np.sum(d["d_v_pn"] * inter["v_pn"]))
    rhs = float(g @ oh.apply_h(b, inter, x))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_density_of_single_element_is_finite_difference():
    """<g|H(V + E_rc)|x> - <g|H(V)|x> = <g|O_rc|x>: perturb one (non-symmetric)
    entry and difference the direct push-form matvec."""
    space = inputs.SD_SHELL_LIKE
    inter, rng = inputs.random_interaction(space, 22)
    b = ob.build_basis(space, 2, 2, 0)
    x = rng.standard_normal(b.dim)
    g = rng.standard_normal(b.dim)
    d = oh.densities(b, g, x)
    base = g @ oh.apply_h(b, inter, x)
    for key, dkey in (("v_pp", "d_v_pp"), ("v_pn", "d_v_pn")):
        nz = np.argwhere(d[dkey] != 0)
        for r, c in nz[rng.choice(len(nz), 5, replace=False)]:
            pert = dict(inter)
            pert[key] = inter[key].copy()
            pert[key][r, c] += 1.0
            diff = g @ oh.apply_h(b, pert, x) - base
            assert abs(diff - d[dkey][r, c]) < 1e-9


# ------------------------------------------ P14 / P10: Lanczos oracle
def test_oracle_lanczos_full_krylov_recovers_spectrum():
    space = inputs.SD_SHELL_LIKE
    inter, rng = inputs.random_interaction(space, 1801084321)
    b = ob.build_basis(space, 2, 2, 0)
    H = oh.dense_h(b, inter)
    ev = np.linalg.eigvalsh(H)
    got, vecs, _, _ = ol.lanczos(lambda v: H @ v, rng.standard_normal(b.dim), b.dim, b.dim)
    assert np.allclose(got, ev, atol=1e-9 * np.max(np.abs(ev)))
    got5, vecs5, _, _ = ol.lanczos(lambda v: H @ v, rng.standard_normal(b.dim), 120, 5)
    assert np.allclose(got5, ev[:5], rtol=1e-10)
    for k in range(5):
        r = H @ vecs5[k] - got5[k] * vecs5[k]
        assert np.linalg.norm(r) < 1e-6


# ------------------------------------- block Lanczos (Ch. "Block Lanczos")
@pytest.mark.parametrize("nb", [2, 4, 8])
def test_oracle_block_lanczos_full_krylov_recovers_spectrum(nb):
    """dim / n_block block iterations span the whole space: T's eigenvalues are
    H's (library eigensolver), and the basis is orthonormal with T = V^T H V."""
    space = inputs.SD_SHELL_LIKE
    inter, rng = inputs.random_interaction(space, 1801084321)
    b = ob.build_basis(space, 2, 2, 0)
    H = oh.dense_h(b, inter)
    ev = np.linalg.eigvalsh(H)
    got, T, k, V = ol.block_lanczos(lambda X: H @ X, rng.standard_normal((b.dim, nb)), b.dim // nb, b.dim)
    assert k * nb == b.dim
    assert np.allclose(got, ev, atol=1e-9 * np.max(np.abs(ev)))
    assert np.allclose(V.T @ V, np.eye(b.dim), atol=1e-12)
    assert np.allclose(V.T @ H @ V, T, atol=1e-10 * np.max(np.abs(ev)))


def test_oracle_block_lanczos_projection_and_lowest_states():
    """A partial run: the basis stays orthonormal, T is the projection of H on
    it (this fixes where B_n and B_n^T go), and the lowest five Ritz values
    converge to H's."""
    space = inputs.SD_SHELL_LIKE
    inter, rng = inputs.random_interaction(space, 7)
    b = ob.build_basis(space, 2, 2, 0)
    H = oh.dense_h(b, inter)
    ev = np.linalg.eigvalsh(H)
    got, T, k, V = ol.block_lanczos(lambda X: H @ X, rng.standard_normal((b.dim, 4)), 40, 5)
    assert k == 40
    assert np.allclose(V.T @ V, np.eye(160), atol=1e-12)
    assert np.allclose(V.T @ H @ V, T, atol=1e-10 * np.max(np.abs(ev)))
    assert np.allclose(got, ev[:5], rtol=1e-10)
    # the one-vector block is standard Lanczos: the same Ritz values
    v0 = rng.standard_normal(b.dim)
    one, _, _, _ = ol.block_lanczos(lambda X: H @ X, v0[:, None], 100, 5)
    std, _, _, _ = ol.lanczos(lambda v: H @ v, v0, 100, 5)
    assert np.allclose(one, std, rtol=1e-12)


@pytest.mark.parametrize("two_j,n,two_M,nb", [(9, 4, 0, 4), (7, 4, 0, 4), (9, 5, 1, 4), (9, 4, 0, 8)])
def test_oracle_block_lanczos_resolves_degenerate_seniority_levels(two_j, n, two_M, nb):
    """Single-j pairing: a block of n_block vectors finds a degenerate level as
    many times as its multiplicity (up to n_block, more with the restarts of a
    nearly singular overlap), standard Lanczos only once; the values follow
    the seniority closed form."""
    G = 0.37
    b = ob.build_basis((two_j,), n, 0, two_M)
    H = oh.dense_h(b, _pairing_interaction(two_j, G))
    omega = (two_j + 1) // 2
    levels = []
    for v in range(n % 2, min(n, 2 * omega - n) + 1, 2):
        mult = _sd_count(two_j, v, two_M) - _sd_count(two_j, v - 2, two_M)
        levels.append((-(G / 4.0) * (n - v) * (2 * omega - n - v + 2), mult))
    levels.sort()
    expect = np.concatenate([[e] * m for e, m in levels])
    n_low = min(levels[0][1] + levels[1][1], 6)   # the two lowest levels, with multiplicity
    assert levels[1][1] > 1
    rng = np.random.default_rng(5)
    got, _, _, _ = ol.block_lanczos(lambda X: H @ X, rng.standard_normal((b.dim, nb)), 20, 6)
    assert np.allclose(got[:n_low], expect[:n_low], atol=1e-12)
    assert np.all(got >= expect[:len(got)] - 1e-10)   # Ritz values interlace from above
    one, _, _, _ = ol.block_lanczos(lambda X: H @ X, rng.standard_normal((b.dim, 1)), 20, 6)
    assert len(one) < 6 and np.allclose(one, [e for e, _ in levels][:len(one)], atol=1e-12)


# ------------------------------------------ one-body transition densities
def _random_pair(b, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(b.dim), rng.standard_normal(b.dim)


@pytest.mark.parametrize("space,Z,N,two_M", [(inputs.SD_SHELL_LIKE, 2, 2, 0), (P_SHELL, 3, 2, 1)])
def test_one_body_density_number_sum_rule(space, Z, N, two_M):
    """sum_a p+_a p_a is the proton number operator: trace(rho_p) = Z <g,x>,
    trace(rho_n) = N <g,x>."""
    b = ob.build_basis(space, Z, N, two_M)
    g, x = _random_pair(b, 5)
    rp, rn = oh.one_body_densities(b, g, x)
    assert abs(np.trace(rp) - Z * g @ x) < 1e-10 * np.abs(g) @ np.abs(x)
    assert abs(np.trace(rn) - N * g @ x) < 1e-10 * np.abs(g) @ np.abs(x)


def test_one_body_density_adjoint_and_selection_rule():
    """(p+_a p_c)^T = p+_c p_a: rho(g, x)[a, c] = rho(x, g)[c, a]; entries that
    change m or parity vanish."""
    space = inputs.SD_SHELL_LIKE
    b = ob.build_basis(space, 3, 2, 1)
    g, x = _random_pair(b, 6)
    rp, rn = oh.one_body_densities(b, g, x)
    tp, tn = oh.one_body_densities(b, x, g)
    assert np.max(np.abs(rp - tp.T)) < 1e-12 and np.max(np.abs(rn - tn.T)) < 1e-12
    ms = b.ms
    for a in range(len(ms)):
        for c in range(len(ms)):
            if ms[a][2] != ms[c][2]:
                assert rp[a, c] == 0.0 and rn[a, c] == 0.0


def test_one_body_density_of_a_single_determinant():
    """For one basis state |S>: rho is diagonal with the occupations of S."""
    space = inputs.SD_SHELL_LIKE
    b = ob.build_basis(space, 2, 3, 1)
    ns = len(b.ms)
    for s in (0, b.dim // 2, b.dim - 1):
        e = np.zeros(b.dim)
        e[s] = 1.0
        rp, rn = oh.one_body_densities(b, e, e)
        pm, nm = b.states()[s]
        assert np.array_equal(rp, np.diag([float((pm >> i) & 1) for i in range(ns)]))
        assert np.array_equal(rn, np.diag([float((nm >> i) & 1) for i in range(ns)]))


@pytest.mark.parametrize("space,Z,N,two_M", [(P_SHELL, 2, 2, 0), (inputs.SD_SHELL_LIKE, 2, 1, 1)])
def test_one_body_density_matches_jordan_wigner(space, Z, N, two_M):
    """rho against g^T (a+_a a_c) x with Jordan-Wigner matrices of each species."""
    b = ob.build_basis(space, Z, N, two_M)
    ns = len(b.ms)
    a = jw.annihilators(ns)
    ad = [m.T.tocsr() for m in a]
    states = b.states()
    pidx = np.array([s[0] for s in states])
    nidx = np.array([s[1] for s in states])
    g, x = _random_pair(b, 7)
    rp, rn = oh.one_body_densities(b, g, x)
    for aa in range(ns):
        for cc in range(ns):
            op = (ad[aa] @ a[cc]).tocsr()
            mp = op[pidx][:, pidx].toarray() * (nidx[:, None] == nidx[None, :])
            mn = op[nidx][:, nidx].toarray() * (pidx[:, None] == pidx[None, :])
            assert abs(rp[aa, cc] - g @ mp @ x) < 1e-12
            assert abs(rn[aa, cc] - g @ mn @ x) < 1e-12


def test_one_body_density_c_matches_python():
    space = inputs.SD_SHELL_LIKE
    b = ob.build_basis(space, 3, 3, 0)
    g, x = _random_pair(b, 8)
    rp, rn = oh.one_body_densities(b, g, x)
    cp, cn = of.one_body_densities(of.Prepared(b), g, x)
    assert np.max(np.abs(rp - cp)) < 1e-12 and np.max(np.abs(rn - cn)) < 1e-12


# ----------------------------------- J-coupled elements and their decoupling
from oracle import angmom as am  # noqa: E402


def test_clebsch_gordan_values_and_symmetries():
    s = 1 / math.sqrt(2)
    assert abs(am.clebsch_gordan(1, 1, 1, -1, 2, 0) - s) < 1e-15
    assert abs(am.clebsch_gordan(1, 1, 1, -1, 0, 0) - s) < 1e-15
    assert abs(am.clebsch_gordan(1, -1, 1, 1, 0, 0) + s) < 1e-15
    assert abs(am.clebsch_gordan(2, 2, 2, -2, 0, 0) - 1 / math.sqrt(3)) < 1e-15
    assert abs(am.clebsch_gordan(2, 2, 2, 0, 4, 2) - s) < 1e-15        # (1 1, 1 0 | 2 1)
    assert abs(am.clebsch_gordan(3, 1, 1, 1, 2, 2) + math.sqrt(0.25)) < 1e-15   # (3/2 1/2, 1/2 1/2 | 1 1) = -1/2
    for tj in (1, 3, 5, 7):   # (j m, j -m | 0 0) = (-1)^(j-m) / sqrt(2j+1)
        for tm in range(-tj, tj + 1, 2):
            ref = (-1) ** ((tj - tm) // 2) / math.sqrt(tj + 1)
            assert abs(am.clebsch_gordan(tj, tm, tj, -tm, 0, 0) - ref) < 1e-14
    for tj1, tj2 in ((1, 3), (5, 7), (3, 3), (7, 7)):
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tm1 in range(-tj1, tj1 + 1, 2):
                for tm2 in range(-tj2, tj2 + 1, 2):
                    a = am.clebsch_gordan(tj1, tm1, tj2, tm2, tJ, tm1 + tm2)
                    b = am.clebsch_gordan(tj2, tm2, tj1, tm1, tJ, tm1 + tm2)
                    assert abs(b - (-1) ** ((tj1 + tj2 - tJ) // 2) * a) < 1e-14
        # orthonormality of the coupled basis
        for tM in range(-(tj1 + tj2), tj1 + tj2 + 1, 2):
            Js = [tJ for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2) if abs(tM) <= tJ]
            rows = [(m1, tM - m1) for m1 in range(-tj1, tj1 + 1, 2) if abs(tM - m1) <= tj2]
            C = np.array([[am.clebsch_gordan(tj1, m1, tj2, m2, tJ, tM) for (m1, m2) in rows] for tJ in Js])
            assert np.max(np.abs(C @ C.T - np.eye(len(Js)))) < 1e-13


def test_pair_states_are_normalised_and_pauli():
    ms = ob.m_states((3, 5))
    for a, b in ((0, 0), (0, 1), (1, 1)):
        ja, jb = (3, 5)[a], (3, 5)[b]
        for tJ in range(abs(ja - jb), ja + jb + 1, 2):
            st = am.pair_state(ms, a, b, tJ, 0)
            norm = sum(v * v for v in st.values())
            if a == b and (tJ // 2) % 2 == 1:
                assert norm < 1e-28          # two identical nucleons in one orbit: odd J vanish
            else:
                assert abs(norm - 1.0) < 1e-13


@pytest.mark.parametrize("space", [(1, 3), (1, 3, 5)])
def test_decoupled_j_squared_matches_direct_construction(space):
    """J^2 written as J-coupled elements and decoupled with Clebsch-Gordan
    coefficients equals J^2 built from the j_z, j_+- matrices."""
    direct = am.j_squared_direct(space)
    eps, pp, nn, pn = am.j_squared_coupled(space)
    dec = am.decouple(space, pp, nn, pn)
    assert np.allclose(eps, direct["eps_p"], atol=1e-14)
    for k in ("v_pp", "v_nn", "v_pn"):
        assert np.max(np.abs(dec[k] - direct[k])) < 1e-12, k


def test_decoupled_two_particle_spectrum():
    """Two protons, no single-particle energies: the M-block spectrum is the
    union over J >= |M| of the eigenvalues of each J-coupled V_J matrix."""
    space = (1, 3, 5)
    rng = np.random.default_rng(12)
    pairs_j = {}
    for a in range(3):
        for b in range(a, 3):
            for tJ in range(abs(space[a] - space[b]), space[a] + space[b] + 1, 2):
                if a == b and (tJ // 2) % 2:
                    continue
                pairs_j.setdefault(tJ, []).append((a, b))
    elems, blocks = [], {}
    for tJ, pl in pairs_j.items():
        n = len(pl)
        m = rng.standard_normal((n, n))
        m = m + m.T
        blocks[tJ] = np.linalg.eigvalsh(m)
        for i in range(n):
            for k in range(i, n):
                elems.append(pl[i] + pl[k] + (tJ, m[i, k]))
    dec = am.decouple(space, pp=elems)
    inter = dict(eps_p=np.zeros(3), eps_n=np.zeros(3), v_pp=dec["v_pp"], v_nn=dec["v_nn"], v_pn=dec["v_pn"])
    for two_M in (0, 2, 4):
        b = ob.build_basis(space, 2, 0, two_M)
        ev = np.linalg.eigvalsh(oh.dense_h(b, inter))
        ref = np.sort(np.concatenate([blocks[tJ] for tJ in blocks if tJ >= two_M]))
        assert np.allclose(ev, ref, atol=1e-12), two_M
