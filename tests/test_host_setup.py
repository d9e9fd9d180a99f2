"""CPU tests of the library's host side against the oracle (no GPU needed).

Basis tables and jump lists must match the oracle bit-exactly; bad inputs
must be rejected with FOTCI_EINVAL; every symbol the header declares must be
exported.
"""
import os
import re

import numpy as np
import pytest

from oracle import basis as ob
from oracle import hamiltonian as oh
from paper_1801_08432_amd import fotci, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "fotci.h")).read()
    names = set(re.findall(r"\b(fotci_[a-zA-Z0-9_]+)\s*\(", hdr))
    names.discard("fotci_lanczos_opts")
    lib = fotci.lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(fotci.EXPORTED)


@pytest.mark.parametrize("name", list(inputs.WORKLOADS))
def test_basis_matches_oracle(name):
    w = inputs.WORKLOADS[name]
    b = fotci.Basis(w["two_j"], w["Z"], w["N"], w["two_M"], w["parity"])
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"], w["parity"])
    e = b.export()
    assert b.dim == o.dim
    assert np.array_equal(e["p_bits"], np.array(o.p_sds, dtype=np.uint32))
    assert np.array_equal(e["n_bits"], np.array(o.n_sds, dtype=np.uint32))
    assert np.array_equal(e["pstart"], np.array(o.pstart, dtype=np.int64))
    assert np.array_equal(e["nstart"], np.array(o.nstart, dtype=np.int64))
    assert np.array_equal(e["sectors"], np.array(ob.sector_table(o), dtype=np.int64))


@pytest.mark.parametrize("space,Z,N,two_M,par", [((5, 1, 3), 5, 6, 1, 1), ((1, 3), 2, 2, 0, 1)])
def test_basis_printed_cases(space, Z, N, two_M, par):
    o = ob.build_basis(space, Z, N, two_M, par)
    b = fotci.Basis(space, Z, N, two_M, par)
    assert b.dim == o.dim and b.n_psd == len(o.p_sds) and b.n_nsd == len(o.n_sds)


def test_basis_with_mixed_parity_orbits():
    space, opar = (1, 3, 5, 1), (1, 1, -1, -1)
    for tot in (1, -1):
        o = ob.build_basis(space, 3, 2, 1, tot, orbit_parity=opar)
        b = fotci.Basis(space, 3, 2, 1, tot, orbit_parity=opar)
        e = b.export()
        assert np.array_equal(e["sectors"], np.array(ob.sector_table(o), dtype=np.int64))
        assert np.array_equal(e["p_bits"], np.array(o.p_sds, dtype=np.uint32))


def _compare_jumps(b, o, species, kinds, src_subset=None):
    j = fotci.Jumps(b)
    ref = oh.jumps(o, species, src_subset)
    for kind, key in kinds:
        got = j.export(kind)
        if src_subset is not None:
            got = got[np.isin(got[:, 0], np.array(sorted(src_subset)))]
        assert got.shape == ref[key].shape, (species, key)
        assert np.array_equal(got, ref[key]), (species, key)
    return j


@pytest.mark.parametrize("name", ["sd_2p2n", "sd_6p6n"])
def test_jumps_match_oracle_exactly(name):
    w = inputs.WORKLOADS[name]
    b = fotci.Basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    _compare_jumps(b, o, "p", [(fotci.JUMP_PP2, "two_body"), (fotci.JUMP_P1, "one_body")])
    _compare_jumps(b, o, "n", [(fotci.JUMP_NN2, "two_body"), (fotci.JUMP_N1, "one_body")])


def test_jumps_mixed_parity_and_unequal_species():
    space, opar = (1, 3, 5, 1), (1, 1, -1, -1)
    b = fotci.Basis(space, 3, 2, 1, -1, orbit_parity=opar)
    o = ob.build_basis(space, 3, 2, 1, -1, orbit_parity=opar)
    _compare_jumps(b, o, "p", [(fotci.JUMP_PP2, "two_body"), (fotci.JUMP_P1, "one_body")])
    _compare_jumps(b, o, "n", [(fotci.JUMP_NN2, "two_body"), (fotci.JUMP_N1, "one_body")])


@pytest.mark.parametrize("name", ["pf_4p4n", "pf_5p5n"])
def test_jumps_match_oracle_sampled(name):
    w = inputs.WORKLOADS[name]
    b = fotci.Basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    rng = np.random.default_rng(5)
    sub = set(rng.choice(len(o.p_sds), 60, replace=False).tolist()) | {0, len(o.p_sds) - 1}
    j = _compare_jumps(b, o, "p", [(fotci.JUMP_PP2, "two_body"), (fotci.JUMP_P1, "one_body")], sub)
    # closed-form count: every SD has n (N_s - n + 1) one-body jumps when all sectors are kept
    assert j.count(fotci.JUMP_P1) == len(o.p_sds) * w["Z"] * (20 - w["Z"] + 1)


@pytest.mark.parametrize("args", [
    dict(two_j=(1, 3, 5), Z=2, N=2, two_M=1),         # 2M parity vs Z+N
    dict(two_j=(1, 3, 5), Z=13, N=2, two_M=1),        # Z > N_s
    dict(two_j=(1, 3, 5), Z=2, N=2, two_M=40),        # empty basis
    dict(two_j=(2, 3), Z=1, N=1, two_M=0),            # even 2j
    dict(two_j=(31, 3), Z=1, N=1, two_M=0),           # more than 32 m-states
])
def test_bad_basis_arguments_are_rejected(args):
    with pytest.raises(fotci.FotciError) as e:
        fotci.Basis(args["two_j"], args["Z"], args["N"], args["two_M"])
    assert e.value.code == -1


def test_bad_interactions_are_rejected():
    w = inputs.workload("sd_2p2n")
    b = fotci.Basis(w["two_j"], 2, 2, 0)
    j = fotci.Jumps(b)
    fotci.Hamiltonian(j, w)        # the good one is accepted
    bad = dict(w)
    bad["v_pp"] = w["v_pp"].copy()
    bad["v_pp"][0, 1] += 1e-3      # not symmetric
    with pytest.raises(fotci.FotciError):
        fotci.Hamiltonian(j, bad)
    bad = dict(w)
    bad["v_pn"] = w["v_pn"].copy()
    # (a=0,b=0) -> (c=0,d=1) changes 2M: must be zero
    bad["v_pn"][0, 1] = bad["v_pn"][1, 0] = 0.5
    with pytest.raises(fotci.FotciError):
        fotci.Hamiltonian(j, bad)
    bad = dict(w)
    bad["eps_p"] = np.array([np.nan, 0, 0])
    with pytest.raises(fotci.FotciError):
        fotci.Hamiltonian(j, bad)


def test_tridiagonal_solver_matches_numpy():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 17, 120):
        d = rng.standard_normal(n)
        e = rng.standard_normal(max(n - 1, 0))
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        ev, vec = fotci.tridiag_eigh(d, e)
        ref = np.linalg.eigvalsh(T)
        assert np.allclose(ev, ref, atol=1e-12 * max(1, np.abs(ref).max()))
        assert np.allclose(T @ vec, vec * ev, atol=1e-10)
        assert np.allclose(vec.T @ vec, np.eye(n), atol=1e-12)
    # degenerate and split cases
    d = np.array([1.0, 1.0, 1.0, 2.0])
    e = np.array([0.0, 0.0, 1e-300])
    ev, vec = fotci.tridiag_eigh(d, e)
    assert np.allclose(ev, [1, 1, 1, 2])


def test_op_counts_pin():
    """Operation counts per apply_H against Table timetable (Ch. 3): 48Cr in the
    pf shell "1.5 B" ops and 24Mg in the sd shell "8.6 M" (the paper notes an
    operation is only approximately a matrix element)."""
    for (space, Z, N, printed) in [(inputs.PF_SHELL_LIKE, 4, 4, 1.5e9), (inputs.SD_SHELL_LIKE, 4, 4, 8.6e6)]:
        inter, _ = inputs.random_interaction(space, 1)
        h = fotci.Hamiltonian.build(space, Z, N, 0, inter, upload=False)
        c = h.op_counts()
        tot = c["pp"] + c["nn"] + c["pn"] + c["diag"]
        assert 0.85 * printed < tot < 1.15 * printed, (c, tot)


@pytest.mark.parametrize("name", ["sd_2p2n", "sd_6p6n"])
def test_pn_work_counts(name):
    """The pn kernels' work counts, recomputed from the exported jump lists.
    Float64 kernel: a (destination row, class, 32-column source tile) is
    visited when the row has proton jumps of the class and some neutron jump
    of the conjugate class leaves the tile into the row's neutron sector; it
    costs 2 * ceil(n_B / 16) * ceil(k_p / 4) matrix-core instructions; its
    gather list is a whole number of 64-entry rounds, at least
    ceil(entries / 64) (a column's entries may be split over lanes) and at
    most one round per entry. Float32 one-vector kernel: the same per pair of
    source tiles, both existing tiles of a pair with any jump contracted, and
    one list per destination-column parity. In both, a row's proton jumps
    that leave its SD unchanged count as one jump (k_p)."""
    w = inputs.WORKLOADS[name]
    space = w["two_j"]
    inter, _ = inputs.random_interaction(space, 3)
    h = fotci.Hamiltonian.build(space, w["Z"], w["N"], w["two_M"], inter, upload=False)
    got = h.pn_work("f64")
    got32 = h.pn_work("f32")
    b, j = h.basis, h.jumps
    e = b.export()
    ms = ob.m_states(space)
    tm = np.array([m[2] for m in ms])
    ns = len(ms)
    p_sec = np.zeros(b.n_psd, int)
    n_sec = np.zeros(b.n_nsd, int)
    n_loc = np.zeros(b.n_nsd, int)
    for si, (m2, par, pf, npp, nf, nnn, off) in enumerate(e["sectors"]):
        p_sec[pf:pf + npp] = si
        n_sec[nf:nf + nnn] = si
        n_loc[nf:nf + nnn] = np.arange(nnn)
    P1, N1 = j.export(fotci.JUMP_P1), j.export(fotci.JUMP_N1)
    dP = tm[P1[:, 3] // ns] - tm[P1[:, 3] % ns]
    dN = tm[N1[:, 3] // ns] - tm[N1[:, 3] % ns]
    n_ops = {d: len(set(N1[dN == d, 3].tolist())) for d in set(dN.tolist())}
    # neutron entries per (destination sector, delta, source tile): count and largest destination multiplicity
    tiles = {}   # (destination sector, delta) -> source tile -> destination columns
    for (src, dst, ph, lab), d in zip(N1.tolist(), dN.tolist()):
        tiles.setdefault((n_sec[dst], d), {}).setdefault(n_loc[src] // 32, []).append(n_loc[dst])
    visits = mfma = lo = hi = 0
    kp, nd = {}, {}
    for (src, dst, ph, lab), d in zip(P1.tolist(), dP.tolist()):
        kp[(dst, d)] = kp.get((dst, d), 0) + 1
        if src == dst:
            nd[(dst, d)] = nd.get((dst, d), 0) + 1
    # the jumps that leave a row's SD unchanged are contracted as one
    kp = {key: k - max(nd.get(key, 0) - 1, 0) for key, k in kp.items()}
    for (row, d), k in kp.items():
        for ent in tiles.get((p_sec[row], -d), {}).values():
            visits += 1
            mfma += 2 * (-(-n_ops[-d] // 16)) * (-(-k // 4))
            lo += 64 * (-(-len(ent) // 64))
            hi += 64 * len(ent)
    assert got["tile_visits"] == visits and got["mfma_instr"] == mfma
    assert got["gather_slots"] % 64 == 0 and lo <= got["gather_slots"] <= hi
    pairs, n_src = {}, {}   # (destination sector, delta) -> pair -> destination columns by parity
    for (src, dst, ph, lab), d in zip(N1.tolist(), dN.tolist()):
        key = (n_sec[dst], d)
        n_src[key] = int(e["sectors"][n_sec[src]][5])
        pairs.setdefault(key, {}).setdefault(n_loc[src] // 64, ([], []))[n_loc[dst] % 2].append(n_loc[dst])
    visits = mfma = lo = hi = 0
    for (row, d), k in kp.items():
        key = (p_sec[row], -d)
        for pair, lists in pairs.get(key, {}).items():
            nt = min(2, -(-n_src[key] // 32) - 2 * pair)
            visits += nt
            mfma += nt * 2 * (-(-n_ops[-d] // 16)) * (-(-k // 4))
            for ent in lists:
                lo += 64 * (-(-len(ent) // 64))
                hi += 64 * len(ent)
    assert got32["tile_visits"] == visits and got32["mfma_instr"] == mfma
    assert got32["gather_slots"] % 64 == 0 and lo <= got32["gather_slots"] <= hi


def test_pn_private_rows_argument():
    w = inputs.WORKLOADS["sd_2p2n"]
    inter, _ = inputs.random_interaction(w["two_j"], 3)
    h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], inter, upload=False)
    h.set_pn_private_rows(False)
    h.set_pn_private_rows(True)
    with pytest.raises(fotci.FotciError) as ei:
        fotci._check(fotci.lib().fotci_ham_set_pn_private_rows(h._h, 2))
    assert ei.value.code == -1   # FOTCI_EINVAL


def test_dense_symmetric_solver_matches_numpy():
    """The Jacobi solver of thick-restart Lanczos: a random symmetric matrix
    and the restart shape (diagonal block, arrow column, tridiagonal tail)."""
    rng = np.random.default_rng(4)
    a = rng.standard_normal((40, 40))
    a = a + a.T
    b = np.zeros((30, 30))
    b[np.arange(12), np.arange(12)] = np.sort(rng.standard_normal(12))
    b[:12, 12] = b[12, :12] = rng.standard_normal(12)
    for i in range(12, 30):
        b[i, i] = rng.standard_normal()
        if i + 1 < 30:
            b[i, i + 1] = b[i + 1, i] = abs(rng.standard_normal())
    for m in (a, b):
        ev, vec = fotci.sym_eigh(m)
        ref = np.linalg.eigvalsh(m)
        assert np.max(np.abs(ev - ref)) < 1e-12 * np.max(np.abs(ref))
        assert np.max(np.abs(vec.T @ vec - np.eye(len(m)))) < 1e-12
        assert np.max(np.abs(m @ vec - vec * ev)) < 1e-11 * np.max(np.abs(ref))
    with pytest.raises(fotci.FotciError):
        fotci.sym_eigh(np.array([[1.0, 2.0], [3.0, 1.0]]))


def test_thick_restart_options_are_checked():
    w = inputs.WORKLOADS["sd_2p2n"]
    inter, _ = inputs.random_interaction(w["two_j"], 3)
    h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], inter, upload=False)
    assert h.trlan_workspace_bytes(5, 10, 20) > 0
    for bad in [dict(n_keep=5, n_thick=4, n_basis=20), dict(n_keep=5, n_thick=10, n_basis=11),
                dict(n_keep=0, n_thick=10, n_basis=20), dict(n_keep=5, n_thick=10, n_basis=20, tol=0.0)]:
        with pytest.raises(fotci.FotciError):
            h.trlan_workspace_bytes(**bad)


@pytest.mark.parametrize("space,parity", [((1, 3, 5), None), ((1, 3, 5, 7), None), ((1, 3, 3), (1, -1, 1))])
def test_decoupling_matches_oracle(space, parity):
    from oracle import angmom as am
    ep, en, pp, nn, pn = inputs.random_jcoupled(space, 9, parity)
    lib = fotci.decouple_tbme(space, pp, nn, pn, parity)
    ora = am.decouple(space, pp, nn, pn, parity)
    for k in ("v_pp", "v_nn", "v_pn"):
        assert np.max(np.abs(lib[k] - ora[k])) < 1e-13, k
        assert np.array_equal(lib[k], lib[k].T), k
    # the arrays pass the Hamiltonian's checks (exact symmetry, Jz and parity zeros)
    inter = dict(eps_p=ep, eps_n=en, **lib)
    b = fotci.Basis(space, 2, 2, 0, 1, orbit_parity=parity)
    fotci.Hamiltonian(fotci.Jumps(b), inter)


def test_decoupled_j_squared_from_library():
    from oracle import angmom as am
    space = (1, 3, 5)
    eps, pp, nn, pn = am.j_squared_coupled(space)
    lib = fotci.decouple_tbme(space, pp, nn, pn)
    direct = am.j_squared_direct(space)
    for k in ("v_pp", "v_nn", "v_pn"):
        assert np.max(np.abs(lib[k] - direct[k])) < 1e-12, k


@pytest.mark.parametrize("elem,kind", [((1, 0, 1, 0, 2, 1.0), "pp"), ((0, 1, 0, 1, 8, 1.0), "pp"),
                                       ((2, 2, 2, 2, 2, 1.0), "nn"), ((0, 5, 0, 1, 2, 1.0), "pn"),
                                       ((0, 1, 0, 1, 3, 1.0), "pn")])
def test_decoupling_rejects_bad_elements(elem, kind):
    with pytest.raises(fotci.FotciError) as e:
        fotci.decouple_tbme((1, 3, 5), **{kind: [elem]})
    assert e.value.code == -1


def test_decoupling_rejects_parity_change():
    with pytest.raises(fotci.FotciError):
        fotci.decouple_tbme((1, 3), pn=[(0, 0, 0, 1, 2, 1.0)], parity=(1, -1))


def test_package_j_squared_elements_match_oracle():
    """The package's J^2 element list decouples to the oracle's directly built J^2."""
    from oracle import angmom as am
    from paper_1801_08432_amd import observables
    for space in ((1, 3, 5), (1, 3, 5, 7)):
        eps, pp, nn, pn = observables.j_squared(space)
        lib = fotci.decouple_tbme(space, pp, nn, pn)
        direct = am.j_squared_direct(space)
        assert np.allclose(eps, direct["eps_p"], atol=0)
        for k in ("v_pp", "v_nn", "v_pn"):
            assert np.max(np.abs(lib[k] - direct[k])) < 1e-12, k


def test_block_options_and_arguments_are_checked():
    """Block Lanczos options and the block apply's arguments are validated on
    the host before anything touches the device."""
    import ctypes
    w = inputs.WORKLOADS["sd_2p2n"]
    inter, _ = inputs.random_interaction(w["two_j"], 3)
    h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], inter, upload=False)
    good = h.block_lanczos_workspace_bytes(5, 4, 40, "f32")
    assert good > h.block_lanczos_workspace_bytes(5, 4, 20, "f32") > 0
    assert h.block_lanczos_workspace_bytes(5, 4, 40, "f64") > good
    for bad in [dict(n_keep=0, n_block=4, n_iter=10), dict(n_keep=17, n_block=4, n_iter=10),
                dict(n_keep=5, n_block=3, n_iter=10), dict(n_keep=5, n_block=4, n_iter=0),
                dict(n_keep=5, n_block=8, n_iter=513), dict(n_keep=5, n_block=4, n_iter=10, mode="f64_plain")]:
        with pytest.raises(fotci.FotciError) as ei:
            h.block_lanczos_workspace_bytes(**bad)
        assert ei.value.code == -1   # FOTCI_EINVAL
    fake = ctypes.c_void_p(1 << 20)
    apply_block = fotci.lib().fotci_apply_H_block
    for mode, nb, code in [(fotci.MODE_F64, 3, -1), (fotci.MODE_F64_PLAIN, 2, -1), (7, 2, -1),
                           (fotci.MODE_F64, 4, -5), (fotci.MODE_F64_PLAIN, 1, -5)]:
        rc = apply_block(h._h, mode, nb, fake, ctypes.c_void_p((1 << 20) + (1 << 24)), None)
        assert rc == code, (mode, nb, rc)
