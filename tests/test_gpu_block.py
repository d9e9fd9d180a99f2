"""GPU parity of the block apply_H and block Lanczos (Ch. "Block Lanczos").

Block apply: every column of Y = H X, X of shape (dim, n_block) stored
row-wise, against the oracle's apply_H of that column -- float64 to 1e-12
relative L2, float32 vectors to 1e-5 (the bars of the one-vector apply) --
and against the one-vector HIP apply of the same column (float64: the same
per-element arithmetic, 1e-15 relative; float32: the same sums in another
order, 1e-6).
Block Lanczos: eigenvalues against dense eigh and ARPACK on the oracle's
operator (1e-9 relative, float64), the float32-vector path against float64
(1e-5), the seniority closed form with degenerate levels (the multiplicities
a block resolves), and the oracle's own block Lanczos.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis as ob
from oracle import fast as of
from oracle import hamiltonian as oh
from oracle import lanczos as ol
from paper_1801_08432_amd import fotci, inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"
_cache = {}


def _say(*a):
    print(*a, flush=True)


def setup(name):
    if name not in _cache:
        w = inputs.workload(name)
        _say("[setup]", name)
        h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
        o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
        _cache[name] = (w, h, o, of.Prepared(o))
    return _cache[name]


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def block(dim, nb, seed):
    return np.random.default_rng(seed).standard_normal((dim, nb))


@pytest.mark.parametrize("name", ["sd_2p2n", "sd_6p6n", "pf_4p4n"])
@pytest.mark.parametrize("nb", [2, 4, 8])
def test_block_apply_f64_matches_oracle(name, nb):
    w, h, o, prep = setup(name)
    X = block(h.dim, nb, 40 + nb)
    _say("[block apply f64]", name, nb, h.dim)
    Y = h.apply_block(torch.from_numpy(X).to(DEV), mode="f64").cpu().numpy()
    for v in range(nb):
        assert rel_l2(Y[:, v], of.apply_h(prep, w, X[:, v].copy())) <= 1e-12, v


@pytest.mark.parametrize("name", ["sd_6p6n", "pf_4p4n"])
@pytest.mark.parametrize("nb", [2, 4, 8])
def test_block_apply_f32_matches_oracle(name, nb):
    w, h, o, prep = setup(name)
    X = block(h.dim, nb, 50 + nb).astype(np.float32)
    _say("[block apply f32]", name, nb, h.dim)
    Y = h.apply_block(torch.from_numpy(X).to(DEV), mode="f32").double().cpu().numpy()
    for v in range(nb):
        assert rel_l2(Y[:, v], of.apply_h(prep, w, X[:, v].astype(np.float64))) <= 1e-5, v


@pytest.mark.parametrize("mode", ["f64", "f32"])
@pytest.mark.parametrize("nb", [2, 4, 8])
def test_block_apply_equals_one_vector_apply(mode, nb):
    """Per column the block kernels repeat the one-vector kernels' arithmetic
    in float64; in float32 the one-vector pn kernel packs its gather lists per
    pair of tiles and destination parity (shared output row), so the sums run
    in another order and the columns agree to float32 rounding."""
    w, h, o, prep = setup("pf_4p4n")
    dt = torch.float64 if mode == "f64" else torch.float32
    X = torch.from_numpy(block(h.dim, nb, 60 + nb)).to(DEV, dt)
    Y = h.apply_block(X, mode=mode)
    worst = 0.0
    for v in range(nb):
        y1 = h.apply(X[:, v].contiguous(), mode=mode)
        worst = max(worst, float((Y[:, v] - y1).norm() / y1.norm()))
    _say("[block vs one-vector]", mode, nb, "max rel diff", worst)
    assert worst <= (1e-15 if mode == "f64" else 1e-6)


def test_block_apply_shared_row_policy():
    """float32 pn kernel with the output row updated by LDS atomics and with
    the row split by column parity between the waves: both match the oracle."""
    w, h, o, prep = setup("sd_6p6n")
    X = block(h.dim, 4, 70).astype(np.float32)
    Xt = torch.from_numpy(X).to(DEV)
    Y1 = h.apply_block(Xt, mode="f32").double().cpu().numpy()
    h.set_pn_private_rows(False)
    try:
        Y0 = h.apply_block(Xt, mode="f32").double().cpu().numpy()
    finally:
        h.set_pn_private_rows(True)
    for v in range(4):
        ref = of.apply_h(prep, w, X[:, v].astype(np.float64))
        assert rel_l2(Y0[:, v], ref) <= 1e-5 and rel_l2(Y1[:, v], ref) <= 1e-5


def test_block_apply_full_size_sampled_rows():
    """pf_5p5n (dim 18.6M), a block of 4 in float64 and float32: every row of
    three windows (first sector, middle of the largest sector, last rows) of
    every column against the oracle."""
    w, h, o, prep = setup("pf_5p5n")
    X = block(h.dim, 4, 71)
    Xt = torch.from_numpy(X).to(DEV)
    _say("[block apply full size]")
    Y64 = h.apply_block(Xt, mode="f64").cpu().numpy()
    Y32 = h.apply_block(Xt.float(), mode="f32").double().cpu().numpy()
    secs = ob.sector_table(o)
    big = max(secs, key=lambda r: r[3] * r[5])
    mid = big[6] + (big[3] // 2) * big[5]
    for v in range(4):
        xv = X[:, v].copy()
        for (r0, r1) in [(0, 3000), (mid, mid + 10000), (h.dim - 3000, h.dim)]:
            ref = of.apply_h(prep, w, xv, rows=(r0, r1))
            assert rel_l2(Y64[r0:r1, v], ref) <= 1e-12
            assert rel_l2(Y32[r0:r1, v], ref) <= 1e-5


@pytest.mark.parametrize("space,Z,N,two_M,par,opar", [
    ((1, 3, 5), 1, 0, 1, 1, None),           # one proton: H = spe only
    ((1, 3, 5), 0, 0, 0, 1, None),           # vacuum, dim 1
    ((1, 3, 5), 3, 1, 2, 1, None),           # unequal species, odd particle numbers
    ((1, 3, 5, 7), 2, 3, 5, 1, None),        # odd 2M, ragged sectors
    ((1, 3, 5, 1), 2, 2, 0, -1, (1, 1, -1, -1)),  # mixed-parity orbits, negative total parity
    ((7,), 4, 4, 0, 1, None),                # single j shell
    ((1, 3, 5), 12, 11, 3, 1, None),         # filled/near-filled shells
])
def test_block_apply_edge_cases(space, Z, N, two_M, par, opar):
    inter, rng = inputs.random_interaction(space, 31, parity=opar)
    o = ob.build_basis(space, Z, N, two_M, par, orbit_parity=opar)
    b = fotci.Basis(space, Z, N, two_M, par, orbit_parity=opar)
    j = fotci.Jumps(b)
    h = fotci.Hamiltonian(j, inter).upload(DEV)
    H = oh.dense_h(o, inter) if o.dim <= 3000 else None
    for nb in (2, 4, 8):
        X = rng.standard_normal((o.dim, nb))
        ref = H @ X if H is not None else np.stack(
            [of.apply_h(of.Prepared(o), inter, X[:, v].copy()) for v in range(nb)], axis=1)
        Y = h.apply_block(torch.from_numpy(X).to(DEV), mode="f64").cpu().numpy()
        nrm = max(np.linalg.norm(ref), 1e-300)
        assert np.linalg.norm(Y - ref) <= 1e-12 * nrm + 1e-300, nb


def test_block_apply_rejects_bad_arguments():
    w, h, o, prep = setup("sd_2p2n")
    X = torch.zeros(h.dim, 4, dtype=torch.float64, device=DEV)
    with pytest.raises(fotci.FotciError):
        h.apply_block(torch.zeros(h.dim, 3, dtype=torch.float64, device=DEV))
    with pytest.raises(fotci.FotciError):
        h.apply_block(X, mode="f64_plain")
    with pytest.raises(fotci.FotciError):   # x and y overlap
        h.apply_block(X, y=X)
    flat = torch.zeros(h.dim * 4 + 1, dtype=torch.float64, device=DEV)
    with pytest.raises(fotci.FotciError):   # 8-byte aligned only
        h.apply_block(flat[1:].view(h.dim, 4))


@pytest.mark.parametrize("nb", [1, 2, 4, 8])
def test_block_lanczos_f64_matches_dense_eigh(nb):
    w, h, o, prep = setup("sd_2p2n")
    ev = np.linalg.eigvalsh(oh.dense_h(o, w))
    piv = torch.from_numpy(block(h.dim, nb, 80 + nb)).to(DEV)
    r = h.lanczos_block(piv, 5, 320 // nb, mode="f64")
    _say("[block lanczos]", nb, "blocks", r["n_done"], "resid", r["resid"])
    assert np.allclose(r["evals"], ev[:5], rtol=1e-9, atol=0)
    assert np.all(r["resid"] < 1e-6)


@pytest.mark.parametrize("nb", [2, 4, 8])
def test_block_lanczos_full_krylov_space(nb):
    """n_iter * n_block = dim: the block Krylov space is the whole space."""
    space = (1, 3, 5)
    inter, rng = inputs.random_interaction(space, 3)
    o = ob.build_basis(space, 1, 2, 1)   # dim 128, both species, odd 2M
    h = fotci.Hamiltonian.build(space, 1, 2, 1, inter, device=DEV)
    ev = np.linalg.eigvalsh(oh.dense_h(o, inter))
    assert o.dim % nb == 0
    piv = torch.from_numpy(rng.standard_normal((o.dim, nb))).to(DEV)
    r = h.lanczos_block(piv, 5, o.dim // nb, mode="f64")
    assert np.allclose(r["evals"], ev[:5], rtol=1e-10)


@pytest.mark.parametrize("two_j,n,two_M,nb", [(9, 4, 0, 4), (7, 4, 0, 4), (9, 5, 1, 4)])
def test_block_lanczos_degenerate_seniority_levels(two_j, n, two_M, nb):
    """Single-j pairing: the block run finds the second level with its
    multiplicity (restarting nearly dependent columns as the oracle does) and
    matches the closed form and the oracle's block Lanczos."""
    import test_oracle_pins as pins
    G = 0.37
    inter = pins._pairing_interaction(two_j, G)
    o = ob.build_basis((two_j,), n, 0, two_M)
    h = fotci.Hamiltonian.build((two_j,), n, 0, two_M, inter, device=DEV)
    omega = (two_j + 1) // 2
    levels = sorted((-(G / 4.0) * (n - v) * (2 * omega - n - v + 2),
                     pins._sd_count(two_j, v, two_M) - pins._sd_count(two_j, v - 2, two_M))
                    for v in range(n % 2, min(n, 2 * omega - n) + 1, 2))
    expect = np.concatenate([[e] * m for e, m in levels])
    n_low = min(levels[0][1] + levels[1][1], 6)
    P = np.random.default_rng(5).standard_normal((o.dim, nb))
    r = h.lanczos_block(torch.from_numpy(P).to(DEV), 6, 20, mode="f64")
    ref, _, _, _ = ol.block_lanczos(lambda X: oh.dense_h(o, inter) @ X, P, 20, 6)
    _say("[block seniority]", two_j, n, r["evals"], "oracle", ref)
    assert np.allclose(r["evals"][:n_low], expect[:n_low], atol=1e-11)
    assert np.allclose(r["evals"], ref, atol=1e-9)


def test_block_lanczos_f64_sd_6p6n_matches_eigsh():
    """A block of 4, 100 block iterations: lowest 10 against ARPACK."""
    import scipy.sparse.linalg as sla
    w, h, o, prep = setup("sd_6p6n")
    op = of.Operator(prep, w)
    lo = sla.LinearOperator(op.shape, matvec=op.matvec, dtype=np.float64)
    ref = np.sort(sla.eigsh(lo, k=10, which="SA", tol=1e-13, ncv=60,
                            v0=inputs.random_vector(h.dim, 17))[0])
    piv = torch.from_numpy(block(h.dim, 4, 90)).to(DEV)
    r = h.lanczos_block(piv, 10, 100, mode="f64")
    _say("[block lanczos sd_6p6n] resid", r["resid"])
    assert np.allclose(r["evals"], ref, rtol=1e-9, atol=0)


def test_block_lanczos_f32_vs_f64_pf_4p4n():
    """The float32-vector block run against the float64 block run (lowest 10,
    1e-5 relative), and the float64 block run against the one-vector run for
    the states 100 block iterations converge on this dense spectrum (the
    lowest three; block Lanczos needs more iterations than the vector
    recurrence of the same Krylov degree)."""
    w, h, o, prep = setup("pf_4p4n")
    piv = torch.from_numpy(block(h.dim, 4, 91)).to(DEV)
    r64 = h.lanczos_block(piv, 10, 100, mode="f64")
    r32 = h.lanczos_block(piv, 10, 100, mode="f32")
    one = h.lanczos_lowest(torch.from_numpy(inputs.random_vector(h.dim, 19)).to(DEV), 10, 300, mode="f64")
    rel = np.abs(r32["evals"] - r64["evals"]) / np.abs(r64["evals"])
    rel1 = np.abs(r64["evals"] - one["evals"]) / np.abs(one["evals"])
    _say("[block f32 vs f64]", rel, "vs one-vector", rel1, "resid32", r32["resid"])
    assert np.all(rel <= 1e-5) and np.all(rel1[:3] <= 1e-6)


def test_block_lanczos_ritz_vectors_and_rejections():
    w, h, o, prep = setup("sd_2p2n")
    H = oh.dense_h(o, w)
    piv = torch.from_numpy(block(h.dim, 4, 92)).to(DEV)
    r = h.lanczos_block(piv, 5, 40, mode="f32", want_vectors=True)
    vecs = r["evecs"].cpu().numpy()
    for k in range(5):
        y = vecs[k]
        assert abs(np.linalg.norm(y) - 1.0) < 1e-12
        assert abs(y @ H @ y - r["evals"][k]) < 1e-10 * abs(r["evals"][k])
        assert np.linalg.norm(H @ y - r["evals"][k] * y) == pytest.approx(r["resid"][k], rel=1e-6, abs=1e-12)
    bad = piv.clone()
    bad[:, 1] = bad[:, 0]
    with pytest.raises(fotci.FotciError) as ei:
        h.lanczos_block(bad, 5, 40, mode="f64")
    assert ei.value.code == -1
