"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

apply_H in float64 must match the oracle to 1e-12 relative L2 (the float64
rounding of ~10^3 accumulated terms per row is ~1e-14); float32 vectors to
1e-5 (float32 rounding, 2^-24 ~ 6e-8, grown by sqrt of the ~10^3 terms per
row and by cancellation). Eigenvalues: 1e-9 relative (float64), 1e-5 relative
for the float32-vector path against the float64 one.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis as ob
from oracle import fast as of
from oracle import hamiltonian as oh
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


@pytest.mark.parametrize("name", ["sd_2p2n", "sd_6p6n", "pf_4p4n"])
@pytest.mark.parametrize("mode", ["f64_plain", "f64"])
def test_apply_f64_matches_oracle(name, mode):
    w, h, o, prep = setup(name)
    x = inputs.random_vector(h.dim, 11)
    _say("[apply]", name, mode, h.dim)
    y = h.apply(torch.from_numpy(x).to(DEV), mode=mode).cpu().numpy()
    ref = of.apply_h(prep, w, x)
    assert rel_l2(y, ref) <= 1e-12


@pytest.mark.parametrize("name", ["sd_6p6n", "pf_4p4n"])
def test_apply_f32_matches_oracle(name):
    w, h, o, prep = setup(name)
    x = inputs.random_vector(h.dim, 12)
    y = h.apply(torch.from_numpy(x).float().to(DEV), mode="f32").double().cpu().numpy()
    ref = of.apply_h(prep, w, x.astype(np.float32).astype(np.float64))
    assert rel_l2(y, ref) <= 1e-5


def test_apply_f32_shared_row_policy():
    """The float32 pn kernel with the output row updated by LDS atomics and
    with the row split by column parity between the waves (plain updates):
    both match the oracle to float32 rounding."""
    w, h, o, prep = setup("sd_6p6n")
    x = inputs.random_vector(h.dim, 13)
    xt = torch.from_numpy(x).float().to(DEV)
    y1 = h.apply(xt, mode="f32").double().cpu().numpy()
    h.set_pn_private_rows(False)
    try:
        y0 = h.apply(xt, mode="f32").double().cpu().numpy()
    finally:
        h.set_pn_private_rows(True)
    ref = of.apply_h(prep, w, x.astype(np.float32).astype(np.float64))
    assert rel_l2(y0, ref) <= 1e-5 and rel_l2(y1, ref) <= 1e-5


def test_apply_full_size_sampled_rows():
    """pf_5p5n (dim 18.6M): every row of three windows (first sector, the
    middle of the largest sector, the last rows) against the oracle."""
    w, h, o, prep = setup("pf_5p5n")
    x = inputs.random_vector(h.dim, 13)
    xt = torch.from_numpy(x).to(DEV)
    y64 = h.apply(xt, mode="f64").cpu().numpy()
    y32 = h.apply(xt.float(), mode="f32").double().cpu().numpy()
    secs = ob.sector_table(o)
    big = max(secs, key=lambda r: r[3] * r[5])
    mid = big[6] + (big[3] // 2) * big[5]
    for (r0, r1) in [(0, 4000), (mid, mid + 20000), (h.dim - 4000, h.dim)]:
        ref = of.apply_h(prep, w, x, rows=(r0, r1))
        assert rel_l2(y64[r0:r1], ref) <= 1e-12
        assert rel_l2(y32[r0:r1], ref) <= 1e-5


def test_hermitian_and_deterministic():
    w, h, o, prep = setup("sd_6p6n")
    x = torch.from_numpy(inputs.random_vector(h.dim, 14)).to(DEV)
    g = torch.from_numpy(inputs.random_vector(h.dim, 15)).to(DEV)
    hx = h.apply(x)
    hg = h.apply(g)
    a, b = float(g @ hx), float(hg @ x)
    assert abs(a - b) <= 1e-12 * abs(a)
    # the plain kernel is a pure gather: bitwise reproducible; the tiled pn
    # kernel sums through LDS atomics, so only rounding-level agreement
    assert torch.equal(h.apply(x, mode="f64_plain"), h.apply(x, mode="f64_plain"))
    assert float((hx - h.apply(x)).norm() / hx.norm()) < 1e-14


@pytest.mark.parametrize("space,Z,N,two_M,par,opar", [
    ((1, 3, 5), 1, 0, 1, 1, None),           # one proton: H = spe only
    ((1, 3, 5), 0, 0, 0, 1, None),           # vacuum, dim 1
    ((1, 3, 5), 3, 1, 2, 1, None),           # unequal species, odd particle numbers
    ((1, 3, 5, 7), 2, 3, 5, 1, None),        # odd 2M, ragged sectors
    ((1, 3, 5, 1), 2, 2, 0, -1, (1, 1, -1, -1)),  # mixed-parity orbits, negative total parity
    ((7,), 4, 4, 0, 1, None),                # single j shell
    ((1, 3, 5), 12, 11, 3, 1, None),         # filled/near-filled shells
])
def test_apply_edge_cases(space, Z, N, two_M, par, opar):
    inter, rng = inputs.random_interaction(space, 31, parity=opar)
    o = ob.build_basis(space, Z, N, two_M, par, orbit_parity=opar)
    b = fotci.Basis(space, Z, N, two_M, par, orbit_parity=opar)
    j = fotci.Jumps(b)
    h = fotci.Hamiltonian(j, inter).upload(DEV)
    x = rng.standard_normal(o.dim)
    ref = oh.dense_h(o, inter) @ x if o.dim <= 3000 else of.apply_h(of.Prepared(o), inter, x)
    for mode in ("f64_plain", "f64"):
        y = h.apply(torch.from_numpy(x).to(DEV), mode=mode).cpu().numpy()
        nrm = max(np.linalg.norm(ref), 1e-300)
        assert np.linalg.norm(y - ref) <= 1e-12 * nrm + 1e-300
    # the float32 path (split-row pn kernel, staged pp) on the same shapes,
    # against the oracle applied to the float32-rounded vector
    x32 = x.astype(np.float32)
    ref32 = oh.dense_h(o, inter) @ x32.astype(np.float64) if o.dim <= 3000 else \
        of.apply_h(of.Prepared(o), inter, x32.astype(np.float64))
    y32 = h.apply(torch.from_numpy(x32).to(DEV), mode="f32").double().cpu().numpy()
    assert np.linalg.norm(y32 - ref32) <= 1e-5 * np.linalg.norm(ref32) + 1e-30


def test_lanczos_f64_matches_dense_eigh():
    w, h, o, prep = setup("sd_2p2n")
    H = oh.dense_h(o, w)
    ev = np.linalg.eigvalsh(H)
    piv = torch.from_numpy(inputs.random_vector(h.dim, 16)).to(DEV)
    for mode in ("f64_plain", "f64"):
        r = h.lanczos_lowest(piv, 5, 120, mode=mode)
        assert np.allclose(r["evals"], ev[:5], rtol=1e-9, atol=0)
        assert np.all(r["resid"] < 1e-6)


def test_lanczos_full_krylov_space():
    """n_iter = dim: the Krylov space is the whole space; Lanczos breaks down
    at the end and returns the lowest eigenvalues exactly."""
    space = (1, 3)
    inter, rng = inputs.random_interaction(space, 3)
    o = ob.build_basis(space, 2, 2, 0)
    h = fotci.Hamiltonian.build(space, 2, 2, 0, inter, device=DEV)
    ev = np.linalg.eigvalsh(oh.dense_h(o, inter))
    piv = torch.from_numpy(rng.standard_normal(o.dim)).to(DEV)
    r = h.lanczos_lowest(piv, 5, o.dim, mode="f64")
    assert np.allclose(r["evals"], ev[:5], rtol=1e-10)


def test_lanczos_f64_sd_6p6n_matches_eigsh():
    """300 iterations, lowest 10 vs ARPACK on the oracle's matrix-free operator."""
    import scipy.sparse.linalg as sla
    w, h, o, prep = setup("sd_6p6n")
    op = of.Operator(prep, w)
    lo = sla.LinearOperator(op.shape, matvec=op.matvec, dtype=np.float64)
    ref = np.sort(sla.eigsh(lo, k=10, which="SA", tol=1e-13, ncv=60,
                            v0=inputs.random_vector(h.dim, 17))[0])
    piv = torch.from_numpy(inputs.random_vector(h.dim, 18)).to(DEV)
    r = h.lanczos_lowest(piv, 10, 300, mode="f64")
    _say("[lanczos] resid", r["resid"])
    assert np.allclose(r["evals"], ref, rtol=1e-9, atol=0)


def test_lanczos_f32_vs_f64_pf_4p4n():
    w, h, o, prep = setup("pf_4p4n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 19)).to(DEV)
    r64 = h.lanczos_lowest(piv, 10, 300, mode="f64")
    r32 = h.lanczos_lowest(piv, 10, 300, mode="f32")
    rel = np.abs(r32["evals"] - r64["evals"]) / np.abs(r64["evals"])
    _say("[lanczos f32 vs f64] rel err", rel, "resid64", r64["resid"], "resid32", r32["resid"])
    assert np.all(rel <= 1e-5)


def test_lanczos_dgks_reorthogonalisation():
    """The conditional second Gram-Schmidt pass: float64 against ARPACK on
    sd_6p6n, float32 vectors against the always-twice float64 run on pf_4p4n."""
    import scipy.sparse.linalg as sla
    w, h, o, prep = setup("sd_6p6n")
    op = of.Operator(prep, w)
    lo = sla.LinearOperator(op.shape, matvec=op.matvec, dtype=np.float64)
    ref = np.sort(sla.eigsh(lo, k=10, which="SA", tol=1e-13, ncv=60,
                            v0=inputs.random_vector(h.dim, 17))[0])
    piv = torch.from_numpy(inputs.random_vector(h.dim, 18)).to(DEV)
    r = h.lanczos_lowest(piv, 10, 300, mode="f64", reorth="dgks")
    assert np.allclose(r["evals"], ref, rtol=1e-9, atol=0)
    w, h, o, prep = setup("pf_4p4n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 19)).to(DEV)
    r64 = h.lanczos_lowest(piv, 10, 300, mode="f64")
    r32 = h.lanczos_lowest(piv, 10, 300, mode="f32", reorth="dgks")
    rel = np.abs(r32["evals"] - r64["evals"]) / np.abs(r64["evals"])
    _say("[lanczos f32 dgks vs f64] rel err", rel)
    assert np.all(rel <= 1e-5)


def test_vjp_matches_oracle_densities():
    for name in ("sd_2p2n", "sd_6p6n"):
        w, h, o, prep = setup(name)
        x = inputs.random_vector(h.dim, 20)
        g = inputs.random_vector(h.dim, 21)
        dx, gr = h.vjp(torch.from_numpy(x).to(DEV), torch.from_numpy(g).to(DEV))
        ref = of.densities(prep, g, x)
        assert rel_l2(dx.cpu().numpy(), of.apply_h(prep, w, g)) <= 1e-12
        for k in ("eps_p", "eps_n", "v_pp", "v_nn", "v_pn"):
            got = gr[k].cpu().numpy()
            want = ref["d_" + k]
            assert np.allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max()), (name, k)


@pytest.mark.parametrize("name", ["sd_2p2n", "sd_6p6n", "pf_4p4n"])
def test_one_body_density_matches_oracle(name):
    """m-scheme one-body transition densities against the oracle's direct
    operator action (float64; ~10^3-10^6 terms per entry, 1e-12 relative)."""
    w, h, o, prep = setup(name)
    g = inputs.random_vector(h.dim, 21)
    x = inputs.random_vector(h.dim, 22)
    _say("[density]", name, h.dim)
    rp, rn = h.one_body_density(torch.from_numpy(g).to(DEV), torch.from_numpy(x).to(DEV))
    ep, en = of.one_body_densities(prep, g, x)
    scale = np.abs(g) @ np.abs(x)
    assert np.max(np.abs(rp.cpu().numpy() - ep)) <= 1e-12 * scale
    assert np.max(np.abs(rn.cpu().numpy() - en)) <= 1e-12 * scale


def test_occupations_of_the_ground_state():
    """Ground state of sd_6p6n from float64 Lanczos: the density diagonals are
    m-state occupations in [0, 1] summing to Z and N, and match the oracle."""
    w, h, o, prep = setup("sd_6p6n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 23)).to(DEV)
    r = h.lanczos_lowest(piv, 1, 150, mode="f64", want_vectors=True)
    psi = r["evecs"][0].contiguous()
    rp, rn = h.one_body_density(psi, psi)
    occ_p, occ_n = np.diag(rp.cpu().numpy()), np.diag(rn.cpu().numpy())
    assert abs(occ_p.sum() - w["Z"]) < 1e-10 and abs(occ_n.sum() - w["N"]) < 1e-10
    assert occ_p.min() > -1e-12 and occ_p.max() < 1 + 1e-12 and occ_n.min() > -1e-12 and occ_n.max() < 1 + 1e-12
    ep, en = of.one_body_densities(prep, psi.cpu().numpy(), psi.cpu().numpy())
    assert np.max(np.abs(rp.cpu().numpy() - ep)) < 1e-12 and np.max(np.abs(rn.cpu().numpy() - en)) < 1e-12
