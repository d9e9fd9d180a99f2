"""GPU gradients: the adjoint kernel behind torch.autograd against finite
differences of the forward kernels, against the oracle's Hellmann-Feynman
densities, and against the Euler identity (H is linear in the interaction,
so sum_theta theta dE/dtheta = E).

Tolerances: L = <g, H x> is linear in V, so its finite difference with a
unit step is exact up to float64 rounding (1e-9 relative is generous).
Eigenvalue finite differences use central steps h = 1e-4 MeV on
Lanczos eigenvalues converged to ~1e-12; the reading adopted for them is
|g_adj - g_fd| <= 1e-6 + 1e-4 |g|.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis as ob
from oracle import fast as of
from oracle import hamiltonian as oh
from paper_1801_08432_amd import autograd as fag
from paper_1801_08432_amd import fotci, inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"
KEYS = fag.KEYS


def _say(*a):
    print(*a, flush=True)


def _theta(w, requires_grad=True):
    return [torch.tensor(np.asarray(w[k], dtype=np.float64), requires_grad=requires_grad) for k in KEYS]


def _independent_elements(w, ms, rng, n):
    """n random independent interaction elements (kind, r, c) with r <= c."""
    cands = []
    for kind in ("v_pp", "v_nn", "v_pn"):
        v = w[kind]
        r, c = np.nonzero(np.triu(v != 0))
        cands += [(kind, int(a), int(b)) for a, b in zip(r, c)]
    idx = rng.choice(len(cands), n, replace=False)
    return [cands[i] for i in idx]


def _perturbed(w, kind, r, c, h):
    out = {k: np.array(w[k], dtype=np.float64, copy=True) for k in KEYS}
    out[kind][r, c] += h
    if r != c:
        out[kind][c, r] += h
    return out


def _indep_grad(grads, kind, r, c):
    g = grads[kind]
    return float(g[r, c] + (g[c, r] if r != c else 0.0))


def test_apply_vjp_against_forward_finite_differences():
    w = inputs.workload("sd_6p6n")
    ham = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
    x = torch.from_numpy(inputs.random_vector(ham.dim, 40)).to(DEV).requires_grad_(True)
    g = torch.from_numpy(inputs.random_vector(ham.dim, 41)).to(DEV)
    theta = _theta(w)
    y = fag.apply_h(ham, x, theta)
    loss = (g * y).sum()
    loss.backward()
    # dL/dx = H g, against the oracle
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    prep = of.Prepared(o)
    hg = of.apply_h(prep, w, g.cpu().numpy())
    assert np.linalg.norm(x.grad.cpu().numpy() - hg) <= 1e-12 * np.linalg.norm(hg)
    # dL/dtheta against unit-step differences of the forward kernel (exact: L is linear)
    grads = {k: t.grad.numpy() for k, t in zip(KEYS, theta)}
    rng = np.random.default_rng(42)
    base = float(loss)
    xd = x.detach()
    for kind, r, c in _independent_elements(w, o.ms, rng, 24):
        ham.set_values(_perturbed(w, kind, r, c, 1.0))
        l1 = float((g * ham.apply(xd)).sum())
        fd = l1 - base
        ad = _indep_grad(grads, kind, r, c)
        assert abs(fd - ad) <= 1e-9 * max(1.0, abs(base)), (kind, r, c, fd, ad)
    # single-particle energies: one orbit at a time
    for sp in ("eps_p", "eps_n"):
        for o_ in range(len(w["two_j"])):
            pert = {k: np.array(w[k], dtype=np.float64, copy=True) for k in KEYS}
            pert[sp][o_] += 1.0
            ham.set_values(pert)
            fd = float((g * ham.apply(xd)).sum()) - base
            assert abs(fd - float(grads[sp][o_])) <= 1e-9 * max(1.0, abs(base))
    ham.set_values(w)


def test_eigenvalue_gradient_matches_oracle_hellmann_feynman():
    """sd_2p2n: oracle eigenvectors by dense diagonalisation, oracle densities."""
    w = inputs.workload("sd_2p2n")
    rng = np.random.default_rng(7)
    wk = rng.uniform(0, 1, 5)
    ham = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
    theta = _theta(w)
    piv = torch.from_numpy(inputs.random_vector(ham.dim, 43)).to(DEV)
    E = fag.lowest_eigenvalues(ham, piv, 5, 200, theta)
    (E.cpu() * torch.from_numpy(wk)).sum().backward()
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    H = oh.dense_h(o, w)
    ev, vec = np.linalg.eigh(H)
    assert np.allclose(E.detach().cpu().numpy(), ev[:5], rtol=1e-10)
    ref = None
    for k in range(5):
        d = oh.densities(o, vec[:, k], vec[:, k])
        part = {kk: wk[k] * d["d_" + kk] for kk in KEYS}
        ref = part if ref is None else {kk: ref[kk] + part[kk] for kk in KEYS}
    for kk, t in zip(KEYS, theta):
        got = t.grad.numpy()
        assert np.allclose(got, ref[kk], atol=1e-8), kk


@pytest.fixture(scope="module")
def pf_grad():
    """The 4p4n pf-shell gradient workload: L = sum_k w_k E_k over the lowest
    5, w ~ U(0,1); gradients from the adjoint densities."""
    w = inputs.workload("pf_4p4n_grad")
    rng = w["rng"]
    wk = rng.uniform(0, 1, 5)
    ham = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
    theta = _theta(w)
    piv = torch.from_numpy(inputs.random_vector(ham.dim, 44)).to(DEV)
    n_iter = 400
    E = fag.lowest_eigenvalues(ham, piv, 5, n_iter, theta)
    L = (E.cpu() * torch.from_numpy(wk)).sum()
    L.backward()
    grads = {k: t.grad.numpy() for k, t in zip(KEYS, theta)}
    _say("[grad] E", E.detach().cpu().numpy())
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    elements = _independent_elements(w, o.ms, rng, 64)
    yield dict(w=w, wk=wk, ham=ham, piv=piv, n_iter=n_iter, L=float(L.detach()), grads=grads,
               elements=elements)
    ham.set_values(w)


def test_eigenvalue_gradient_pf_4p4n_euler(pf_grad):
    """Euler identity: H is linear in theta, so sum theta dL/dtheta = L."""
    w, grads, L = pf_grad["w"], pf_grad["grads"], pf_grad["L"]
    euler = sum(float(np.sum(grads[k] * np.asarray(w[k]))) for k in KEYS)
    _say("[grad] Euler identity: sum theta dL/dtheta = %.12f, L = %.12f" % (euler, L))
    assert abs(euler - L) <= 1e-9 * abs(L)


def test_eigenvalue_gradient_pf_4p4n_matches_oracle_densities(pf_grad):
    """dL/dtheta from the adjoint kernel against sum_k w_k <psi_k|dH/dtheta|psi_k>
    computed by the oracle (float64, direct operator action) on the float64
    Lanczos eigenvectors of the same run (Hellmann-Feynman)."""
    w, wk, ham, piv = pf_grad["w"], pf_grad["wk"], pf_grad["ham"], pf_grad["piv"]
    r = ham.lanczos_lowest(piv, 5, pf_grad["n_iter"], mode="f64", want_vectors=True)
    _say("[grad] resid", r["resid"])
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    prep = of.Prepared(o)
    ref = None
    for k in range(5):
        v = r["evecs"][k].cpu().numpy()
        d = of.densities(prep, v, v)
        part = {kk: wk[k] * d["d_" + kk] for kk in KEYS}
        ref = part if ref is None else {kk: ref[kk] + part[kk] for kk in KEYS}
        _say("[grad] oracle densities of state", k)
    for kk in KEYS:
        err = np.max(np.abs(pf_grad["grads"][kk] - ref[kk]))
        _say("[grad]", kk, "max |adjoint - oracle|", err)
        assert err <= 1e-8, kk


@pytest.mark.parametrize("chunk", range(4))
def test_eigenvalue_gradient_pf_4p4n_fd(pf_grad, chunk):
    """Adjoint densities against central differences (h = 1e-4 MeV) of the
    float64 Lanczos eigenvalues, on 64 random independent elements (16 per
    chunk)."""
    import time
    w, wk, ham, piv = pf_grad["w"], pf_grad["wk"], pf_grad["ham"], pf_grad["piv"]
    h = 1e-4
    worst = 0.0
    for i in range(16 * chunk, 16 * chunk + 16):
        kind, r, c = pf_grad["elements"][i]
        t0 = time.time()
        vals = []
        for sgn in (1.0, -1.0):
            ham.set_values(_perturbed(w, kind, r, c, sgn * h))
            ev = ham.lanczos_lowest(piv, 5, pf_grad["n_iter"], mode="f64")["evals"]
            vals.append(float(np.dot(wk, ev)))
        ham.set_values(w)
        fd = (vals[0] - vals[1]) / (2 * h)
        ad = _indep_grad(pf_grad["grads"], kind, r, c)
        worst = max(worst, abs(fd - ad) / (1e-6 + 1e-4 * abs(ad)))
        _say("[grad] %2d %s[%d,%d] fd %.9f adjoint %.9f (%.1f s)" % (i, kind, r, c, fd, ad, time.time() - t0))
        assert abs(fd - ad) <= 1e-6 + 1e-4 * abs(ad), (kind, r, c, fd, ad)
    _say("[grad] worst FD ratio to tolerance", worst)
