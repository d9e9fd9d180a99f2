"""GPU thick-restart Lanczos (Ch. 7, "Thick-restart Lanczos") against the
oracle's eigenvalues: dense diagonalisation on the small space, ARPACK on the
oracle's operator for sd_6p6n, and the float64 path for the float32-vector
path on pf_4p4n. Every case checks that restarts actually happened (or, for a
basis smaller than n_basis, that the Krylov space closed exactly)."""
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


def _say(*a):
    print(*a, flush=True)


def _build(name):
    w = inputs.workload(name)
    h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
    return w, h


def test_thick_restart_sd_2p2n_matches_dense():
    w, h = _build("sd_2p2n")
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    ref = np.linalg.eigvalsh(oh.dense_h(o, w))[:5]
    piv = torch.from_numpy(inputs.random_vector(h.dim, 31)).to(DEV)
    r = h.lanczos_thick_restart(piv, 5, 10, 20, max_restarts=200, mode="f64", tol=1e-11)
    _say("[trlan] restarts", r["restarts"], "applies", r["applies"], "resid", r["resid"])
    assert r["converged"] and r["restarts"] >= 1
    assert np.allclose(r["evals"], ref, rtol=1e-9, atol=0)
    assert np.all(r["resid"] <= 1e-8 * np.abs(ref))


def test_thick_restart_exact_when_the_space_is_small():
    """dim < n_basis: the Krylov space closes inside the first cycle."""
    space, Z, N = (1, 3), 1, 1
    inter, _ = inputs.random_interaction(space, 77)
    h = fotci.Hamiltonian.build(space, Z, N, 0, inter, device=DEV)
    o = ob.build_basis(space, Z, N, 0)
    ref = np.linalg.eigvalsh(oh.dense_h(o, inter))
    piv = torch.from_numpy(inputs.random_vector(h.dim, 32)).to(DEV)
    r = h.lanczos_thick_restart(piv, min(4, h.dim), min(4, h.dim), h.dim + 5, mode="f64")
    assert r["converged"] and r["restarts"] == 0
    assert np.allclose(r["evals"], ref[:len(r["evals"])], rtol=1e-10, atol=1e-12)


def test_thick_restart_sd_6p6n_matches_eigsh():
    import scipy.sparse.linalg as sla
    w, h = _build("sd_6p6n")
    o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
    op = of.Operator(of.Prepared(o), w)
    lo = sla.LinearOperator(op.shape, matvec=op.matvec, dtype=np.float64)
    ref = np.sort(sla.eigsh(lo, k=10, which="SA", tol=1e-13, ncv=60, v0=inputs.random_vector(h.dim, 17))[0])
    piv = torch.from_numpy(inputs.random_vector(h.dim, 33)).to(DEV)
    r = h.lanczos_thick_restart(piv, 10, 25, 45, max_restarts=200, mode="f64", tol=1e-11)
    _say("[trlan] restarts", r["restarts"], "applies", r["applies"], "resid", r["resid"])
    assert r["converged"] and r["restarts"] >= 1
    assert np.allclose(r["evals"], ref, rtol=1e-9, atol=0)


def test_thick_restart_f32_vs_f64_pf_4p4n():
    """Float32 vectors and matrix-core pn against float64, both thick-restarted
    with a 61-vector basis (the standard path would hold 300)."""
    w, h = _build("pf_4p4n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 34)).to(DEV)
    r64 = h.lanczos_thick_restart(piv, 10, 25, 60, max_restarts=100, mode="f64", tol=1e-9)
    r32 = h.lanczos_thick_restart(piv, 10, 25, 60, max_restarts=100, mode="f32", tol=1e-9)
    rel = np.abs(r32["evals"] - r64["evals"]) / np.abs(r64["evals"])
    _say("[trlan f32 vs f64] rel", rel, "restarts", r64["restarts"], r32["restarts"])
    assert r64["converged"] and r64["restarts"] >= 1
    assert np.all(rel <= 1e-5)
    # the flag reports the true float64 residual of the returned vectors
    for r in (r64, r32):
        if r["converged"]:
            assert np.all(r["resid"] <= 1e-9 * np.maximum(1.0, np.abs(r["evals"])))
