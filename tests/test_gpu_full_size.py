"""GPU parity at the full-size workloads, through the C-ABI, against the CPU
oracle's C matvec (Ch. 2, "Representation of the Hamiltonian"; Ch. 7,
"Standard Lanczos algorithm" and "Thick-restart Lanczos").

- apply_H on pf_5p5n (dim 18,600,516): every row of y = H x against the
  oracle, float64 to 1e-12 relative L2 and float32 to 1e-5 (x is a float32-
  representable vector, so both paths see the same input; float32 rounding
  2^-24 grown by the ~10^3 terms per row stays far below 1e-5).
- Eigenvalues on pf_5p5n: the lowest 10 of the float32-vector path against
  the float64 path at 1e-5 relative, both thick-restarted to convergence.
- Ritz vectors at pf_4p4n and pf_5p5n: <y, H y> and ||H y - theta y||
  recomputed with the oracle's matvec must equal the eigenvalue and the
  residual the library returns (which it computes with its own float64
  apply_H), so neither rests on the GPU checking itself.
- The convergence flag of thick restart: converged implies that every
  returned residual meets tol * max(1, |E|), in float32 and float64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import basis as ob
from oracle import fast as of
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
        _cache.clear()   # one full-size Hamiltonian resident at a time
        torch.cuda.empty_cache()
        w = inputs.workload(name)
        _say("[setup]", name)
        h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
        o = ob.build_basis(w["two_j"], w["Z"], w["N"], w["two_M"])
        _cache[name] = (w, h, of.Prepared(o))
    return _cache[name]


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_ritz_check(prep, w, y, e_lib, r_lib):
    """Rayleigh quotient and residual of a returned Ritz vector from the
    oracle's matvec; they must match the library's within float64 rounding
    of the two matvecs (the residual up to an absolute 1e-9 MeV)."""
    hy = of.apply_h(prep, w, y)
    yy = float(y @ y)
    theta = float(y @ hy) / yy
    res = float(np.linalg.norm(hy - theta * y) / np.sqrt(yy))
    _say("[ritz] lib E %.12f resid %.3e | oracle E %.12f resid %.3e" % (e_lib, r_lib, theta, res))
    assert abs(theta - e_lib) <= 1e-12 * abs(e_lib)
    assert abs(res - r_lib) <= 1e-9 + 1e-3 * r_lib
    return theta, res


def check_flag(r, tol):
    if r["converged"]:
        assert np.all(r["resid"] <= tol * np.maximum(1.0, np.abs(r["evals"])))


def test_apply_full_vector_pf_5p5n():
    """Every one of the 18.6 M rows, float64 and float32, against the oracle."""
    w, h, prep = setup("pf_5p5n")
    x = inputs.random_vector(h.dim, 13).astype(np.float32).astype(np.float64)
    xt = torch.from_numpy(x).to(DEV)
    _say("[apply] pf_5p5n f64/f32", h.dim)
    y64 = h.apply(xt, mode="f64").cpu().numpy()
    y32 = h.apply(xt.float(), mode="f32").double().cpu().numpy()
    ref = of.apply_h(prep, w, x)
    e64, e32 = rel_l2(y64, ref), rel_l2(y32, ref)
    _say("[apply] rel L2 f64 %.3e f32 %.3e" % (e64, e32))
    assert e64 <= 1e-12
    assert e32 <= 1e-5


def test_thick_restart_f32_vs_f64_pf_5p5n_and_oracle_ritz():
    """Lowest 10 eigenvalues: float32 vectors + float32 matrix-core pn
    against float64, both converged by thick restart; the lowest Ritz vector
    of each run checked with the oracle's matvec."""
    w, h, prep = setup("pf_5p5n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 1802)).to(DEV)
    r64 = h.lanczos_thick_restart(piv, 10, 30, 80, max_restarts=60, mode="f64", tol=1e-8, want_vectors=True)
    _say("[trlan f64] restarts", r64["restarts"], "converged", r64["converged"], "resid", r64["resid"])
    r32 = h.lanczos_thick_restart(piv, 10, 30, 80, max_restarts=60, mode="f32", tol=1e-6, want_vectors=True)
    _say("[trlan f32] restarts", r32["restarts"], "converged", r32["converged"], "resid", r32["resid"])
    rel = np.abs(r32["evals"] - r64["evals"]) / np.abs(r64["evals"])
    _say("[trlan f32 vs f64] rel", rel)
    assert r64["converged"] and r32["converged"]
    check_flag(r64, 1e-8)
    check_flag(r32, 1e-6)
    assert np.all(rel <= 1e-5)
    for r in (r64, r32):
        y = r["evecs"][0].cpu().numpy()
        oracle_ritz_check(prep, w, y, r["evals"][0], r["resid"][0])


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_lanczos_ritz_vectors_pf_4p4n_against_oracle(mode):
    """Standard Lanczos (300 iterations, lowest 10) on pf_4p4n: every returned
    Ritz vector's eigenvalue and residual recomputed with the oracle."""
    w, h, prep = setup("pf_4p4n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 19)).to(DEV)
    r = h.lanczos_lowest(piv, 10, 300, mode=mode, want_vectors=True)
    for k in range(10):
        y = r["evecs"][k].cpu().numpy()
        oracle_ritz_check(prep, w, y, r["evals"][k], r["resid"][k])


def test_thick_restart_flag_means_true_residual():
    """A float32 run asked for a residual below the float32 storage floor
    reports converged = 0; float64 with the same tol converges and meets it."""
    w, h, prep = setup("pf_4p4n")
    piv = torch.from_numpy(inputs.random_vector(h.dim, 34)).to(DEV)
    r64 = h.lanczos_thick_restart(piv, 5, 20, 50, max_restarts=100, mode="f64", tol=1e-10)
    r32 = h.lanczos_thick_restart(piv, 5, 20, 50, max_restarts=100, mode="f32", tol=1e-10)
    _say("[flag] f64", r64["converged"], r64["resid"], "f32", r32["converged"], r32["resid"])
    assert r64["converged"]
    check_flag(r64, 1e-10)
    check_flag(r32, 1e-10)
    assert not r32["converged"]
