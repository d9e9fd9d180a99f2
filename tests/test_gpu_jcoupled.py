"""Rotational invariance on the GPU with J-coupled input (App. A, eq. hamdef):
a random interaction given as J-coupled elements and decoupled by the library
makes H commute with J^2, so
- the levels of the 2M = 2 basis reappear in the 2M = 0 spectrum,
- every eigenvector has <J^2> = J(J+1) for an integer J (J^2 built as a
  J-coupled operator, decoupled by the library and applied with apply_H),
- the decoupled J^2 itself, diagonalised, starts at J = 0 for 2M = 0 and
  at J = 1 for 2M = 2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import angmom as am
from paper_1801_08432_amd import fotci, inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _interaction(space, seed):
    ep, en, pp, nn, pn = inputs.random_jcoupled(space, seed)
    return dict(eps_p=ep, eps_n=en, **fotci.decouple_tbme(space, pp, nn, pn))


def _j_squared(space):
    eps, pp, nn, pn = am.j_squared_coupled(space)
    return dict(eps_p=eps, eps_n=eps.copy(), **fotci.decouple_tbme(space, pp, nn, pn))


def _expect(h, v):
    hv = h.apply(v, mode="f64")
    return float(torch.dot(v, hv) / torch.dot(v, v))


def test_m2_levels_reappear_at_m0():
    space = inputs.SD_SHELL_LIKE
    inter = _interaction(space, 101)
    h0 = fotci.Hamiltonian.build(space, 6, 6, 0, inter, device=DEV)
    h2 = fotci.Hamiltonian.build(space, 6, 6, 2, inter, device=DEV)
    ev0 = h0.lanczos_lowest(torch.from_numpy(inputs.random_vector(h0.dim, 1)).to(DEV), 12, 400, mode="f64")
    ev2 = h2.lanczos_lowest(torch.from_numpy(inputs.random_vector(h2.dim, 2)).to(DEV), 3, 300, mode="f64")
    _say("[jcoupled] M=0", ev0["evals"][:6], "M=2", ev2["evals"])
    for e in ev2["evals"]:
        assert np.min(np.abs(ev0["evals"] - e)) <= 1e-9 * abs(e), e


def test_eigenvectors_have_good_j_pf_4p4n():
    space = inputs.PF_SHELL_LIKE
    inter = _interaction(space, 102)
    h = fotci.Hamiltonian.build(space, 4, 4, 0, inter, device=DEV)
    hj = fotci.Hamiltonian.build(space, 4, 4, 0, _j_squared(space), device=DEV)
    piv = torch.from_numpy(inputs.random_vector(h.dim, 3)).to(DEV)
    r = h.lanczos_lowest(piv, 5, 300, mode="f64", want_vectors=True)
    for k in range(5):
        j2 = _expect(hj, r["evecs"][k].contiguous())
        J = round((-1 + np.sqrt(1 + 4 * j2)) / 2)
        _say("[jcoupled] E %.8f <J^2> %.10f J %d" % (r["evals"][k], j2, J))
        assert abs(j2 - J * (J + 1)) < 1e-7


def test_decoupled_j_squared_spectrum():
    space = inputs.SD_SHELL_LIKE
    jsq = _j_squared(space)
    for two_M, lowest in ((0, 0.0), (2, 2.0)):
        h = fotci.Hamiltonian.build(space, 2, 2, two_M, jsq, device=DEV)
        r = h.lanczos_lowest(torch.from_numpy(inputs.random_vector(h.dim, 4)).to(DEV), 1, min(h.dim, 200),
                             mode="f64")
        assert abs(r["evals"][0] - lowest) < 1e-9
