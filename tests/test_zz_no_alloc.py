"""fotci_apply_H_vjp_static (the adjoint with the library's static device
scratch, for callers that cannot allocate) against fotci_apply_H_vjp: two
calls in a row through the C-ABI, the second on a smaller basis, every output
(dx and each label-density array) equal to float64 rounding of the atomic
sums (1e-12 relative, the bar of the adjoint's oracle parity)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1801_08432_amd import fotci, inputs

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = "cuda:0"


def _close(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    scale = max(np.abs(b).max(), 1e-300)
    return np.max(np.abs(a - b)) <= 1e-12 * scale


def _one(name, seed):
    w = inputs.workload(name)
    h = fotci.Hamiltonian.build(w["two_j"], w["Z"], w["N"], w["two_M"], w, device=DEV)
    x = torch.from_numpy(inputs.random_vector(h.dim, seed)).to(DEV)
    g = torch.from_numpy(inputs.random_vector(h.dim, seed + 1)).to(DEV)
    print("[no-alloc vjp]", name, h.dim, h.basis.n_nsd, flush=True)
    dx_s, gr_s = h.vjp(x, g, static_scratch=True)
    dx_w, gr_w = h.vjp(x, g)
    torch.cuda.synchronize()
    assert _close(dx_s, dx_w)
    for k in ("eps_p", "eps_n", "v_pp", "v_nn", "v_pn"):
        assert _close(gr_s[k], gr_w[k]), k
    # the densities only (no dx): the same entry point with dx = NULL
    _, gr_s2 = h.vjp(x, g, want_dx=False, static_scratch=True)
    for k in ("eps_n", "v_nn"):
        assert _close(gr_s2[k], gr_w[k]), k


def test_vjp_static_scratch_matches_workspace_variant():
    _one("pf_4p4n", 501)   # 4,845 neutron SDs
    _one("sd_2p2n", 503)   # then a smaller basis: the array keeps the last call's contents
