"""ctypes binding of libfotci (argument marshalling only).

Every step of the path runs in the library: host setup in its C++ code,
apply_H, its adjoint and Lanczos in its HIP kernels. PyTorch provides device
memory (workspaces and vectors are torch tensors) and the current HIP stream.
There is no fallback: if the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfotci.so")

MODE_F64_PLAIN = 0
MODE_F64 = 1
MODE_F32 = 2
MODES = {"f64_plain": MODE_F64_PLAIN, "f64": MODE_F64, "f32": MODE_F32}
REORTH = {"cgs2": 0, "dgks": 1}

JUMP_PP2, JUMP_NN2, JUMP_P1, JUMP_N1 = 0, 1, 2, 3

EXPORTED = [
    "fotci_last_error", "fotci_version", "fotci_build_basis", "fotci_free_basis", "fotci_basis_info",
    "fotci_basis_export", "fotci_build_jumps", "fotci_free_jumps", "fotci_jumps_count", "fotci_jumps_export",
    "fotci_set_interaction", "fotci_free_ham", "fotci_ham_set_values", "fotci_ham_workspace_bytes",
    "fotci_ham_upload", "fotci_apply_H", "fotci_apply_H_vjp", "fotci_apply_H_vjp_static", "fotci_one_body_density",
    "fotci_lanczos_workspace_bytes",
    "fotci_lanczos_lowest", "fotci_trlan_workspace_bytes", "fotci_lanczos_thick_restart",
    "fotci_ham_op_counts", "fotci_ham_pn_work", "fotci_ham_set_pn_private_rows",
    "fotci_tridiag_eigh", "fotci_sym_eigh", "fotci_decouple_tbme", "fotci_profile_start",
    "fotci_profile_stop", "fotci_apply_H_block", "fotci_block_lanczos_workspace_bytes", "fotci_lanczos_block",
]


class FotciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fotci error %d: %s" % (code, msg))
        self.code = code


class LanczosOpts(ctypes.Structure):
    _fields_ = [("n_keep", ctypes.c_int32), ("n_iter", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("refine", ctypes.c_int32), ("reorth", ctypes.c_int32)]


class Tbme(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("c", ctypes.c_int32), ("d", ctypes.c_int32),
                ("two_J", ctypes.c_int32), ("v", ctypes.c_double)]


class TrlanOpts(ctypes.Structure):
    _fields_ = [("n_keep", ctypes.c_int32), ("n_thick", ctypes.c_int32), ("n_basis", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("mode", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("tol", ctypes.c_double)]


class BlockLanczosOpts(ctypes.Structure):
    _fields_ = [("n_keep", ctypes.c_int32), ("n_block", ctypes.c_int32), ("n_iter", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("refine", ctypes.c_int32)]


_lib = None


def lib():
    """Load libfotci.so (built in-tree by build.py); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfotci.so is not built (run paper_1801_08432_amd/build.py)")
    l = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "fotci_last_error": (ctypes.c_char_p, []),
        "fotci_version": (ctypes.c_char_p, []),
        "fotci_build_basis": (ctypes.c_int, [I32, P, P, I32, I32, I32, I32, P]),
        "fotci_free_basis": (None, [P]),
        "fotci_basis_info": (ctypes.c_int, [P, P, P, P, P, P]),
        "fotci_basis_export": (ctypes.c_int, [P, P, P, P, P, P]),
        "fotci_build_jumps": (ctypes.c_int, [P, P]),
        "fotci_free_jumps": (None, [P]),
        "fotci_jumps_count": (ctypes.c_int, [P, I32, P]),
        "fotci_jumps_export": (ctypes.c_int, [P, I32, P, P, P, P]),
        "fotci_set_interaction": (ctypes.c_int, [P, P, P, P, P, P, P]),
        "fotci_free_ham": (None, [P]),
        "fotci_ham_set_values": (ctypes.c_int, [P, P, P, P, P, P, P]),
        "fotci_ham_workspace_bytes": (I64, [P]),
        "fotci_ham_upload": (ctypes.c_int, [P, P, I64, P]),
        "fotci_apply_H": (ctypes.c_int, [P, I32, P, P, P]),
        "fotci_apply_H_vjp": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P]),
        "fotci_apply_H_vjp_static": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P]),
        "fotci_one_body_density": (ctypes.c_int, [P, P, P, P, P, P]),
        "fotci_lanczos_workspace_bytes": (I64, [P, P]),
        "fotci_lanczos_lowest": (ctypes.c_int, [P, P, P, P, I64, P, P, P, P, P, P]),
        "fotci_trlan_workspace_bytes": (I64, [P, P]),
        "fotci_lanczos_thick_restart": (ctypes.c_int, [P, P, P, P, I64, P, P, P, P, P]),
        "fotci_ham_op_counts": (ctypes.c_int, [P, P, P, P, P]),
        "fotci_ham_pn_work": (ctypes.c_int, [P, ctypes.c_int32, P, P, P]),
        "fotci_ham_set_pn_private_rows": (ctypes.c_int, [P, ctypes.c_int32]),
        "fotci_tridiag_eigh": (ctypes.c_int, [I32, P, P, P, P]),
        "fotci_sym_eigh": (ctypes.c_int, [I32, P, P, P]),
        "fotci_decouple_tbme": (ctypes.c_int, [I32, P, P, I32, P, I32, P, I32, P, P, P, P]),
        "fotci_profile_start": (ctypes.c_int, [P, I32]),
        "fotci_profile_stop": (ctypes.c_int, [P, P, P, P, P]),
        "fotci_apply_H_block": (ctypes.c_int, [P, I32, I32, P, P, P]),
        "fotci_block_lanczos_workspace_bytes": (I64, [P, P]),
        "fotci_lanczos_block": (ctypes.c_int, [P, P, P, P, I64, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args
    _lib = l
    return l


def _check(rc):
    if rc != 0:
        raise FotciError(rc, lib().fotci_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Basis:
    """fotci_build_basis: the factorised M-scheme basis (host)."""

    def __init__(self, two_j, Z, N, two_M, parity=1, orbit_parity=None):
        two_j = np.ascontiguousarray(two_j, dtype=np.int32)
        par = np.ascontiguousarray(orbit_parity if orbit_parity is not None else np.ones(len(two_j)),
                                   dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().fotci_build_basis(len(two_j), _np_ptr(two_j), _np_ptr(par), Z, N, two_M, parity,
                                       ctypes.byref(h)))
        self._h = h
        self.two_j, self.Z, self.N, self.two_M, self.parity = tuple(int(x) for x in two_j), Z, N, two_M, parity
        dim, nsec, npsd, nnsd, ns = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fotci_basis_info(h, ctypes.byref(dim), ctypes.byref(nsec), ctypes.byref(npsd),
                                      ctypes.byref(nnsd), ctypes.byref(ns)))
        self.dim, self.n_sectors, self.n_psd, self.n_nsd, self.n_states = (
            dim.value, nsec.value, npsd.value, nnsd.value, ns.value)

    def export(self):
        pb = np.zeros(self.n_psd, np.uint32)
        nb = np.zeros(self.n_nsd, np.uint32)
        ps = np.zeros(self.n_psd, np.int64)
        nst = np.zeros(self.n_nsd, np.int64)
        st = np.zeros((self.n_sectors, 7), np.int64)
        _check(lib().fotci_basis_export(self._h, _np_ptr(pb), _np_ptr(nb), _np_ptr(ps), _np_ptr(nst), _np_ptr(st)))
        return dict(p_bits=pb, n_bits=nb, pstart=ps, nstart=nst, sectors=st)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fotci_free_basis(self._h)
            self._h = None


class Jumps:
    """fotci_build_jumps: one-species jump lists (host)."""

    def __init__(self, basis):
        h = ctypes.c_void_p()
        _check(lib().fotci_build_jumps(basis._h, ctypes.byref(h)))
        self._h = h
        self.basis = basis

    def count(self, kind):
        c = ctypes.c_int64()
        _check(lib().fotci_jumps_count(self._h, kind, ctypes.byref(c)))
        return c.value

    def export(self, kind):
        n = self.count(kind)
        src = np.zeros(n, np.int32)
        dst = np.zeros(n, np.int32)
        ph = np.zeros(n, np.int8)
        lab = np.zeros(n, np.int32)
        _check(lib().fotci_jumps_export(self._h, kind, _np_ptr(src), _np_ptr(dst), _np_ptr(ph), _np_ptr(lab)))
        return np.stack([src.astype(np.int64), dst.astype(np.int64), ph.astype(np.int64), lab.astype(np.int64)], 1)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fotci_free_jumps(self._h)
            self._h = None


def _inter_arrays(inter):
    a = {k: np.ascontiguousarray(inter[k], dtype=np.float64) for k in ("eps_p", "eps_n", "v_pp", "v_nn", "v_pn")}
    return a


class Hamiltonian:
    """fotci_set_interaction (+ upload): H on a basis, resident on the GPU."""

    def __init__(self, jumps, inter):
        self.jumps = jumps
        self.basis = jumps.basis
        self.dim = self.basis.dim
        a = _inter_arrays(inter)
        h = ctypes.c_void_p()
        _check(lib().fotci_set_interaction(jumps._h, _np_ptr(a["eps_p"]), _np_ptr(a["eps_n"]), _np_ptr(a["v_pp"]),
                                           _np_ptr(a["v_nn"]), _np_ptr(a["v_pn"]), ctypes.byref(h)))
        self._h = h
        self.ws = None

    @classmethod
    def build(cls, two_j, Z, N, two_M, inter, parity=1, upload=True, device="cuda"):
        b = Basis(two_j, Z, N, two_M, parity)
        j = Jumps(b)
        h = cls(j, inter)
        if upload:
            h.upload(device)
        return h

    def workspace_bytes(self):
        n = lib().fotci_ham_workspace_bytes(self._h)
        if n < 0:
            _check(int(n))
        return int(n)

    def upload(self, device="cuda", stream=None):
        import torch
        nbytes = self.workspace_bytes()
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        _check(lib().fotci_ham_upload(self._h, self._ws_ptr, nbytes, _stream(stream)))
        return self

    def set_values(self, inter, stream=None):
        a = _inter_arrays(inter)
        _check(lib().fotci_ham_set_values(self._h, _np_ptr(a["eps_p"]), _np_ptr(a["eps_n"]), _np_ptr(a["v_pp"]),
                                          _np_ptr(a["v_nn"]), _np_ptr(a["v_pn"]),
                                          _stream(stream) if self.ws is not None else None))

    def op_counts(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().fotci_ham_op_counts(self._h, *[ctypes.byref(x) for x in v]))
        return dict(pp=v[0].value, nn=v[1].value, pn=v[2].value, diag=v[3].value)

    def pn_work(self, mode="f32"):
        """Visited tiles, matrix-core instructions and gather slots of the pn kernel per apply in `mode`."""
        v = [ctypes.c_int64() for _ in range(3)]
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        _check(lib().fotci_ham_pn_work(self._h, m, *[ctypes.byref(x) for x in v]))
        return dict(tile_visits=v[0].value, mfma_instr=v[1].value, gather_slots=v[2].value)

    def set_pn_private_rows(self, enable):
        _check(lib().fotci_ham_set_pn_private_rows(self._h, 1 if enable else 0))

    def apply(self, x, y=None, mode="f64", stream=None):
        """y = H x on the device (x: float64 for f64 modes, float32 otherwise)."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        dt = torch.float64 if m in (MODE_F64, MODE_F64_PLAIN) else torch.float32
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous() or x.numel() != self.dim:
            raise ValueError("x must be a contiguous %s device vector of length %d" % (dt, self.dim))
        if y is None:
            y = torch.empty_like(x)
        _check(lib().fotci_apply_H(self._h, m, _dev_ptr(x), _dev_ptr(y), _stream(stream)))
        return y

    def apply_block(self, x, y=None, mode="f64", stream=None):
        """Y = H X for a block X of shape (dim, n_block), row-major (vector index fastest)."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        dt = torch.float64 if m in (MODE_F64, MODE_F64_PLAIN) else torch.float32
        if (x.dtype != dt or not x.is_cuda or not x.is_contiguous() or x.dim() != 2 or x.shape[0] != self.dim):
            raise ValueError("x must be a contiguous %s device tensor of shape (%d, n_block)" % (dt, self.dim))
        if y is None:
            y = torch.empty_like(x)
        _check(lib().fotci_apply_H_block(self._h, m, int(x.shape[1]), _dev_ptr(x), _dev_ptr(y), _stream(stream)))
        return y

    def vjp(self, x, g, want_dx=True, stream=None, static_scratch=False):
        """(dx, grads) of L = <g, H x>: dx = H g and label-wise densities.
        static_scratch: call fotci_apply_H_vjp_static (the library's static
        device scratch instead of the Hamiltonian's workspace)."""
        import torch
        ns = self.basis.n_states
        npairs = ns * (ns - 1) // 2
        n_orb = len(self.basis.two_j)
        dev = x.device
        grads = dict(eps_p=torch.zeros(n_orb, dtype=torch.float64, device=dev),
                     eps_n=torch.zeros(n_orb, dtype=torch.float64, device=dev),
                     v_pp=torch.zeros(npairs, npairs, dtype=torch.float64, device=dev),
                     v_nn=torch.zeros(npairs, npairs, dtype=torch.float64, device=dev),
                     v_pn=torch.zeros(ns * ns, ns * ns, dtype=torch.float64, device=dev))
        dx = torch.empty_like(x) if want_dx else None
        fn = lib().fotci_apply_H_vjp_static if static_scratch else lib().fotci_apply_H_vjp
        _check(fn(self._h, _dev_ptr(x), _dev_ptr(g), _dev_ptr(dx), _dev_ptr(grads["eps_p"]),
                  _dev_ptr(grads["eps_n"]), _dev_ptr(grads["v_pp"]), _dev_ptr(grads["v_nn"]),
                  _dev_ptr(grads["v_pn"]), _stream(stream)))
        return dx, grads

    def one_body_density(self, g, x, stream=None):
        """(rho_p, rho_n): device float64 [N_s, N_s] with rho[a, c] = <g| c+_a c_c |x>."""
        import torch
        ns = self.basis.n_states
        rp = torch.empty(ns, ns, dtype=torch.float64, device=x.device)
        rn = torch.empty_like(rp)
        _check(lib().fotci_one_body_density(self._h, _dev_ptr(g), _dev_ptr(x), _dev_ptr(rp), _dev_ptr(rn),
                                            _stream(stream)))
        return rp, rn

    def lanczos_workspace_bytes(self, n_keep, n_iter, mode="f64", refine=True):
        o = LanczosOpts(n_keep, n_iter, MODES[mode] if isinstance(mode, str) else int(mode), int(refine), 0)
        n = lib().fotci_lanczos_workspace_bytes(self._h, ctypes.byref(o))
        if n < 0:
            _check(int(n))
        return int(n)

    def lanczos_lowest(self, pivot, n_keep, n_iter, mode="f64", refine=True, want_vectors=False,
                       work=None, stream=None, reorth="cgs2"):
        """Lowest n_keep eigenvalues; returns dict(evals, resid, alpha, beta[, evecs])."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        o = LanczosOpts(n_keep, n_iter, m, int(refine), REORTH[reorth])
        nbytes = self.lanczos_workspace_bytes(n_keep, n_iter, m, refine)
        if work is None or work.numel() < nbytes + 256:
            work = torch.empty(nbytes + 256, dtype=torch.uint8, device=pivot.device)
        off = (-work.data_ptr()) % 256
        wptr = ctypes.c_void_p(work.data_ptr() + off)
        if pivot.dtype != torch.float64 or pivot.numel() != self.dim or not pivot.is_contiguous():
            raise ValueError("pivot must be a contiguous float64 device vector of length dim")
        evals = np.zeros(n_keep)
        resid = np.zeros(n_keep)
        alpha = np.zeros(n_iter)
        beta = np.zeros(n_iter)
        evecs = torch.empty(n_keep, self.dim, dtype=torch.float64, device=pivot.device) if want_vectors else None
        _check(lib().fotci_lanczos_lowest(self._h, ctypes.byref(o), _dev_ptr(pivot), wptr, nbytes, _np_ptr(evals),
                                          _np_ptr(resid), _dev_ptr(evecs), _np_ptr(alpha), _np_ptr(beta),
                                          _stream(stream)))
        out = dict(evals=evals, resid=resid, alpha=alpha, beta=beta)
        if want_vectors:
            out["evecs"] = evecs
        return out

    def block_lanczos_workspace_bytes(self, n_keep, n_block, n_iter, mode="f64", refine=True):
        o = BlockLanczosOpts(n_keep, n_block, n_iter, MODES[mode] if isinstance(mode, str) else int(mode),
                             int(refine))
        n = lib().fotci_block_lanczos_workspace_bytes(self._h, ctypes.byref(o))
        if n < 0:
            _check(int(n))
        return int(n)

    def lanczos_block(self, pivot, n_keep, n_iter, mode="f64", refine=True, want_vectors=False, work=None,
                      stream=None):
        """Block Lanczos from a pivot block (dim, n_block) float64; returns dict(evals, resid, n_done[, evecs])."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        if (pivot.dtype != torch.float64 or pivot.dim() != 2 or pivot.shape[0] != self.dim
                or not pivot.is_contiguous()):
            raise ValueError("pivot must be a contiguous float64 device tensor of shape (dim, n_block)")
        nb = int(pivot.shape[1])
        o = BlockLanczosOpts(n_keep, nb, n_iter, m, int(refine))
        nbytes = self.block_lanczos_workspace_bytes(n_keep, nb, n_iter, m, refine)
        if work is None or work.numel() < nbytes + 256:
            work = torch.empty(nbytes + 256, dtype=torch.uint8, device=pivot.device)
        wptr = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        evals = np.zeros(n_keep)
        resid = np.zeros(n_keep)
        done = np.zeros(1, dtype=np.int32)
        evecs = torch.empty(n_keep, self.dim, dtype=torch.float64, device=pivot.device) if want_vectors else None
        _check(lib().fotci_lanczos_block(self._h, ctypes.byref(o), _dev_ptr(pivot), wptr, nbytes, _np_ptr(evals),
                                         _np_ptr(resid), _dev_ptr(evecs), _np_ptr(done), _stream(stream)))
        out = dict(evals=evals, resid=resid, n_done=int(done[0]), workspace_bytes=int(nbytes))
        if want_vectors:
            out["evecs"] = evecs
        return out

    def lanczos_thick_restart(self, pivot, n_keep, n_thick, n_basis, max_restarts=50, mode="f64", refine=True,
                              tol=1e-10, want_vectors=False, stream=None, reorth="cgs2"):
        """Thick-restart Lanczos; returns dict(evals, resid, restarts, applies, converged[, evecs])."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        o = TrlanOpts(n_keep, n_thick, n_basis, max_restarts, m, int(refine), REORTH[reorth], float(tol))
        nbytes = lib().fotci_trlan_workspace_bytes(self._h, ctypes.byref(o))
        if nbytes < 0:
            _check(int(nbytes))
        if pivot.dtype != torch.float64 or pivot.numel() != self.dim or not pivot.is_contiguous():
            raise ValueError("pivot must be a contiguous float64 device vector of length dim")
        work = torch.empty(nbytes + 256, dtype=torch.uint8, device=pivot.device)
        wptr = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
        evals = np.zeros(n_keep)
        resid = np.zeros(n_keep)
        stats = np.zeros(3, dtype=np.int32)
        evecs = torch.empty(n_keep, self.dim, dtype=torch.float64, device=pivot.device) if want_vectors else None
        _check(lib().fotci_lanczos_thick_restart(self._h, ctypes.byref(o), _dev_ptr(pivot), wptr, nbytes,
                                                 _np_ptr(evals), _np_ptr(resid), _dev_ptr(evecs), _np_ptr(stats),
                                                 _stream(stream)))
        out = dict(evals=evals, resid=resid, restarts=int(stats[0]), applies=int(stats[1]),
                   converged=bool(stats[2]), workspace_bytes=int(nbytes))
        if want_vectors:
            out["evecs"] = evecs
        return out

    def trlan_workspace_bytes(self, n_keep, n_thick, n_basis, mode="f64", max_restarts=50, tol=1e-10):
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        o = TrlanOpts(n_keep, n_thick, n_basis, max_restarts, m, 1, 0, float(tol))
        n = lib().fotci_trlan_workspace_bytes(self._h, ctypes.byref(o))
        if n < 0:
            _check(int(n))
        return int(n)

    def profile_start(self, max_calls):
        """Record HIP events around each apply_H kernel for up to max_calls calls."""
        _check(lib().fotci_profile_start(self._h, int(max_calls)))

    def profile_stop(self):
        """Mean milliseconds per kernel over the recorded calls: dict name -> ms."""
        ms = (ctypes.c_double * 4)()
        names = (ctypes.c_char_p * 4)()
        nk, nc = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fotci_profile_stop(self._h, ms, names, ctypes.byref(nk), ctypes.byref(nc)))
        return {names[k].decode(): ms[k] for k in range(nk.value)}, nc.value

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.fotci_free_ham(self._h)
            self._h = None


def decouple_tbme(two_j, pp=(), nn=(), pn=(), parity=None):
    """m-scheme (v_pp, v_nn, v_pn) from J-coupled elements (a, b, c, d, two_J, V) (host)."""
    tj = np.ascontiguousarray(two_j, dtype=np.int32)
    par = None if parity is None else np.ascontiguousarray(parity, dtype=np.int32)
    ns = int(np.sum(tj + 1))
    npairs = ns * (ns - 1) // 2

    def arr(elems):
        elems = list(elems)
        a = (Tbme * max(len(elems), 1))()
        for i, (x, y, z, w, tJ, v) in enumerate(elems):
            a[i] = Tbme(int(x), int(y), int(z), int(w), int(tJ), float(v))
        return len(elems), a

    n_pp, app = arr(pp)
    n_nn, ann = arr(nn)
    n_pn, apn = arr(pn)
    out = dict(v_pp=np.zeros((npairs, npairs)), v_nn=np.zeros((npairs, npairs)), v_pn=np.zeros((ns * ns, ns * ns)))
    _check(lib().fotci_decouple_tbme(len(tj), _np_ptr(tj), _np_ptr(par) if par is not None else None, n_pp, app,
                                     n_nn, ann, n_pn, apn, _np_ptr(out["v_pp"]), _np_ptr(out["v_nn"]),
                                     _np_ptr(out["v_pn"])))
    return out


def sym_eigh(a):
    """Host float64 dense symmetric eigensolver of the library (cyclic Jacobi)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    ev = np.zeros(n)
    vec = np.zeros((n, n))
    _check(lib().fotci_sym_eigh(n, _np_ptr(a), _np_ptr(ev), _np_ptr(vec)))
    return ev, vec


def tridiag_eigh(diag, offdiag):
    """Host float64 tridiagonal eigensolver of the library (for tests)."""
    d = np.ascontiguousarray(diag, dtype=np.float64)
    e = np.ascontiguousarray(offdiag, dtype=np.float64)
    n = len(d)
    ev = np.zeros(n)
    vec = np.zeros((n, n))
    _check(lib().fotci_tridiag_eigh(n, _np_ptr(d), _np_ptr(e), _np_ptr(ev), _np_ptr(vec)))
    return ev, vec
