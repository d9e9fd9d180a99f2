"""ctypes front-end for the oracle's C part (same definitions as hamiltonian.py).

Takes an ``oracle.basis.Basis`` and plain numpy arrays. Checks that V is
exactly symmetric before the row-wise matvec relies on it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from .basis import sector_table

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        l = ctypes.CDLL(path)
        p = ctypes.c_void_p
        l.orc_apply_h.argtypes = [ctypes.c_int, p, p, p, p, p, ctypes.c_int, p, ctypes.c_int, p,
                                  ctypes.c_int, p, p, p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        l.orc_apply_h.restype = ctypes.c_int
        l.orc_densities.argtypes = [ctypes.c_int, p, p, ctypes.c_int, p, ctypes.c_int, p,
                                    ctypes.c_int, p, p, p, p, ctypes.c_int]
        l.orc_densities.restype = ctypes.c_int
        l.orc_one_body_densities.argtypes = [ctypes.c_int, p, p, ctypes.c_int, p, ctypes.c_int, p,
                                             ctypes.c_int, p, p, p, p, p, ctypes.c_int]
        l.orc_one_body_densities.restype = ctypes.c_int
        _lib = l
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Prepared:
    """Basis arrays in the layout the C oracle reads, built once per basis."""

    def __init__(self, b):
        self.b = b
        self.ns = len(b.ms)
        self.sectab = np.ascontiguousarray(np.array(sector_table(b), dtype=np.int64).reshape(-1, 7))
        self.p_masks = np.ascontiguousarray(np.array(b.p_sds, dtype=np.uint32))
        self.n_masks = np.ascontiguousarray(np.array(b.n_sds, dtype=np.uint32))
        self.two_m = np.ascontiguousarray(np.array([m[2] for m in b.ms], dtype=np.int32))
        self.par = np.ascontiguousarray(np.array([m[3] for m in b.ms], dtype=np.int32))
        self.orbit = np.array([m[0] for m in b.ms])
        self.n_orb = int(self.orbit.max()) + 1


def _eps_m(prep, inter, sp):
    key = "eps_%s_mstate" % sp
    if key in inter:
        return np.ascontiguousarray(inter[key], dtype=np.float64)
    return np.ascontiguousarray(np.asarray(inter["eps_" + sp], dtype=np.float64)[prep.orbit])


def apply_h(prep, inter, x, rows=None, nthreads=0):
    """y[rows] of y = H x (all rows by default)."""
    for k in ("v_pp", "v_nn", "v_pn"):
        v = inter[k]
        if not np.array_equal(v, v.T):
            raise ValueError("%s is not exactly symmetric" % k)
    r0, r1 = (0, prep.b.dim) if rows is None else rows
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(r1 - r0)
    vpp = np.ascontiguousarray(inter["v_pp"], dtype=np.float64)
    vnn = np.ascontiguousarray(inter["v_nn"], dtype=np.float64)
    vpn = np.ascontiguousarray(inter["v_pn"], dtype=np.float64)
    ep, en = _eps_m(prep, inter, "p"), _eps_m(prep, inter, "n")
    rc = lib().orc_apply_h(prep.ns, _ptr(ep), _ptr(en), _ptr(vpp), _ptr(vnn), _ptr(vpn),
                           len(prep.sectab), _ptr(prep.sectab), len(prep.p_masks), _ptr(prep.p_masks),
                           len(prep.n_masks), _ptr(prep.n_masks), _ptr(x), _ptr(y),
                           r0, r1, nthreads)
    if rc != 0:
        raise AssertionError("H left the basis")
    return y


def densities(prep, g, x, nthreads=0):
    """Same dict as hamiltonian.densities, computed in C."""
    ns = prep.ns
    npairs = ns * (ns - 1) // 2
    nb = 2 * ns + 2 * npairs * npairs + ns ** 4
    bins = np.zeros(nb)
    g = np.ascontiguousarray(g, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rc = lib().orc_densities(ns, _ptr(prep.two_m), _ptr(prep.par), len(prep.sectab), _ptr(prep.sectab),
                             len(prep.p_masks), _ptr(prep.p_masks), len(prep.n_masks), _ptr(prep.n_masks),
                             _ptr(g), _ptr(x), _ptr(bins), nthreads)
    if rc != 0:
        raise AssertionError("operator left the basis")
    o = 0
    ep = bins[o:o + ns]; o += ns
    en = bins[o:o + ns]; o += ns
    vpp = bins[o:o + npairs * npairs].reshape(npairs, npairs); o += npairs * npairs
    vnn = bins[o:o + npairs * npairs].reshape(npairs, npairs); o += npairs * npairs
    vpn = bins[o:o + ns ** 4].reshape(ns * ns, ns * ns)
    d_eps_p = np.zeros(prep.n_orb)
    d_eps_n = np.zeros(prep.n_orb)
    np.add.at(d_eps_p, prep.orbit, ep)
    np.add.at(d_eps_n, prep.orbit, en)
    return dict(d_eps_p=d_eps_p, d_eps_n=d_eps_n, d_v_pp=vpp, d_v_nn=vnn, d_v_pn=vpn)


def one_body_densities(prep, g, x, nthreads=0):
    """Same (rho_p, rho_n) as hamiltonian.one_body_densities, computed in C."""
    ns = prep.ns
    rp = np.zeros(ns * ns)
    rn = np.zeros(ns * ns)
    g = np.ascontiguousarray(g, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rc = lib().orc_one_body_densities(ns, _ptr(prep.two_m), _ptr(prep.par), len(prep.sectab), _ptr(prep.sectab),
                                      len(prep.p_masks), _ptr(prep.p_masks), len(prep.n_masks),
                                      _ptr(prep.n_masks), _ptr(g), _ptr(x), _ptr(rp), _ptr(rn), nthreads)
    if rc != 0:
        raise AssertionError("operator left the basis")
    return rp.reshape(ns, ns), rn.reshape(ns, ns)


class Operator:
    """scipy LinearOperator-style wrapper (matvec only) for eigsh / Lanczos."""

    def __init__(self, prep, inter, nthreads=0):
        self.prep, self.inter, self.nthreads = prep, inter, nthreads
        self.shape = (prep.b.dim, prep.b.dim)
        self.dtype = np.dtype(np.float64)

    def matvec(self, x):
        return apply_h(self.prep, self.inter, np.ravel(x), nthreads=self.nthreads)
