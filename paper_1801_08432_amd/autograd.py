"""torch.autograd wrappers over the library's apply_H and its adjoint.

ApplyH      y = H(theta) x; backward gives dL/dx = H g (H is symmetric) and
            dL/dtheta[label] = <g| O_label |x>, the label-wise transition
            densities computed by fotci_apply_H_vjp.
LanczosEig  the lowest eigenvalues E_k(theta); backward gives
            dL/dtheta = sum_k dL/dE_k <psi_k| O_label |psi_k> (Hellmann-Feynman,
            valid for non-degenerate, converged states), the m-scheme analogue
            of the paper's diagonal two-body densities (Ch. 5, "Two-body
            densities": the energy of a state under an interaction whose
            elements are all zero except one, which is 1).

theta is the interaction as five float64 tensors (eps_p, eps_n, v_pp, v_nn,
v_pn) in the layout of fotci_set_interaction. The gradient of an array entry
is unsymmetrised: entries (r, c) and (c, r) are separate; parametrise V
symmetrically (e.g. V = (A + A^T)/2) to obtain gradients of independent
elements. The forward pass loads theta into the Hamiltonian (validation and
a small host-to-device copy), so theta must be exactly symmetric and zero
where Jz or parity would change.
"""
from __future__ import annotations

import torch

from . import fotci

KEYS = ("eps_p", "eps_n", "v_pp", "v_nn", "v_pn")


def _load(ham, theta):
    if theta is None:
        return
    ham.set_values({k: t.detach().to("cpu", torch.float64).numpy() for k, t in zip(KEYS, theta)})


class ApplyH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, ham, mode, *theta):
        _load(ham, theta if theta else None)
        y = ham.apply(x.contiguous(), mode=mode)
        ctx.ham = ham
        ctx.has_theta = bool(theta)
        ctx.theta_dev = [(t.device, t.dtype) for t in theta]
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        ham = ctx.ham
        xd = x.detach().to(torch.float64).contiguous()
        gd = g.detach().to(torch.float64).contiguous()
        dx, grads = ham.vjp(xd, gd, want_dx=ctx.needs_input_grad[0])
        dx = dx.to(x.dtype) if dx is not None else None
        out = [dx, None, None]
        if ctx.has_theta:
            out += [grads[k].to(dev, dt) for k, (dev, dt) in zip(KEYS, ctx.theta_dev)]
        return tuple(out)


def apply_h(ham, x, theta=None, mode="f64"):
    """y = H x with autograd through x and (optionally) theta."""
    return ApplyH.apply(x, ham, mode, *(theta or ()))


class LanczosEig(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pivot, ham, n_keep, n_iter, mode, *theta):
        _load(ham, theta if theta else None)
        r = ham.lanczos_lowest(pivot, n_keep, n_iter, mode=mode, refine=True, want_vectors=True)
        ctx.ham = ham
        ctx.theta_dev = [(t.device, t.dtype) for t in theta]
        ctx.vecs = r["evecs"]
        ctx.resid = r["resid"]
        return torch.as_tensor(r["evals"], dtype=torch.float64, device=pivot.device)

    @staticmethod
    def backward(ctx, gE):
        ham = ctx.ham
        gE = gE.detach().to("cpu", torch.float64)
        total = None
        for k in range(ctx.vecs.shape[0]):
            if float(gE[k]) == 0.0:
                continue
            psi = ctx.vecs[k].contiguous()
            _, grads = ham.vjp(psi, psi, want_dx=False)
            part = [float(gE[k]) * grads[key] for key in KEYS]
            total = part if total is None else [a + b for a, b in zip(total, part)]
        if total is None:
            return (None, None, None, None, None) + (None,) * len(ctx.theta_dev)
        total = [t.to(dev, dt) for t, (dev, dt) in zip(total, ctx.theta_dev)]
        return (None, None, None, None, None) + tuple(total)


def lowest_eigenvalues(ham, pivot, n_keep, n_iter, theta, mode="f64"):
    """E_1..E_n_keep(theta) with Hellmann-Feynman gradients w.r.t. theta."""
    return LanczosEig.apply(pivot, ham, n_keep, n_iter, mode, *theta)
