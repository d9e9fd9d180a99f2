"""Float64 Lanczos with full reorthogonalisation (Ch. 7, "Standard Lanczos").

Steps per iteration i, in the chapter's order:
  (1) w = H v_i; (2) alpha_i = <v_i|w>; (3) w -= alpha_i v_i;
  (4) w -= beta_{i-1} v_{i-1}; then, since finite arithmetic lets earlier
  vectors creep back, w -= v_j <v_j|w> for every earlier vector j (the
  chapter computes alpha first and reorthogonalises afterwards; done twice
  here); (5) beta_i = ||w||; (6) v_{i+1} = w / beta_i.
The Ritz values are the eigenvalues of the tridiagonal matrix of alphas and
betas (numpy's symmetric eigensolver stands in for the LAPACK call).
"""
from __future__ import annotations

import numpy as np


def lanczos(matvec, v1, n_iter, n_keep):
    """Return (lowest n_keep Ritz values, Ritz vectors, alphas, betas)."""
    v = np.asarray(v1, dtype=np.float64)
    v = v / np.linalg.norm(v)
    dim = v.size
    k = min(n_iter, dim)
    V = np.zeros((k, dim))
    alphas, betas = [], []
    V[0] = v
    for i in range(k):
        w = matvec(V[i])
        a = float(np.dot(V[i], w))
        alphas.append(a)
        w = w - a * V[i]
        if i > 0:
            w = w - betas[-1] * V[i - 1]
        for _ in range(2):
            for j in range(i + 1):
                w = w - V[j] * np.dot(V[j], w)
        b = float(np.linalg.norm(w))
        if i == k - 1:
            break
        betas.append(b)
        if b == 0.0:
            k = i + 1
            break
        V[i + 1] = w / b
    T = np.diag(alphas[:k]) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    evals, evecs = np.linalg.eigh(T)
    n = min(n_keep, k)
    ritz = evecs[:, :n].T @ V[:k]
    return evals[:n], ritz, np.array(alphas[:k]), np.array(betas[:k - 1])
