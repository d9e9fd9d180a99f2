"""Float64 Lanczos with full reorthogonalisation (Ch. 7, "Standard Lanczos"),
and block Lanczos (Ch. "Block Lanczos"). Test infrastructure: plain dense
numpy, float64.

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


def restart_index(fill, col, n_block, dim):
    """Basis vector e_k that replaces column `col` of a new block at the
    fill-th restart of a run: k = ((fill * n_block + col) * 2654435761) mod dim
    (a multiplicative hash, so successive restarts spread over the basis)."""
    return ((fill * n_block + col) * 2654435761) % dim


def block_lanczos(matmul, V1, n_iter, n_keep, tol=1e-7, weak=1e-4, floor=1e-12):
    """Block Lanczos (Ch. "Block Lanczos"), float64, dense blocks.

    matmul(X) = H X for X of shape (dim, n_block). Steps per block n:
      W = H V_n; W -= V_j (V_j^T W) for the earlier blocks j < n;
      A_n = V_n^T W; W' = W - V_n A_n (then once more against every block,
      which rounding makes necessary); the overlap O = W'^T W' = U L U^T gives
      B_n = L^{1/2} U^T and V_{n+1} = W' U L^{-1/2}.
    A column u whose overlap eigenvalue is too small (sqrt(L_u) <= tol ||T||;
    eigenvalues of a Gram matrix resolve sqrt(L) only to about sqrt(eps)
    times the block's norm, so exactly dependent directions show up near
    1e-8) is replaced by a new vector, as the chapter prescribes for a nearly
    singular overlap: the basis vector e_k of restart_index, with row u of
    B_n zero. After a replacement, or when the weakest kept column has
    sqrt(L_u) < weak ||T|| (its division by sqrt(L_u) magnifies rounding), the
    new block is orthogonalised against the basis again (twice) and
    orthonormalised once more by its own overlap, B_n taking that factor too.
    The iteration stops when every column is dependent or the refreshed block
    of unit columns has an overlap eigenvalue <= floor (a new vector inside
    the span). T is block tridiagonal with A_n on the
    diagonal, B_n below and B_n^T above.

    Returns (lowest n_keep eigenvalues of T, T, number of blocks, the basis
    [V_0 V_1 ...] as a dim x (blocks * n_block) matrix)."""
    V1 = np.array(V1, dtype=np.float64)
    dim, nb = V1.shape
    lam, U = np.linalg.eigh(V1.T @ V1)
    if not lam[0] > 1e-24 * lam[-1]:
        raise ValueError("pivot block columns are linearly dependent")
    blocks = [V1 @ U / np.sqrt(lam)]
    As, Bs = [], []
    fills = 0
    tnorm = 0.0
    for n in range(n_iter):
        V = blocks[n]
        W = matmul(V)
        for j in range(n):
            W = W - blocks[j] @ (blocks[j].T @ W)
        A = V.T @ W
        A = 0.5 * (A + A.T)
        W = W - V @ A
        for j in range(n + 1):
            W = W - blocks[j] @ (blocks[j].T @ W)
        As.append(A)
        if n == n_iter - 1:
            break
        side = np.linalg.norm(Bs[-1]) if Bs else 0.0
        tnorm = max(tnorm, np.linalg.norm(A) + side)
        lam, U = np.linalg.eigh(W.T @ W)
        root = np.sqrt(np.maximum(lam, 0.0))
        bad = root <= tol * tnorm
        if bad.all():
            break
        Y = np.zeros((dim, nb))
        B = np.zeros((nb, nb))
        for u in range(nb):
            if not bad[u]:
                Y[:, u] = W @ U[:, u] / root[u]
                B[u] = root[u] * U[:, u]
        for u in np.nonzero(bad)[0]:
            Y[restart_index(fills, int(u), nb, dim), u] = 1.0
        if bad.any():
            fills += 1
        if bad.any() or root[~bad].min() < weak * tnorm:
            for _ in range(2):
                for Q in blocks:
                    Y = Y - Q @ (Q.T @ Y)
        lam2, U2 = np.linalg.eigh(Y.T @ Y)
        if not lam2[0] > floor:
            break
        Bs.append((np.sqrt(lam2)[:, None] * U2.T) @ B)
        blocks.append(Y @ U2 / np.sqrt(lam2))
    k = len(As)
    m = k * nb
    T = np.zeros((m, m))
    for j in range(k):
        T[j * nb:(j + 1) * nb, j * nb:(j + 1) * nb] = As[j]
    for j in range(k - 1):
        T[(j + 1) * nb:(j + 2) * nb, j * nb:(j + 1) * nb] = Bs[j]
        T[j * nb:(j + 1) * nb, (j + 1) * nb:(j + 2) * nb] = Bs[j].T
    ev = np.linalg.eigvalsh(T)
    return ev[:min(n_keep, m)], T, k, np.hstack(blocks[:k])
