"""Spectral truncation (the step before the path): the r largest eigenpairs of
the matrix that the low-rank factor V = U diag(sqrt(lambda)) approximates.
Test infrastructure only; FP64, dense for small n.

Two matrices:
  Laplacian    L = D - A of a weighted graph (Max-K-Cut, Sec. 5)
  phase sync   Q = U U^H + sigma W, U (n x p) with unit-modulus entries and W
               Hermitian Gaussian (off-diagonal N_C(0,1): real and imaginary
               parts N(0, 1/2); diagonal N(0,1)) as in the phase
               synchronisation workload

W is regenerated from a counter-based definition (the paper fixes none; the
library's matrix-free operator evaluates the same definition): for i <= j,
Philox4x32-10 with key (seed lo, seed hi) and counter (i, j >> 1, 0x57484D41, 0)
gives four words (w0, w1, w2, w3); column j takes (w0, w1) when j is even and
(w2, w3) when j is odd, so one call serves the columns 2q and 2q + 1 of row i.
The two words give uniforms u = ((w >> 9) + 1/2) 2^-23 and
  W_ij = sqrt(-log u0) (cos 2 pi u1 + i sin 2 pi u1)   (i < j)
  W_ii = sqrt(-2 log u0) cos 2 pi u1,                  W_ji = conj(W_ij).

Factor convention: eigenvalues in descending order; each eigenvector is
multiplied by the unit phase that makes its largest-modulus entry real and
positive (the lowest index among equal moduli); V = U diag(sqrt(max(l, 0))).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox4x32_10, uniform

W_STREAM = 0x57484D41


def w_entry(seed: int, i: int, j: int) -> complex:
    """W_ij by the definition above, FP64."""
    a, b = (i, j) if i <= j else (j, i)
    o = philox4x32_10([a & 0xFFFFFFFF, (b >> 1) & 0xFFFFFFFF, W_STREAM, 0],
                      [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    h = 2 * (b & 1)
    u0, u1 = uniform(int(o[h])), uniform(int(o[h + 1]))
    if a == b:
        return complex(math.sqrt(-2.0 * math.log(u0)) * math.cos(2.0 * math.pi * u1), 0.0)
    rad = math.sqrt(-math.log(u0))
    w = complex(rad * math.cos(2.0 * math.pi * u1), rad * math.sin(2.0 * math.pi * u1))
    return w if i <= j else w.conjugate()


def w_matrix(n: int, seed: int) -> np.ndarray:
    W = np.empty((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(i, n):
            W[i, j] = w_entry(seed, i, j)
            W[j, i] = W[i, j].conjugate()
    return W


def phase_sync_matrix(U: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    U = np.asarray(U, dtype=np.complex128)
    return U @ U.conj().T + sigma * w_matrix(U.shape[0], seed)


def laplacian_dense(n: int, edges) -> np.ndarray:
    i, j, w = edges
    L = np.zeros((n, n))
    for a, b, x in zip(i, j, w):
        L[a, b] -= x
        L[b, a] -= x
        L[a, a] += x
        L[b, b] += x
    return L


def fix_phase(u: np.ndarray) -> np.ndarray:
    k = int(np.argmax(np.abs(u)))
    return u * (np.conj(u[k]) / abs(u[k]))


def top_factor(M: np.ndarray, r: int):
    """(eigenvalues desc, factor V) of a dense Hermitian M (numpy eigh)."""
    lam, U = np.linalg.eigh(M)
    lam, U = lam[::-1][:r], U[:, ::-1][:, :r]
    U = np.stack([fix_phase(U[:, k].astype(np.complex128)) for k in range(r)], axis=1)
    return lam, U * np.sqrt(np.maximum(lam, 0.0))[None, :]
