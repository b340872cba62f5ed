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


# ------------------------------------------------ rows of W, vectorised
# The same definition as w_entry, evaluated for a whole row with Philox in
# numpy (64-bit products of 32-bit words), so that rows of Q = U U^H + sigma W
# can be formed at n ~ 10^5 - 10^6 on the host.

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)


def philox_np(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32-10 on arrays of counters (uint32), one key."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint32).copy() for c in (c0, c1, c2, c3))
    ka, kb = np.uint32(k0), np.uint32(k1)
    mask = np.uint64(0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            ka = np.uint32((int(ka) + int(_W0)) & 0xFFFFFFFF)
            kb = np.uint32((int(kb) + int(_W1)) & 0xFFFFFFFF)
        p0 = _M0 * x0.astype(np.uint64)
        p1 = _M1 * x2.astype(np.uint64)
        hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & mask).astype(np.uint32)
        hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & mask).astype(np.uint32)
        x0, x1, x2, x3 = hi1 ^ x1 ^ ka, lo1, hi0 ^ x3 ^ kb, lo0
    return x0, x1, x2, x3


def w_row(seed: int, i: int, n: int) -> np.ndarray:
    """Row i of W (n entries) by the definition of w_entry."""
    j = np.arange(n, dtype=np.int64)
    lo = np.minimum(i, j)               # the generating pair is (min, max)
    hi = np.maximum(i, j)
    o = philox_np(lo.astype(np.uint32), (hi >> 1).astype(np.uint32), np.full(n, W_STREAM, np.uint32),
                  np.zeros(n, np.uint32), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    odd = (hi & 1).astype(bool)
    w0 = np.where(odd, o[2], o[0])
    w1 = np.where(odd, o[3], o[1])
    u0 = ((w0 >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    u1 = ((w1 >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    rad = np.sqrt(-np.log(u0))
    w = rad * np.exp(2j * np.pi * u1)
    w = np.where(j < i, np.conj(w), w)          # W_ij = conj(W_ji) below the diagonal
    w[i] = np.sqrt(-2.0 * np.log(u0[i])) * np.cos(2.0 * np.pi * u1[i])
    return w


def phase_sync_rows_times(U: np.ndarray, sigma: float, seed: int, rows, X: np.ndarray) -> np.ndarray:
    """(Q X)[rows, :] for Q = U U^H + sigma W, one row of W at a time (FP64)."""
    U = np.asarray(U, dtype=np.complex128)
    X = np.asarray(X, dtype=np.complex128)
    UX = U.conj().T @ X
    out = np.empty((len(rows), X.shape[1]), dtype=np.complex128)
    for t, i in enumerate(rows):
        out[t] = U[i] @ UX + sigma * (w_row(seed, int(i), U.shape[0]) @ X)
    return out
