"""The problem by its definition: max over all K^n assignments (Sec. 1,
eq. max_quad; factor form ||V^H z||^2 of Sec. 2.2).  Test infrastructure only;
feasible for K^n up to a few tens of millions."""
from __future__ import annotations

import numpy as np


def all_objectives(V: np.ndarray, K: int, chunk: int = 1 << 18):
    """Yield (labels block (m, n) int64, objective block (m,)) over all K^n
    labellings in lexicographic order of the base-K digits (row 0 most
    significant)."""
    V = np.asarray(V, dtype=np.complex128)
    n, r = V.shape
    total = K ** n
    Vc = V.conj()
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    powers = K ** np.arange(n - 1, -1, -1, dtype=np.int64)
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        digits = (idx[:, None] // powers[None, :]) % K          # (m, n)
        z = roots[digits]                                       # (m, n)
        s = z @ Vc                                              # (m, r): sum_i conj(V_ij) z_i
        f = np.sum(s.real ** 2 + s.imag ** 2, axis=1)
        yield digits, f


def brute_force(V: np.ndarray, K: int, rtol: float = 1e-12):
    """(OPT, first maximiser, number of maximisers within rtol of OPT)."""
    best, best_z = -np.inf, None
    blocks = []
    for digits, f in all_objectives(V, K):
        j = int(np.argmax(f))
        if f[j] > best:
            best, best_z = float(f[j]), digits[j].copy()
        blocks.append(f)
    allf = np.concatenate(blocks)
    ties = int(np.sum(allf >= best * (1.0 - rtol)))
    return best, best_z.astype(np.uint8), ties


def max_assignment_for_direction(V: np.ndarray, K: int, c: np.ndarray):
    """argmax over all K^n labellings of Re(z^H V c), the inner maximisation of
    the double-max form (Sec. 2.2); the decision rule must reproduce it."""
    V = np.asarray(V, dtype=np.complex128)
    w = V @ np.asarray(c, dtype=np.complex128)
    n = V.shape[0]
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    powers = K ** np.arange(n - 1, -1, -1, dtype=np.int64)
    idx = np.arange(K ** n, dtype=np.int64)
    digits = (idx[:, None] // powers[None, :]) % K
    val = np.real(np.conj(roots[digits]) @ w)
    j = int(np.argmax(val))
    return digits[j].astype(np.uint8), float(val[j])
