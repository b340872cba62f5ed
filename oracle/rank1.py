"""Alg. 1: exact rank-1 sweep (Sec. 2.5, Thm. rank1).  Test infrastructure only.

For Q = q q^H the optimum is reached in one of the n+1 cells of the sweep of
the auxiliary angle phi over (-pi/K, pi/K]: start from k = floor(K theta/2pi)
(the assignment at phi = -pi/K) and advance one coordinate by one label at
each boundary point phi_i = (2pi/K)(1/2 + floor(K theta_i/2pi) - K theta_i/2pi),
taken in sorted order.
"""
from __future__ import annotations

import numpy as np


def rank1_sweep(q: np.ndarray, K: int):
    """(OPT, labels) of max |z^H q|^2 over z in A_K^n, by Alg. 1."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    n = q.size
    theta = np.angle(q)                                    # (-pi, pi]
    x = K * theta / (2.0 * np.pi)
    phi = (2.0 * np.pi / K) * (0.5 + np.floor(x) - x)     # boundary points
    order = np.argsort(phi, kind="stable")
    k = np.mod(np.floor(x).astype(np.int64), K)
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    s = np.sum(np.conj(q) * roots[k])                      # z^H q conjugated: sum conj(q_i) z_i
    best, best_k = abs(s) ** 2, k.copy()
    for i in order:
        new = (k[i] + 1) % K
        s += np.conj(q[i]) * (roots[new] - roots[k[i]])
        k[i] = new
        f = abs(s) ** 2
        if f > best:
            best, best_k = f, k.copy()
    return float(best), best_k.astype(np.uint8)


def rank1_cells(q: np.ndarray, K: int):
    """Objective of every cell of the sweep, in sweep order: f[0] is the
    assignment at phi = -pi/K, f[l] the one after the l-th boundary point.
    Returns (f, order, k0) with `order` the stable argsort of the boundary
    points and k0 the starting labels."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    theta = np.angle(q)
    x = K * theta / (2.0 * np.pi)
    phi = (2.0 * np.pi / K) * (0.5 + np.floor(x) - x)
    order = np.argsort(phi, kind="stable")
    k0 = np.mod(np.floor(x).astype(np.int64), K)
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    k = k0.copy()
    s = np.sum(np.conj(q) * roots[k])
    f = np.empty(q.size + 1)
    f[0] = abs(s) ** 2
    for l, i in enumerate(order, start=1):
        new = (k[i] + 1) % K
        s += np.conj(q[i]) * (roots[new] - roots[k[i]])
        k[i] = new
        f[l] = abs(s) ** 2
    return f, order, k0
