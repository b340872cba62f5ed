"""Exact rank-1 maximisation (Sec. 2.5, Alg. 1, Thm. rank1).  Test
infrastructure only.

For V = q (one column) the objective is |sum_i conj(q_i) z_i|^2.  Rotating the
direction c = e^{i phi} moves every w_i = q_i e^{i phi} by the same angle, and
the decision rule changes the label of coordinate i exactly when
arg(q_i) + phi crosses a boundary pi(2m+1)/K.  Inside the window
phi in (-pi/K, pi/K] (one label step; a wider window only rotates every
label, Lemma phase_equiv) each coordinate crosses exactly one boundary, at

    phi_i = (2 pi / K) (1/2 + floor(x_i) - x_i),   x_i = K arg(q_i) / (2 pi),

where its label advances from floor(x_i) to floor(x_i) + 1 (mod K).  The
window is thus cut into at most n + 1 cells on which the labels are constant,
and Thm. rank1 says the optimum is the labelling of one of them.

Two forms, each checked against the other and against brute force:

* ``rank1_cells_direct`` is the definition: one representative angle inside
  each cell, the decision rule applied there, the objective summed from the
  labels (O(n^2), small n only).
* ``rank1_cells`` takes the cells in boundary order and forms every cell's
  sum V^H z from the first cell's by cumulative sums of the label steps
  (O(n log n)); ``rank1_sweep`` returns its best cell (ties to the earlier
  cell).  These are the references of the GPU sweep.
"""
from __future__ import annotations

import numpy as np


def _roots(K: int) -> np.ndarray:
    return np.exp(2j * np.pi * np.arange(K) / K)


def boundary_points(q: np.ndarray, K: int):
    """(phi, start labels): phi_i as above, and floor(x_i) mod K, the label of
    coordinate i at the left end phi = -pi/K of the window."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    x = K * np.angle(q) / (2.0 * np.pi)
    fl = np.floor(x)
    phi = (2.0 * np.pi / K) * (0.5 + fl - x)
    return phi, np.mod(fl.astype(np.int64), K)


def rank1_cells(q: np.ndarray, K: int):
    """Objective of every cell, in boundary order: f[0] is the labelling at
    phi = -pi/K, f[l] the one after the l-th boundary point (equal points in
    coordinate order).  Returns (f, order, k0): the stable order of the
    boundary points and the start labels."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    phi, k0 = boundary_points(q, K)
    order = np.argsort(phi, kind="stable")
    w = _roots(K)
    # crossing the point of coordinate i changes z_i from w[k0] to w[k0 + 1]
    step = np.conj(q[order]) * (w[(k0[order] + 1) % K] - w[k0[order]])
    s = np.empty(q.size + 1, dtype=np.complex128)
    s[0] = np.sum(np.conj(q) * w[k0])
    s[1:] = s[0] + np.cumsum(step)
    return np.abs(s) ** 2, order, k0


def cell_labels(k0: np.ndarray, order: np.ndarray, l: int, K: int) -> np.ndarray:
    """Labels of cell l: the start labels with the first l coordinates of the
    boundary order advanced by one."""
    k = np.array(k0, dtype=np.int64)
    k[order[:l]] = (k[order[:l]] + 1) % K
    return k.astype(np.uint8)


def rank1_sweep(q: np.ndarray, K: int):
    """(OPT, labels): the best cell of rank1_cells, ties to the earlier cell."""
    f, order, k0 = rank1_cells(q, K)
    l = int(np.argmax(f))
    return float(f[l]), cell_labels(k0, order, l, K)


def rank1_cells_direct(q: np.ndarray, K: int):
    """The definition, cell by cell: for the sorted distinct boundary points
    p_1 < ... < p_m, one angle inside each cell (the midpoints, and for the
    cell that wraps around the window end the midpoint of (p_m, p_1 + 2pi/K),
    taken modulo the window); labels from the decision rule at
    w = q e^{i phi}; objective |sum conj(q_i) z_i|^2 summed directly.
    Returns (f, labels) with one row per cell."""
    q = np.asarray(q, dtype=np.complex128).ravel()
    phi, _ = boundary_points(q, K)
    p = np.unique(phi)
    width = 2.0 * np.pi / K
    mids = list(0.5 * (p[:-1] + p[1:])) + [0.5 * (p[-1] + p[0] + width)]
    w = _roots(K)
    fs, zs = [], []
    for a in mids:
        wi = q * np.exp(1j * a)
        k = np.mod(np.floor(K * np.angle(wi) / (2.0 * np.pi) + 0.5).astype(np.int64), K)
        k[wi == 0] = 0
        fs.append(abs(np.sum(np.conj(q) * w[k])) ** 2)
        zs.append(k.astype(np.uint8))
    return np.array(fs), np.array(zs)
