"""Full objective on the graph and greedy local refinement: FP64 / integer
reference.  Test infrastructure only; plain loops over edges and vertices.

The sampled and exact paths maximise the low-rank surrogate ||V^H z||^2.  The
step after them scores the returned labels on the original sparse matrix and
improves them by local search (appendix "Rank-1 at Scale": incremental
scoring, eq. incremental; hybrid warm start).  For a graph with weights w_ij
and Q = L = D - A (the Laplacian used for Max-K-Cut, Sec. 5):

  objective   z^H L z = sum over undirected edges {i, j} of w_ij |z_i - z_j|^2
  cut weight  sum over undirected edges {i, j} with k_i != k_j of w_ij
              (for K = 3, |1 - omega|^2 = 3, so z^H L z = 3 cut)
  gain        moving vertex i from label a to label b changes z^H L z by
              sum_j w_ij (|omega^b - omega^k_j|^2 - |omega^a - omega^k_j|^2),
              the value of eq. incremental for this Q

Local search rule (one round): every vertex takes its best label b != a
(largest gain, ties to the lowest b) and is a candidate when that gain is
positive; a candidate moves when its (gain, -index) is larger than that of
every neighbouring candidate.  Moving vertices are pairwise non-adjacent, so
the round's change of the objective is the sum of their gains; rounds repeat
until no vertex has a positive gain, which is a 1-flip local optimum.

Graphs are given as undirected edge lists (i, j, w) with i != j, each edge
once.
"""
from __future__ import annotations

import math

import numpy as np


def root(K: int, k: int) -> complex:
    return complex(math.cos(2.0 * math.pi * k / K), math.sin(2.0 * math.pi * k / K))


def sqdist_table(K: int) -> np.ndarray:
    """|omega^a - omega^b|^2 for all label pairs, by the definition."""
    T = np.empty((K, K))
    for a in range(K):
        for b in range(K):
            T[a, b] = abs(root(K, a) - root(K, b)) ** 2
    if K in (2, 3, 4):
        T = np.round(T)      # the values are the integers 0..4 exactly
    return T


def quadratic_form(edges, K: int, z) -> float:
    """z^H L z as a sum over undirected edges."""
    T = sqdist_table(K)
    i, j, w = edges
    return float(np.sum(np.asarray(w, dtype=np.float64) * T[np.asarray(z)[i], np.asarray(z)[j]]))


def cut_weight(edges, z) -> float:
    i, j, w = edges
    z = np.asarray(z)
    return float(np.sum(np.asarray(w, dtype=np.float64)[z[i] != z[j]]))


def adjacency(n: int, edges):
    """Neighbour lists (both directions) with weights."""
    nb = [[] for _ in range(n)]
    for a, b, w in zip(*edges):
        nb[int(a)].append((int(b), float(w)))
        nb[int(b)].append((int(a), float(w)))
    return nb


def gains(n: int, nb, K: int, z):
    """Best move of every vertex: (gain, target label), gain from the
    definition (sum over the neighbours of the change of |z_i - z_j|^2)."""
    T = sqdist_table(K)
    g = np.zeros(n)
    tgt = np.array(z, dtype=np.int64)
    for v in range(n):
        a = int(z[v])
        best, bl = -math.inf, -1
        for b in range(K):
            if b == a:
                continue
            d = 0.0
            for u, w in nb[v]:
                d += w * (T[b, z[u]] - T[a, z[u]])
            if d > best:
                best, bl = d, b
        if bl >= 0:
            g[v], tgt[v] = best, bl
    return g, tgt


def greedy_round(n: int, nb, K: int, z):
    """One round of the rule; returns (new labels, moved vertex list, gains)."""
    g, tgt = gains(n, nb, K, z)
    moved = []
    for v in range(n):
        if g[v] <= 0.0:
            continue
        wins = True
        for u, _ in nb[v]:
            if g[u] > 0.0 and (g[u] > g[v] or (g[u] == g[v] and u < v)):
                wins = False
                break
        if wins:
            moved.append(v)
    z2 = np.array(z, dtype=np.int64)
    for v in moved:
        z2[v] = tgt[v]
    return z2, moved, g


def greedy(n: int, edges, K: int, z, max_rounds: int = 10_000):
    """Rounds until no vertex has a positive gain.  Returns (labels, rounds
    that moved at least one vertex, total moves)."""
    nb = adjacency(n, edges)
    z = np.array(z, dtype=np.int64)
    rounds = moves = 0
    while rounds < max_rounds:
        z2, moved, _ = greedy_round(n, nb, K, z)
        if not moved:
            break
        z = z2
        rounds += 1
        moves += len(moved)
    return z, rounds, moves


def is_local_optimum(n: int, edges, K: int, z, tol: float = 0.0) -> bool:
    g, _ = gains(n, adjacency(n, edges), K, z)
    return bool(np.all(g <= tol))


def gains_vectorized(n: int, edges, K: int, z):
    """The same best moves as `gains`, with numpy scatter-adds over the edge
    list (for graphs too large for the loops): D[b, v] = sum over the
    neighbours u of w (T[b, z_u] - T[z_v, z_u])."""
    T = sqdist_table(K)
    i, j, w = (np.asarray(a) for a in edges)
    w = w.astype(np.float64)
    z = np.asarray(z, dtype=np.int64)
    src = np.concatenate([i, j])
    dst = np.concatenate([j, i])
    ww = np.concatenate([w, w])
    D = np.zeros((K, n))
    for b in range(K):
        np.add.at(D[b], src, ww * (T[b, z[dst]] - T[z[src], z[dst]]))
    D[z, np.arange(n)] = -np.inf            # staying is not a move
    tgt = np.argmax(D, axis=0)               # ties -> lowest label
    return D[tgt, np.arange(n)], tgt
