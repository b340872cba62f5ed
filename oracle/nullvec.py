"""Null-vector randomized sampler: the randomized form of Alg. 2 compared with
uniform sphere sampling in Sec. 5 ("Randomized Rounding", Table samplers).
Test infrastructure only; FP64, plain loops over the draws.

Draw s picks 2r-1 rows of the augmented matrix (eq. tildeV) at random and,
when they are linearly independent, scores the vertex they cut out exactly
as Alg. 2 scores an enumerated index set (both signs of the null vector,
every label combination the vertex leaves open).  Draws whose rows repeat,
hold three rows of one coordinate or fail the rank test are infeasible.

Row generator (the paper gives none; both implementations follow this
definition): with M = 2r-1 and N = n B_K, word t of block b is word t of
Philox4x32-10 with key (seed lo, seed hi) and counter (s lo, s hi,
0x4E554C4C, b); row j is (2^32 w[2j+1] + w[2j]) mod N; the set is the sorted
rows.
"""
from __future__ import annotations

import numpy as np

from . import exact, philox4x32_10

NULLVEC_STREAM = 0x4E554C4C


def draw_set(seed: int, s: int, N: int, M: int):
    """(sorted rows, valid) of draw s."""
    words = []
    for b in range((2 * M + 3) // 4):
        words.extend(int(x) for x in philox4x32_10(
            [s & 0xFFFFFFFF, (s >> 32) & 0xFFFFFFFF, NULLVEC_STREAM, b],
            [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]))
    rows = sorted(((words[2 * j + 1] << 32) | words[2 * j]) % N for j in range(M))
    return rows


def is_valid(rows, B: int) -> bool:
    if any(rows[t] == rows[t + 1] for t in range(len(rows) - 1)):
        return False
    g = [x // B for x in rows]
    return not any(g[t] == g[t + 2] for t in range(len(g) - 2))


def nullvec_sampler(V: np.ndarray, K: int, S: int, seed: int, score: bool = True):
    """Best FP64 objective over S draws (ties to the earlier draw), its
    labels and the draw statistics; with score=False only the statistics of
    validity and rank."""
    V = np.asarray(V, dtype=np.complex128)
    n, r = V.shape
    B = exact.boundary_count(K)
    N, M = n * B, 2 * r - 1
    stats = {"index_sets": 0, "rank_deficient": 0, "candidates": 0}
    best, best_z, best_s = -np.inf, None, -1
    A = exact.tilde_rows(V, K) if not score else None
    for s in range(S):
        rows = draw_set(seed, s, N, M)
        if not is_valid(rows, B):
            continue
        stats["index_sets"] += 1
        if not score:
            sv = np.linalg.svd(A[rows], compute_uv=False)
            stats["rank_deficient"] += int(not sv[-1] / sv[0] > 1e-10)
            continue
        for Z in exact.set_candidates(V, K, r, [rows], stats):
            f = exact.objective_many(V, K, Z)
            j = int(np.argmax(f))
            if f[j] > best:
                best, best_z, best_s = float(f[j]), Z[j].copy(), s
    return {"opt": best, "z": None if best_z is None else best_z.astype(np.uint8), "draw": best_s,
            "valid": stats["index_sets"], "rank_deficient": stats["rank_deficient"],
            "candidates": stats["candidates"]}
