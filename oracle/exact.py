"""Alg. 2: exact rank-r solver by enumerating arrangement vertices (Sec. 3).
Test infrastructure only; plain, slow, FP64.

Steps, in the paper's order and notation:

1. Augmented matrix (eq. tildeV).  With rotation factors
   rho_m = exp(-i pi (2m+1)/K), m < B_K (Def. BK: B_K = K/2 for even K, K for
   odd K), the row of coordinate i and boundary m is
   a_{i,m} = [Im(rho_m V_i), Re(rho_m V_i)] in R^{2r}, so that
   a_{i,m} . [Re c; Im c] = Im(rho_m V_i c): the row vanishes exactly when
   V_i c lies on the boundary line at angle pi(2m+1)/K (Lemma antipodal,
   Cor. two_implies_all).  Rows are ordered group-major, j = i B_K + m, so
   the coordinate group of row j is floor(j / B_K).
2. Every index set I of 2r-1 rows with at most two rows per coordinate group
   (the valid sets of Alg. 2; Lemma rank_deficiency), in lexicographic order.
3. Rank test and unit null vector of the (2r-1) x 2r block by SVD:
   rank 2r-1 when sigma_min / sigma_max > 1e-10.
4. For both signs of the null vector: c = c~_{1:r} + i c~_{r+1:2r}, w = V c.
5. Rows outside I take the decision rule (eq. decision_rule).
6. A coordinate with one row (i, m) in I has V_i c on the line of boundary m:
   on the ray pi(2m+1)/K it borders labels m and m+1; on the opposite ray it
   is, for odd K, a root direction (decision rule), and for even K the
   boundary between labels m+K/2 and m+K/2+1.
7. A coordinate with two rows in I has V_i c = 0 (Cor. two_implies_all): all
   K labels are tried.  This enumerates a superset of the (B_K-1)^p adjacent
   cells of Lemma adjacent_cells and replaces the fixed-angle construction of
   the ambiguity-resolution subroutine (Alg. resolve, appendix to Sec. 3),
   whose embedding matrix is not dimensionally consistent as printed.
8. Every combination is scored in FP64 with the full factor; the maximum is
   kept, ties going to the first candidate in enumeration order.
9. For r > 1 the same enumeration runs on the leading columns V_{:,1:d},
   d = r-1, ..., 1 (the recursion of Alg. 2), its directions padded with
   zeros and scored with the full factor.
"""
from __future__ import annotations

import itertools

import numpy as np


def boundary_count(K: int) -> int:
    """B_K of Def. BK."""
    return K // 2 if K % 2 == 0 else K


def tilde_rows(V: np.ndarray, K: int) -> np.ndarray:
    """(n B_K, 2r) augmented real matrix, group-major."""
    V = np.asarray(V, dtype=np.complex128)
    n, r = V.shape
    B = boundary_count(K)
    rho = np.exp(-1j * np.pi * (2 * np.arange(B) + 1) / K)
    RV = rho[None, :, None] * V[:, None, :]                    # (n, B, r)
    return np.concatenate([RV.imag, RV.real], axis=2).reshape(n * B, 2 * r)


def decision_labels(w: np.ndarray, K: int) -> np.ndarray:
    """eq. decision_rule: k = floor(K arg(w)/2pi + 1/2) mod K; w = 0 -> 0."""
    w = np.asarray(w, dtype=np.complex128)
    k = np.mod(np.floor(K * np.angle(w) / (2.0 * np.pi) + 0.5).astype(np.int64), K)
    k[w == 0] = 0
    return k


def objective_many(V: np.ndarray, K: int, Z: np.ndarray) -> np.ndarray:
    """||V^H z||^2 for each row of the label matrix Z (m, n)."""
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    s = roots[Z] @ np.conj(V)                                  # (m, r)
    return np.sum(s.real ** 2 + s.imag ** 2, axis=1)


def _single_options(wi: complex, m: int, K: int):
    rho = np.exp(-1j * np.pi * (2 * m + 1) / K)
    if (rho * wi).real > 0:
        return [m % K, (m + 1) % K]
    if K % 2 == 1:
        return [int(decision_labels(np.array([wi]), K)[0])]
    return [(m + K // 2) % K, (m + K // 2 + 1) % K]


def _near_boundary_rows(V, w, K, c, skip):
    """Rows outside I lying on a boundary line to within 1e-12 of their scale
    (only for a factor that violates general position)."""
    B = boundary_count(K)
    scale = np.abs(V) @ np.abs(c)
    out = []
    for i in np.nonzero(scale > 0)[0]:
        if i in skip:
            continue
        for m in range(B):
            rho = np.exp(-1j * np.pi * (2 * m + 1) / K)
            if abs((rho * w[i]).imag) <= 1e-12 * scale[i] and abs(w[i]) > 1e-12 * scale[i]:
                out.append((int(i), m))
                break
    return out


def level_candidates(V: np.ndarray, K: int, d: int, stats: dict):
    """Yield (Z block of candidate labellings) from the vertices of the
    arrangement built on the leading d columns of V, in enumeration order."""
    n = np.asarray(V).shape[0]
    B = boundary_count(K)
    size = 2 * d - 1
    sets = []
    for I in itertools.combinations(range(n * B), size):
        g = [j // B for j in I]
        if any(g[t] == g[t + 1] == g[t + 2] for t in range(size - 2)):
            continue
        sets.append(I)
    stats["index_sets"] = stats.get("index_sets", 0) + len(sets)
    yield from set_candidates(V, K, d, sets, stats)


def set_candidates(V: np.ndarray, K: int, d: int, sets, stats: dict):
    """Yield, for each valid index set I (sorted rows of the augmented matrix
    of the leading d columns, at most two per coordinate) in the given order,
    the candidate labellings of its vertex: rank test and null vector by SVD,
    both signs, the decision rule outside I and the open labels of the
    coordinates in I."""
    V = np.asarray(V, dtype=np.complex128)
    Vd = V[:, :d]
    B = boundary_count(K)
    A = tilde_rows(Vd, K)
    if len(sets) == 0:
        return
    sets = np.asarray(sets, dtype=np.int64)
    _, sv, Vt = np.linalg.svd(A[sets], full_matrices=True)     # (m, size), (m, 2d, 2d)
    ok = sv[:, -1] / sv[:, 0] > 1e-10
    stats["rank_deficient"] = stats.get("rank_deficient", 0) + int(np.sum(~ok))
    for t in np.nonzero(ok)[0]:
        I = sets[t]
        v = Vt[t, -1, :]
        groups = {}
        for j in I:
            groups.setdefault(int(j // B), []).append(int(j % B))
        for sign in (1.0, -1.0):
            c = sign * (v[:d] + 1j * v[d:])
            w = Vd @ c
            k = decision_labels(w, K)
            rows, opts = [], []
            for i, ms in groups.items():
                rows.append(i)
                opts.append(list(range(K)) if len(ms) >= 2 else _single_options(w[i], ms[0], K))
            for i, m in _near_boundary_rows(Vd, w, K, c, groups):
                rows.append(i)
                opts.append(_single_options(w[i], m, K))
            combos = np.array(list(itertools.product(*opts)), dtype=np.int64)
            Z = np.repeat(k[None, :], combos.shape[0], axis=0)
            Z[:, rows] = combos
            stats["candidates"] = stats.get("candidates", 0) + Z.shape[0]
            yield Z


def solve_exact(V: np.ndarray, K: int, recurse: bool = True, collect_distinct: bool = False):
    """Alg. 2 (with the recursion over leading columns).  Returns a dict with
    'opt', 'z' (uint8 labels), and enumeration statistics."""
    V = np.asarray(V, dtype=np.complex128)
    n, r = V.shape
    stats: dict = {}
    best, best_z = -np.inf, None
    distinct = set() if collect_distinct else None
    for d in (range(r, 0, -1) if recurse else [r]):
        for Z in level_candidates(V, K, d, stats):
            f = objective_many(V, K, Z)
            j = int(np.argmax(f))
            if f[j] > best:
                best, best_z = float(f[j]), Z[j].copy()
            if distinct is not None:
                distinct.update(map(bytes, Z.astype(np.uint8)))
    out = {"opt": best, "z": None if best_z is None else best_z.astype(np.uint8), **stats}
    if distinct is not None:
        out["distinct"] = len(distinct)
        out["distinct_set"] = distinct
    return out


def card_formula(n: int, r: int, K: int) -> int:
    """Candidate-set size of Thm. candidate_size_simp (eq. card)."""
    from math import comb

    B = boundary_count(K)
    tot = 0
    for d in range(1, r + 1):
        for i in range(0, d):
            k2 = 2 * (d - i) - 1
            if n - i < k2 or k2 < 0:
                continue
            tot += comb(n, i) * comb(n - i, k2) * B ** (2 * (d - i) - 2) * (B - 1) ** i
    return tot
