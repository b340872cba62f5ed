"""More pins of the FP64 oracle (CPU only): the rank-1 cell values against the
cell-by-cell definition and brute force, the enumeration counts of Alg. 2
against their closed form, the per-row margin of f(c) against a direct numpy
evaluation, and the FP32-reach interval of f against brute force over the
near-boundary rows."""
import itertools
import os
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute, exact, rank1
from paper_2602_20376_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ rank-1 cells

@pytest.mark.parametrize("n,K", [(7, 3), (9, 4), (6, 5), (10, 2), (8, 7), (200, 3), (150, 16)])
def test_rank1_cells_match_definition(oracle_lib, n, K):
    """Thm. rank1's cell structure: the cumulative-sum cells equal, cell by
    cell, the decision rule evaluated inside each cell and summed directly;
    cell l's value is the objective of cell l's labels."""
    q = inputs.random_V(n, 1, 4100 + 7 * n + K)[:, 0]
    f, order, k0 = rank1.rank1_cells(q, K)
    fd, zd = rank1.rank1_cells_direct(q, K)
    # random q: distinct boundary points, so n + 1 sweep cells; the last cell
    # and the first are the same cell seen from both window ends (labels one
    # step apart, a global rotation: equal objective)
    assert f.size == n + 1 and fd.size == n
    assert abs(f[0] - f[n]) <= 1e-12 * f[0]
    for l in range(n):
        zl = rank1.cell_labels(k0, order, l + 1 if l < n else n, K)
        # the cell after the (l+1)-th point is the l-th direct cell (midpoint
        # of points l and l+1); the wrap-around cell is the last
        assert np.array_equal(zl, zd[l]), l
        val = oracle.objective(q[:, None], K, zl)
        assert abs(f[l + 1] - val) <= 1e-12 * max(val, 1e-300)
        assert abs(fd[l] - val) <= 1e-12 * max(val, 1e-300)


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_rank1_cells_hold_brute_force_optimum(oracle_lib, K):
    """At n <= 10 the best cell is the maximum over all K^n assignments, and
    the brute-force maximiser (up to rotation) is one of the cells."""
    for seed in range(4):
        q = inputs.random_V(9, 1, 5200 + 10 * K + seed)[:, 0]
        opt, zb, _ = brute.brute_force(q[:, None], K)
        f, order, k0 = rank1.rank1_cells(q, K)
        assert abs(f.max() - opt) <= 1e-12 * opt
        o1, z1 = rank1.rank1_sweep(q, K)
        assert o1 == f.max()
        cells = {bytes(oracle.canonical(rank1.cell_labels(k0, order, l, K), K)) for l in range(q.size + 1)}
        assert bytes(oracle.canonical(zb, K)) in cells
        assert np.array_equal(oracle.canonical(z1, K), oracle.canonical(zb, K))


# ------------------------------------------------------------ Alg. 2 counts

def valid_set_count(n: int, r: int, K: int) -> int:
    """Index sets of 2d-1 augmented rows with at most two rows per coordinate,
    summed over the levels d = r..1: p coordinates give two of their B_K rows,
    2d-1-2p others one row each."""
    B = exact.boundary_count(K)
    tot = 0
    for d in range(1, r + 1):
        M = 2 * d - 1
        for p in range(0, M // 2 + 1):
            tot += comb(n, p) * comb(B, 2) ** p * comb(n - p, M - 2 * p) * B ** (M - 2 * p)
    return tot


def test_valid_set_count_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "valid_set_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for n, r, K, val in rows:
        assert valid_set_count(int(n), int(r), int(K)) == int(val)


@pytest.mark.parametrize("n,r,K", [(12, 2, 3), (7, 3, 3), (9, 2, 4), (8, 2, 5), (10, 1, 3), (6, 2, 8), (6, 3, 4),
                                   (10, 5, 2), (7, 6, 4)])
def test_enumeration_counts_closed_form(oracle_lib, n, r, K):
    """The oracle's index-set count equals the closed form (and, for a complex
    factor in general position, no valid set is rank deficient)."""
    V = inputs.random_V(n, r, 900 + 13 * n + r + K)
    ex = exact.solve_exact(V, K)
    assert ex["index_sets"] == valid_set_count(n, r, K)
    assert ex["rank_deficient"] == 0


def test_enumeration_counts_by_itertools():
    """The closed form against a direct count of the combinations."""
    for n, r, K in [(5, 2, 3), (4, 3, 3), (6, 2, 4), (5, 2, 5)]:
        B = exact.boundary_count(K)
        direct = 0
        for d in range(1, r + 1):
            for I in itertools.combinations(range(n * B), 2 * d - 1):
                g = [j // B for j in I]
                if all(g.count(x) <= 2 for x in set(g)):
                    direct += 1
        assert direct == valid_set_count(n, r, K)


# ------------------------------------------------------------ f(c) margin

@pytest.mark.parametrize("K", [2, 3, 5, 16])
def test_f_of_c_margin_direct(oracle_lib, K):
    """min_i dist_i |w_i| / sum_j |V_ij||c_j| from numpy's angle."""
    rng = np.random.default_rng(40 + K)
    V = inputs.random_V(300, 3, 60 + K)
    for _ in range(5):
        g = rng.standard_normal(6)
        c = (g[0::2] + 1j * g[1::2]) / np.linalg.norm(g)
        f, mm = oracle.f_of_c(V, K, c)
        w = V @ c
        x = K * np.angle(w) / (2 * np.pi) + 0.5
        fr = x - np.floor(x)
        dist = np.minimum(fr, 1 - fr) * 2 * np.pi / K
        scale = np.abs(V) @ np.abs(c)
        assert abs(mm - np.min(dist * np.abs(w) / scale)) <= 1e-12
        k = np.mod(np.floor(x).astype(np.int64), K)
        zz = np.exp(2j * np.pi * k / K)
        assert abs(f - np.sum(np.abs(np.conj(V).T @ zz) ** 2)) <= 1e-10 * f


# ------------------------------------------------------------ FP32-reach interval

def test_score_interval_encloses_every_near_boundary_labelling(oracle_lib):
    """oracle.score_dirs: rows whose Euclidean distance to a decision-boundary
    line is within `reach` of their scale are ambiguous; every labelling that
    changes any subset of them to a neighbouring label (all labels when w_i is
    within reach of 0) has its objective inside [lo, hi], and lo <= f <= hi."""
    K = 3
    V = inputs.random_V(40, 2, 77)
    rng = np.random.default_rng(5)
    dirs = []
    for _ in range(6):
        g = rng.standard_normal(4)
        dirs.append((g[0::2] + 1j * g[1::2]) / np.linalg.norm(g))
    # a large reach so that a few rows per direction are ambiguous
    res = oracle.score_dirs(V, K, np.array(dirs), reach=0.15)
    assert np.any(res["nambig"] > 0)
    for t, c in enumerate(dirs):
        w = V @ c
        z0, _ = oracle.labels(V, K, c)
        scale = np.abs(V) @ np.abs(c)
        amb = []
        for i in range(V.shape[0]):
            opts = set()
            for m in range(K):
                ang = np.pi * (2 * m + 1) / K
                d = abs(np.imag(np.exp(-1j * ang) * w[i]))
                along = np.real(np.exp(-1j * ang) * w[i])
                if along > 0 and d <= 0.15 * scale[i]:
                    opts |= {m % K, (m + 1) % K}
            if abs(w[i]) <= 0.15 * scale[i]:
                opts = set(range(K))
            if opts:
                amb.append((i, sorted(opts)))
        assert len(amb) == res["nambig"][t]
        f = res["f"][t]
        assert res["lo"][t] <= f <= res["hi"][t]
        for combo in itertools.product(*[o for _, o in amb]):
            z = z0.copy()
            for (i, _), k in zip(amb, combo):
                z[i] = k
            val = oracle.objective(V, K, z)
            assert res["lo"][t] - 1e-9 <= val <= res["hi"][t] + 1e-9


def test_score_interval_is_tight_without_ambiguity(oracle_lib):
    """With no row within reach, lo = f = hi and f equals f_of_c."""
    V = inputs.random_V(500, 3, 9)
    c = oracle.direction(3, 17, 3)
    res = oracle.score_dirs(V, 5, c[None, :], reach=0.0)
    f, _ = oracle.f_of_c(V, 5, c)
    assert res["nambig"][0] == 0
    assert res["lo"][0] == res["f"][0] == res["hi"][0]
    assert abs(res["f"][0] - f) <= 1e-12 * f


# ------------------------------------------------------------ opposite-ray label

@pytest.mark.parametrize("K", [3, 5, 7, 9, 15])
def test_opposite_ray_label_odd_k(K):
    """For odd K the ray opposite boundary m, at angle pi (2m + 1)/K + pi,
    is the direction of root m + (K + 1)/2 (mod K): the decision rule gives
    that label there and on both sides of the ray up to pi/K away, which the
    exact path's open labels take without evaluating the rule."""
    for m in range(K):
        ang = np.pi * (2 * m + 1) / K + np.pi
        want = (m + (K + 1) // 2) % K
        offs = np.array([0.0, 1e-9, -1e-9, 0.4, -0.4, 0.99, -0.99]) * np.pi / K
        w = 3.7 * np.exp(1j * (ang + offs))
        assert np.all(exact.decision_labels(w, K) == want), (K, m)
        assert all(oracle.label(complex(x), K) == want for x in w), (K, m)
