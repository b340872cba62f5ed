"""Pins of the graph-objective and local-search reference (oracle/graph.py)
against facts outside it: the dense quadratic form, the K = 3 cut identity,
brute-force re-evaluation of every move, and a hand-worked example."""
import numpy as np
import pytest

from oracle import graph as og


def _random_graph(n, m, seed, integer=True):
    rng = np.random.default_rng(seed)
    pairs = set()
    while len(pairs) < m:
        a, b = rng.integers(0, n, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    i = np.array([p[0] for p in pairs])
    j = np.array([p[1] for p in pairs])
    w = rng.integers(1, 4, m).astype(np.float64) if integer else rng.uniform(0.1, 2.0, m)
    return i, j, w


def _dense_laplacian(n, edges):
    i, j, w = edges
    L = np.zeros((n, n))
    for a, b, x in zip(i, j, w):
        L[a, b] -= x
        L[b, a] -= x
        L[a, a] += x
        L[b, b] += x
    return L


@pytest.mark.parametrize("K", [2, 3, 5, 8])
def test_quadratic_form_is_the_dense_product(K):
    n = 30
    edges = _random_graph(n, 80, K, integer=False)
    z = np.random.default_rng(K).integers(0, K, n)
    zc = np.exp(2j * np.pi * z / K)
    dense = float(np.real(zc.conj() @ _dense_laplacian(n, edges) @ zc))
    assert abs(og.quadratic_form(edges, K, z) - dense) <= 1e-12 * abs(dense)


def test_k3_objective_is_three_times_the_cut():
    n = 50
    edges = _random_graph(n, 200, 1)
    for s in range(5):
        z = np.random.default_rng(s).integers(0, 3, n)
        assert og.quadratic_form(edges, 3, z) == 3.0 * og.cut_weight(edges, z)


@pytest.mark.parametrize("K", [2, 3, 4, 7])
def test_gain_is_the_change_of_the_objective(K):
    n = 14
    edges = _random_graph(n, 30, 10 + K, integer=(K <= 4))
    nb = og.adjacency(n, edges)
    z = np.random.default_rng(K).integers(0, K, n)
    g, tgt = og.gains(n, nb, K, z)
    base = og.quadratic_form(edges, K, z)
    for v in range(n):
        best = -np.inf
        for b in range(K):
            if b == z[v]:
                continue
            z2 = z.copy()
            z2[v] = b
            best = max(best, og.quadratic_form(edges, K, z2) - base)
        assert abs(g[v] - best) <= 1e-9 * max(1.0, abs(best)), (v, g[v], best)
        z2 = z.copy()
        z2[v] = tgt[v]
        assert abs(og.quadratic_form(edges, K, z2) - base - g[v]) <= 1e-9 * max(1.0, abs(g[v]))


@pytest.mark.parametrize("K", [2, 3, 4, 6])
def test_rounds_move_independent_sets_and_reach_a_local_optimum(K):
    n = 60
    edges = _random_graph(n, 150, 20 + K, integer=(K <= 4))
    nb = og.adjacency(n, edges)
    z = np.random.default_rng(K).integers(0, K, n)
    f = og.quadratic_form(edges, K, z)
    for _ in range(1000):
        z2, moved, g = og.greedy_round(n, nb, K, z)
        if not moved:
            break
        mset = set(moved)
        for v in moved:
            assert all(u not in mset for u, _ in nb[v])
        f2 = og.quadratic_form(edges, K, z2)
        assert abs(f2 - f - sum(g[v] for v in moved)) <= 1e-9 * max(1.0, abs(f2))
        assert f2 > f
        z, f = z2, f2
    assert og.is_local_optimum(n, edges, K, z)
    zg, rounds, moves = og.greedy(n, edges, K, np.random.default_rng(K).integers(0, K, n))
    assert np.array_equal(zg, z) and rounds >= 1 and moves >= rounds


def test_triangle_by_hand():
    # K = 2, all labels 0: every vertex gains 2 edges x |1 - (-1)|^2 = 8; the
    # tie goes to vertex 0, which moves alone.  Then vertices 1 and 2 each
    # have one neighbour on either side: gain 0, no move.  Cut 2 of 3 edges.
    edges = (np.array([0, 0, 1]), np.array([1, 2, 2]), np.ones(3))
    nb = og.adjacency(3, edges)
    z2, moved, g = og.greedy_round(3, nb, 2, np.zeros(3, dtype=np.int64))
    assert list(g) == [8.0, 8.0, 8.0] and moved == [0] and list(z2) == [1, 0, 0]
    z, rounds, moves = og.greedy(3, edges, 2, np.zeros(3, dtype=np.int64))
    assert list(z) == [1, 0, 0] and rounds == 1 and moves == 1
    assert og.cut_weight(edges, z) == 2.0 and og.quadratic_form(edges, 2, z) == 8.0


@pytest.mark.parametrize("K", [3, 5])
def test_vectorized_gains_match_the_loops(K):
    n = 40
    edges = _random_graph(n, 100, 30 + K, integer=False)
    z = np.random.default_rng(K).integers(0, K, n)
    g1, t1 = og.gains(n, og.adjacency(n, edges), K, z)
    g2, t2 = og.gains_vectorized(n, edges, K, z)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-12)
    assert np.array_equal(t1, t2)
