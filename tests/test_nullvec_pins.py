"""Pins of the null-vector sampler reference (oracle/nullvec.py): enough draws
reach the exact level-r optimum (and the brute-force optimum), and on a real
factor the fraction of rank-deficient draws is the closed form the structure
of the augmented rows fixes."""
import numpy as np

from oracle import brute, exact, nullvec
from paper_2602_20376_amd import inputs


def test_many_draws_reach_the_exact_optimum(oracle_lib):
    V = inputs.random_V(6, 2, 123)
    K = 3
    res = nullvec.nullvec_sampler(V, K, 20000, seed=9)
    ex = exact.solve_exact(V, K, recurse=False)
    opt, _, _ = brute.brute_force(V, K)
    assert abs(res["opt"] - ex["opt"]) <= 1e-12 * ex["opt"]
    assert abs(res["opt"] - opt) <= 1e-12 * opt
    assert res["rank_deficient"] == 0          # complex V: every valid set is full rank
    assert res["valid"] < 20000                # repeated rows and triples occur at N = 18


def test_real_factor_rank_deficient_fraction_is_one_ninth(oracle_lib):
    """Real V, K = 3, r = 2: row (i, m) is [sin a_m V_i, cos a_m V_i], so all
    rows of one boundary index m lie in a 2-dimensional subspace; three rows
    are dependent exactly when they share m, probability 3 (1/3)^3 = 1/9."""
    V = inputs.random_V(400, 2, 77, real=True)
    res = nullvec.nullvec_sampler(V, 3, 6000, seed=4, score=False)
    frac = res["rank_deficient"] / res["valid"]
    assert abs(frac - 1.0 / 9.0) < 0.015, frac


def test_rows_are_uniform():
    N, M, S = 30, 3, 6000
    counts = np.zeros(N)
    for s in range(S):
        for x in nullvec.draw_set(11, s, N, M):
            counts[x] += 1
    expect = S * M / N
    assert np.all(np.abs(counts - expect) < 5 * np.sqrt(expect)), counts
