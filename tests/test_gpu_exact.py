"""GPU parity of the exact solver (Alg. 2) against the FP64 oracle and the
brute-force definition, through the C-ABI.

Bar: the objective equals the oracle's OPT to 1e-12 relative, the labels
equal the oracle's maximiser up to the symmetry orbit (global K-th-root
rotation; conjugation too for a real factor), and the enumeration statistics
(valid index sets, rank-deficient sets, scored label vectors) match the
oracle's counts exactly.
"""
import os
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute, exact, rank1
from paper_2602_20376_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "valid_set_counts.txt"))
            if l.strip() and not l.startswith("#")]
    return {(int(a), int(b), int(c)): int(d) for a, b, c, d in rows}


pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrqo_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20376_amd import lrqo

    lrqo.load()
    return lrqo


def _solve(lrqo_mod, V, K):
    z, res = lrqo_mod.solve_exact(torch.from_numpy(np.ascontiguousarray(V)).cuda(), K)
    return z.cpu().numpy(), res


def _check(V, K, z, res, real=False, stats=True):
    ex = exact.solve_exact(V, K)
    assert abs(res.obj - ex["opt"]) <= 1e-12 * ex["opt"], (res.obj, ex["opt"])
    assert abs(oracle.objective(V, K, z) - res.obj) <= 1e-12 * res.obj
    assert np.array_equal(oracle.canonical(z, K, real), oracle.canonical(ex["z"], K, real))
    if stats:
        assert res.index_sets == ex["index_sets"]
        assert res.rank_deficient == ex.get("rank_deficient", 0)
        assert res.candidates == ex["candidates"]
    return ex


def test_exact_small_workload(lrqo_mod):
    """The 12 x 2 complex N_C(0,1) workload with K = 3 against brute force over 3^12."""
    inst = inputs.exact_small()
    z, res = _solve(lrqo_mod, inst.V, 3)
    _check(inst.V, 3, z, res)
    opt, zb, ties = brute.brute_force(inst.V, 3)
    assert abs(res.obj - opt) <= 1e-12 * opt and ties == 3
    assert np.array_equal(oracle.canonical(z, 3), oracle.canonical(zb, 3))


@pytest.mark.parametrize("n,r,K", [(9, 2, 4), (8, 2, 5), (7, 3, 3), (10, 1, 3), (9, 2, 2),
                                   (6, 3, 4), (7, 1, 8), (6, 2, 8), (6, 4, 3), (4, 2, 17), (3, 1, 255)])
def test_exact_vs_brute(lrqo_mod, n, r, K):
    V = inputs.random_V(n, r, 100 * n + 10 * r + K)
    z, res = _solve(lrqo_mod, V, K)
    _check(V, K, z, res)
    opt, zb, _ = brute.brute_force(V, K)
    assert abs(res.obj - opt) <= 1e-12 * opt


HIGH_RANK = [(10, 5, 2), (6, 5, 3), (7, 6, 4), (12, 6, 2), (14, 7, 2), (15, 8, 2), (8, 8, 4)]


@pytest.mark.parametrize("n,r,K", HIGH_RANK)
def test_exact_high_rank_vs_brute(lrqo_mod, n, r, K):
    """r = 5 .. 8 (sets of 9 to 15 rows; their levels solve each vertex with
    sixteen lanes, the lower levels one thread per set): optimum, labels and
    every count equal to the oracle's, and the optimum is the brute force."""
    V = inputs.random_V(n, r, 100 * n + 10 * r + K)
    z, res = _solve(lrqo_mod, V, K)
    _check(V, K, z, res)
    opt, _, _ = brute.brute_force(V, K)
    assert abs(res.obj - opt) <= 1e-12 * opt


@pytest.mark.parametrize("n,r,K,chunk,form", [(10, 5, 2, 7, "fused"), (7, 6, 4, 100, "split"), (12, 6, 2, 5, "fused"),
                                              (14, 7, 2, 1000, "fused"), (15, 8, 2, 4096, "split")])
def test_exact_high_rank_forms(lrqo_mod, n, r, K, chunk, form, monkeypatch):
    """The fused and split scorers and ragged chunks at r = 5 .. 8 against
    the oracle."""
    monkeypatch.setenv("LRQO_EXACT_CHUNK", str(chunk))
    if form:
        monkeypatch.setenv("LRQO_EXACT_FORM", form)
    V = inputs.random_V(n, r, 100 * n + 10 * r + K)
    z, res = _solve(lrqo_mod, V, K)
    _check(V, K, z, res)


def test_exact_high_rank_real_factor(lrqo_mod):
    """A real factor at r = 5, K = 4 (not in general position: a quarter of
    the sets are rank deficient): optimum and labels up to rotation and
    conjugation against the oracle and the brute force."""
    V = inputs.random_V(7, 5, 515, real=True)
    z, res = _solve(lrqo_mod, V, 4)
    _check(V, 4, z, res, real=True, stats=False)
    opt, _, _ = brute.brute_force(V, 4)
    assert abs(res.obj - opt) <= 1e-12 * opt
    assert res.warning == -6


@pytest.mark.parametrize("n,r", [(10, 1), (8, 3), (6, 4)])
def test_exact_real_factor_k3_ranks(lrqo_mod, n, r):
    """Real factors with K = 3 at r = 1, 3, 4 (the row pass in the q basis
    with the clamped label tests): optimum and labels up to rotation and
    conjugation against the oracle and the brute force."""
    V = inputs.random_V(n, r, 300 + n + r, real=True)
    z, res = _solve(lrqo_mod, V, 3)
    _check(V, 3, z, res, real=True, stats=False)
    opt, _, _ = brute.brute_force(V, 3)
    assert abs(res.obj - opt) <= 1e-12 * opt


@pytest.mark.parametrize("r", [2, 6])
def test_exact_real_factor_k2_is_flagged(lrqo_mod, r):
    """A real factor with K = 2 is far from general position: every augmented
    row is [-V_i, 0], so the rows only constrain Re c and every set of more
    than one row is rank deficient.  Assumption 1 fails, the call says so
    (LRQO_EDEGENERATE) and returns the best candidate it found, whose FP64
    objective is the returned one; optimality is not claimed (the oracle,
    which branches every row lying on a boundary line, reaches the brute-force
    optimum here by enumerating every labelling)."""
    V = inputs.random_V(12, r, 515, real=True)
    z, res = _solve(lrqo_mod, V, 2)
    assert res.warning == -6 and res.rank_deficient > 0
    assert abs(oracle.objective(V, 2, z) - res.obj) <= 1e-12 * res.obj


def test_exact_high_rank_at_scale(lrqo_mod):
    """n = 30, r = 5, K = 2: 1.7e7 index sets (beyond the oracle's reach; the
    fused scorer runs).  Held to what holds at any size: the count equals
    sum_d C(30, 2d-1), the FP64 objective of the returned labels is the
    returned objective, and the exact optimum is at least the best of 2^20
    sampled directions."""
    V = inputs.random_V(30, 5, 3050)
    z, res = _solve(lrqo_mod, V, 2)
    print(f"exact n=30 r=5: {res.index_sets} sets in {res.device_ms:.0f} ms", flush=True)
    assert res.index_sets == sum(comb(30, 2 * d - 1) for d in range(1, 6))
    assert res.rank_deficient == 0 and res.warning == 0
    assert abs(oracle.objective(V, 2, z) - res.obj) <= 1e-12 * res.obj
    samp = lrqo_mod.solve_sampled(torch.from_numpy(V.astype(np.complex64)).cuda(), 2, 1 << 20, 3)
    V32 = V.astype(np.complex64).astype(np.complex128)
    assert oracle.objective(V32, 2, z) >= oracle.objective(V32, 2, samp.z.cpu().numpy()) * (1 - 1e-6)


def test_exact_larger_n(lrqo_mod):
    """n = 20 (34,220 index sets at r = 2): several tiles of 256 threads and a
    ragged last block; no brute force, the oracle's Alg. 2 decides."""
    V = inputs.random_V(20, 2, 2020)
    z, res = _solve(lrqo_mod, V, 3)
    _check(V, 3, z, res)


def test_exact_fused_form_at_scale(lrqo_mod):
    """n = 80, r = 2, K = 3: C(240, 3) + 240 index sets (2.3 million), more
    than the split scorer's buffers take, so the fused scorer runs.  Too
    large for the oracle's enumeration; held to what holds at any size: the
    FP64 objective of the returned labels is the returned objective, and the
    exact optimum is at least the best of 2^18 sampled directions on the same
    factor."""
    V = inputs.random_V(80, 2, 8080)
    z, res = _solve(lrqo_mod, V, 3)
    assert res.index_sets > 2_000_000
    assert abs(oracle.objective(V, 3, z) - res.obj) <= 1e-12 * res.obj
    samp = lrqo_mod.solve_sampled(torch.from_numpy(V.astype(np.complex64)).cuda(), 3, 1 << 18, 80)
    V32 = V.astype(np.complex64).astype(np.complex128)
    f_samp = oracle.objective(V32, 3, samp.z.cpu().numpy())
    f_exact_on_32 = oracle.objective(V32, 3, z)
    assert res.obj >= samp.obj * (1 - 1e-6), (res.obj, samp.obj)
    assert f_exact_on_32 >= f_samp * (1 - 1e-6)


def test_exact_first_chunk_floor_drops_nothing(lrqo_mod, monkeypatch):
    """The first chunk's selection floor (the 64th largest distinct maximum of
    its groups of 2,048 scores) may only drop scores that cannot enter the
    best 64.  A one-chunk solve (n = 80, r = 2, K = 3: 2.3 million sets, the
    floor on) returns the same objective, labels and counts as the same solve
    in chunks of 100,000 sets, which never take that floor (later chunks take
    the shortlist's).  Both run the fused scorer, so every set's FP32 score is
    the same number in both."""
    V = inputs.random_V(80, 2, 8081)
    monkeypatch.setenv("LRQO_EXACT_FORM", "fused")
    z1, r1 = _solve(lrqo_mod, V, 3)
    monkeypatch.setenv("LRQO_EXACT_CHUNK", "100000")
    z2, r2 = _solve(lrqo_mod, V, 3)
    assert r1.index_sets > 20 * 100_000
    assert r1.obj == r2.obj and np.array_equal(z1, z2)
    assert (r1.index_sets, r1.candidates, r1.rank_deficient) == (r2.index_sets, r2.candidates, r2.rank_deficient)


def test_exact_real_factor(lrqo_mod):
    """A real factor violates general position (Assumption 1): at vertices
    c ~ exp(i pi(2m+1)/K) x, x real, every row lies on boundary line m.  The
    oracle branches such rows (a superset), the GPU path does not, so only the
    optimum and its labels are compared, not the candidate counts."""
    for seed in (55, 56, 57):
        V = inputs.random_V(9, 2, seed, real=True)
        z, res = _solve(lrqo_mod, V, 3)
        _check(V, 3, z, res, real=True, stats=False)
        opt, _, _ = brute.brute_force(V, 3)
        assert abs(res.obj - opt) <= 1e-12 * opt


@pytest.mark.parametrize("n,r,K", [(40, 2, 3), (14, 3, 4), (300, 1, 5)])
def test_exact_real_and_rotated_factor_agree(lrqo_mod, n, r, K):
    """A real factor (all imaginary parts zero: the row scorers take real
    arithmetic) and the same factor times a global phase (complex
    arithmetic) have the same optimum, since |(e^{it} V)^H z| = |V^H z|."""
    V = inputs.random_V(n, r, 70 + n, real=True)
    _, r1 = _solve(lrqo_mod, V, K)
    _, r2 = _solve(lrqo_mod, V * np.exp(0.7j), K)
    assert abs(r1.obj - r2.obj) <= 1e-12 * r1.obj
    if r == 1:   # against Alg. 1, an independent exact algorithm
        opt = rank1.rank1_sweep(V[:, 0], K)[0]
        assert abs(r1.obj - opt) <= 1e-12 * opt


def test_exact_rank1_long(lrqo_mod):
    """r = 1, n = 3000 against Alg. 1 (independent exact algorithm)."""
    q = inputs.random_V(3000, 1, 31)
    z, res = _solve(lrqo_mod, q, 5)
    o1, z1 = rank1.rank1_sweep(q[:, 0], 5)
    assert abs(res.obj - o1) <= 1e-11 * o1
    assert np.array_equal(oracle.canonical(z, 5), oracle.canonical(z1, 5))


def test_exact_degenerate_duplicate_rows(lrqo_mod):
    """Duplicated rows break general position: rank-deficient sets are
    counted and skipped, the optimum is still the brute-force one."""
    V = inputs.random_V(7, 2, 77)
    V[3] = V[1]
    z, res = _solve(lrqo_mod, V, 3)
    opt, _, _ = brute.brute_force(V, 3)
    assert abs(res.obj - opt) <= 1e-12 * opt
    assert res.rank_deficient > 0
    assert res.warning == -6            # LRQO_EDEGENERATE: general position violated


def test_exact_general_position_no_warning(lrqo_mod):
    V = inputs.random_V(9, 2, 78)
    _, res = _solve(lrqo_mod, V, 3)
    assert res.rank_deficient == 0 and res.warning == 0


@pytest.mark.parametrize("form", ["fused", "split"])
@pytest.mark.parametrize("n,r,K", [(12, 2, 3), (16, 2, 3), (20, 2, 3), (9, 3, 3), (13, 2, 4), (14, 1, 7)])
def test_exact_forms_vs_oracle(lrqo_mod, n, r, K, form, monkeypatch):
    """Each form forced at small n: the fused scorer (one pass over all rows
    per set) and the split one (vertex records, the row pass, the
    combinations; small sizes take the fused form by default): optimum,
    labels and every count equal to the oracle's."""
    monkeypatch.setenv("LRQO_EXACT_FORM", form)
    V = inputs.random_V(n, r, 600 + 7 * n + r + K)
    z, res = _solve(lrqo_mod, V, K)
    _check(V, K, z, res)


@pytest.mark.parametrize("chunk,form", [(1, ""), (7, "fused"), (1000, "split"), (1000, "fused"), (4096, "split"),
                                        (4096, "")])
def test_exact_chunked_shortlist(lrqo_mod, chunk, form, monkeypatch):
    """The sets taken in chunks, each chunk's best distinct scores merged into
    the shortlist (chunk = 1: every set merged on its own; 7: ragged
    chunks), against the oracle on the 12 x 2 workload and the brute force."""
    monkeypatch.setenv("LRQO_EXACT_CHUNK", str(chunk))
    if form:
        monkeypatch.setenv("LRQO_EXACT_FORM", form)
    inst = inputs.exact_small()
    z, res = _solve(lrqo_mod, inst.V, 3)
    _check(inst.V, 3, z, res)
    assert res.index_sets == _golden_counts()[(12, 2, 3)]


def test_exact_counts_closed_form(lrqo_mod):
    """Valid index sets equal the closed form at several sizes (golden values
    evaluated by hand, and the formula beyond them)."""
    gold = _golden_counts()
    for (n, r, K) in [(12, 2, 3), (6, 2, 3), (10, 1, 4)]:
        V = inputs.random_V(n, r, 40 + n)
        _, res = _solve(lrqo_mod, V, K)
        assert res.index_sets == gold[(n, r, K)]
    B = 3
    for n in (64, 160):
        V = inputs.random_V(n, 2, 4000 + n)
        _, res = _solve(lrqo_mod, V, 3)
        want = n * B + comb(n, 3) * B ** 3 + n * comb(B, 2) * (n - 1) * B
        assert res.index_sets == want


def test_exact_cap_and_force(lrqo_mod):
    """Above the cap the call is refused before device work; a negative cap
    lifts it (n = 1,200 at r = 2, K = 3: 7.8e9 sets, refused under
    max_sets = 10^9)."""
    V = torch.from_numpy(inputs.random_V(1200, 2, 5)).cuda()
    with pytest.raises(lrqo_mod.LrqoError, match="ETOOBIG"):
        lrqo_mod.solve_exact(V, 3, max_sets=10 ** 9)
    small = torch.from_numpy(inputs.random_V(30, 2, 6)).cuda()
    with pytest.raises(lrqo_mod.LrqoError, match="ETOOBIG"):
        lrqo_mod.solve_exact(small, 3, max_sets=1000)
    _, res = lrqo_mod.solve_exact(small, 3, max_sets=-1)
    assert res.index_sets == 30 * 3 + comb(30, 3) * 27 + 30 * 3 * 29 * 3


@pytest.mark.parametrize("n", [1000, 1500])
def test_exact_beyond_2_32_sets(lrqo_mod, n):
    """Rank-2 exact enumeration at the sizes of the paper's GPU campaign
    (n = 1,000: 4.5e9 index sets; n = 1,500: 1.5e10, both beyond 32-bit set
    indices), K = 3: every set enumerated (the count equals the closed form),
    the FP64 objective of the returned labels is the returned objective, and
    the exact optimum is at least the best of 2^20 sampled directions."""
    V = inputs.random_V(n, 2, 7000 + n)
    z, res = _solve(lrqo_mod, V, 3)
    print(f"exact n={n}: {res.index_sets} sets in {res.device_ms:.0f} ms, obj {res.obj!r}", flush=True)
    assert res.index_sets == _golden_counts()[(n, 2, 3)]
    assert res.rank_deficient == 0 and res.warning == 0
    assert abs(oracle.objective(V, 3, z) - res.obj) <= 1e-11 * res.obj
    samp = lrqo_mod.solve_sampled(torch.from_numpy(V.astype(np.complex64)).cuda(), 3, 1 << 20, 99 + n)
    V32 = V.astype(np.complex64).astype(np.complex128)
    assert oracle.objective(V32, 3, z) >= oracle.objective(V32, 3, samp.z.cpu().numpy()) * (1 - 1e-6)


def test_exact_nonfinite(lrqo_mod):
    V = inputs.random_V(6, 2, 1)
    V[2, 0] = np.inf
    with pytest.raises(lrqo_mod.LrqoError, match="ENOTFINITE"):
        _solve(lrqo_mod, V, 3)
