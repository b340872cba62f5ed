"""Pins of the FP64 oracle to facts outside itself: published known-answer
vectors, the problem's definition by brute force, an independent exact
algorithm (Alg. 1), closed forms and the paper's lemmas and bounds."""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import brute, exact, rank1
from paper_2602_20376_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ RNG stream

def test_philox_known_answers(oracle_lib):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        vals = [int(x, 16) for x in row]
        out = oracle.philox4x32_10(vals[0:4], vals[4:6])
        assert out.tolist() == vals[6:10]


def test_uniform_is_open_interval_and_exact(oracle_lib):
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # 23 random bits: the low 9 bits of the word do not matter
    assert oracle.uniform(0x12345600) == oracle.uniform(0x123457FF)
    # every value is an FP32 number (so both precisions see the same uniform)
    for x in (1, 0x80000000, 0xDEADBEEF, 0x7FFFFFFF):
        u = oracle.uniform(x)
        assert float(np.float32(u)) == u


@pytest.mark.parametrize("r", [2, 3, 4])
def test_sphere_sampler_beta_law(oracle_lib, r):
    """Lemma innerIsBeta (proof of Thm. rr_tail): for c uniform on the complex
    unit sphere, |u^H c|^2 ~ Beta(1, r-1) with mean 1/r, for any unit u."""
    N = 6000
    C = np.array([oracle.direction(77 + r, s, r) for s in range(N)])
    assert np.allclose(np.linalg.norm(C, axis=1), 1.0, atol=1e-14)
    u = inputs.complex_gaussian(_rng(5), r)
    u /= np.linalg.norm(u)
    for vec in (np.eye(r)[0], u):
        x = np.abs(C @ np.conj(vec)) ** 2
        p = stats.kstest(x, stats.beta(1, r - 1).cdf).pvalue
        assert p > 1e-3, p
        assert abs(x.mean() - 1.0 / r) < 4.0 * x.std() / np.sqrt(N)
    # the phase of each coordinate is uniform
    ph = (np.angle(C[:, 0]) + np.pi) / (2 * np.pi)
    assert stats.kstest(ph, "uniform").pvalue > 1e-3


def test_direction_stream_depends_on_all_counter_words(oracle_lib):
    a = oracle.direction(1, 5, 3, instance=0)
    assert not np.allclose(a, oracle.direction(2, 5, 3, instance=0))
    assert not np.allclose(a, oracle.direction(1, 6, 3, instance=0))
    assert not np.allclose(a, oracle.direction(1, 5, 3, instance=1))
    assert not np.allclose(a, oracle.direction(1, 5 + (1 << 32), 3, instance=0))


# ------------------------------------------------------------ decision rule

@pytest.mark.parametrize("K", [2, 3, 4, 5, 8, 16, 255])
def test_label_is_nearest_root(oracle_lib, K):
    """eq. decision_rule: the label maximises Re(conj(omega^k) w)."""
    rng = _rng(K)
    roots = np.exp(2j * np.pi * np.arange(K) / K)
    for w in rng.standard_normal(400) + 1j * rng.standard_normal(400):
        k = oracle.label(w, K)
        d = np.real(np.conj(roots) * w)
        if np.sort(d)[-1] - np.sort(d)[-2] > 1e-9:
            assert k == int(np.argmax(d))
    assert oracle.label(0j, K) == 0


def test_boundary_distance_closed_form(oracle_lib):
    K = 3
    # a point exactly at a root is pi/K from both neighbouring boundaries
    assert abs(oracle.boundary_distance(np.exp(2j * np.pi / 3), K) - np.pi / 3) < 1e-12
    # just past the first boundary (angle pi/3)
    w = np.exp(1j * (np.pi / 3 + 1e-3))
    assert abs(oracle.boundary_distance(w, K) - 1e-3) < 1e-12
    assert oracle.label(w, K) == 1
    assert oracle.label(np.exp(1j * (np.pi / 3 - 1e-3)), K) == 0


@pytest.mark.parametrize("K", [2, 3, 4])
def test_labels_solve_inner_maximisation(oracle_lib, K):
    """For a fixed c, the decision rule is the argmax over all K^n labellings
    of Re(z^H V c) (inner maximisation of eq. rankr_double)."""
    V = inputs.random_V(7, 2, 11 + K)
    for s in range(5):
        c = oracle.direction(3, s, 2)
        z, dist = oracle.labels(V, K, c)
        zb, _ = brute.max_assignment_for_direction(V, K, c)
        assert dist.min() > 1e-9
        assert np.array_equal(z, zb)


def test_objective_is_quadratic_form(oracle_lib):
    """||V^H z||^2 = z^H Q z with Q = V V^H (eq. quad_max-norm)."""
    V = inputs.random_V(30, 3, 4)
    Q = V @ V.conj().T
    rng = _rng(1)
    for K in (2, 3, 8):
        z = rng.integers(0, K, 30).astype(np.uint8)
        zc = np.exp(2j * np.pi * z / K)
        assert abs(oracle.objective(V, K, z) - np.real(zc.conj() @ Q @ zc)) < 1e-10


def test_phase_equivalence(oracle_lib):
    """Lemma phase_equiv: a global K-th-root rotation keeps the objective."""
    V = inputs.random_V(25, 3, 8)
    z = _rng(2).integers(0, 5, 25).astype(np.uint8)
    f = oracle.objective(V, 5, z)
    for t in range(1, 5):
        assert abs(oracle.objective(V, 5, (z + t) % 5) - f) < 1e-11 * f


def test_rotation_equivariance_of_labels(oracle_lib):
    """Periodicity z(omega c) = omega z(c) (Lemma angle_reduction)."""
    K = 5
    V = inputs.random_V(40, 3, 9)
    om = np.exp(2j * np.pi / K)
    for s in range(10):
        c = oracle.direction(4, s, 3)
        z, dist = oracle.labels(V, K, c)
        z2, _ = oracle.labels(V, K, om * c)
        ok = dist > 1e-9
        assert np.array_equal(z2[ok], ((z.astype(int) + 1) % K)[ok])


@pytest.mark.parametrize("K", [2, 3, 5, 8])
def test_pointwise_rounding_bound(oracle_lib, K):
    """eq. f_pointwise: f(c) >= cos^2(pi/K) ||V c||_1^2 for every unit c."""
    V = inputs.random_V(60, 3, 10 + K)
    for s in range(50):
        c = oracle.direction(5, s, 3)
        f, _ = oracle.f_of_c(V, K, c)
        assert f >= np.cos(np.pi / K) ** 2 * np.sum(np.abs(V @ c)) ** 2 * (1 - 1e-12)


# ------------------------------------------------------------ exact solvers

EXACT_CASES = [(12, 2, 3), (9, 2, 4), (8, 2, 5), (7, 3, 3), (10, 1, 3), (9, 2, 2),
               (6, 3, 4), (7, 1, 8), (6, 2, 8),
               # r = 5 .. 8: levels whose sets have 9 to 15 rows
               (10, 5, 2), (12, 6, 2), (7, 6, 4), (14, 7, 2)]


@pytest.mark.parametrize("n,r,K", EXACT_CASES)
def test_exact_equals_brute_force(oracle_lib, n, r, K):
    """Thm. rankr: Alg. 2 reaches the maximum over all K^n assignments."""
    V = inputs.random_V(n, r, 100 * n + 10 * r + K)
    ex = exact.solve_exact(V, K)
    opt, zb, ties = brute.brute_force(V, K)
    assert abs(ex["opt"] - opt) <= 1e-12 * opt
    assert ties == K          # unique up to the K global rotations
    assert np.array_equal(oracle.canonical(ex["z"], K), oracle.canonical(zb, K))
    assert abs(oracle.objective(V, K, ex["z"]) - opt) <= 1e-12 * opt


def test_exact_real_factor_orbit(oracle_lib):
    """For a real V, conjugation is a symmetry too: 2K maximisers for K >= 3."""
    V = inputs.random_V(9, 2, 55, real=True)
    ex = exact.solve_exact(V, 3)
    opt, zb, ties = brute.brute_force(V, 3)
    assert abs(ex["opt"] - opt) <= 1e-12 * opt
    assert ties == 6
    assert np.array_equal(oracle.canonical(ex["z"], 3, True), oracle.canonical(zb, 3, True))


@pytest.mark.parametrize("K", [2, 3, 4, 7])
def test_rank1_sweep_equals_brute_force(oracle_lib, K):
    """Alg. 1 (Thm. rank1) against the definition."""
    q = inputs.random_V(8, 1, 300 + K)[:, 0]
    opt, _, _ = brute.brute_force(q[:, None], K)
    o1, z1 = rank1.rank1_sweep(q, K)
    assert abs(o1 - opt) <= 1e-12 * opt
    assert abs(oracle.objective(q[:, None], K, z1) - opt) <= 1e-12 * opt


@pytest.mark.parametrize("K", [3, 4])
def test_exact_rank1_equals_sweep_large_n(oracle_lib, K):
    """Two independent exact algorithms agree at r = 1, n = 400."""
    q = inputs.random_V(400, 1, 77 + K)
    o1, z1 = rank1.rank1_sweep(q[:, 0], K)
    ex = exact.solve_exact(q, K)
    assert abs(ex["opt"] - o1) <= 1e-11 * o1
    assert np.array_equal(oracle.canonical(ex["z"], K), oracle.canonical(z1, K))


def test_rank1_binary_is_sign(oracle_lib):
    """K = 2 and a real rank-1 factor: the maximiser is sign(q) (Sec. 1)."""
    q = _rng(3).standard_normal(500)
    o1, z1 = rank1.rank1_sweep(q.astype(complex), 2)
    assert abs(o1 - np.sum(np.abs(q)) ** 2) <= 1e-10 * o1
    sgn = (q < 0).astype(np.uint8)        # label 1 is the root -1
    assert np.array_equal(oracle.canonical(z1, 2), oracle.canonical(sgn, 2))


def test_card_formula_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "card_formula.txt"))
            if l.strip() and not l.startswith("#")]
    for n, r, K, val in rows:
        assert exact.card_formula(int(n), int(r), int(K)) == int(val)


def test_candidate_count_bounded_by_card(oracle_lib):
    """Distinct candidates never exceed eq. card (they are far fewer)."""
    V = inputs.random_V(6, 2, 12)
    ex = exact.solve_exact(V, 3, collect_distinct=True)
    # per rotation class: canonicalise to count cells up to the K-fold symmetry
    classes = {bytes(oracle.canonical(np.frombuffer(b, np.uint8), 3)) for b in ex["distinct_set"]}
    assert len(classes) <= exact.card_formula(6, 2, 3)


@pytest.mark.parametrize("n,r,K", [(8, 2, 3), (7, 3, 3), (6, 2, 4), (9, 2, 2), (10, 5, 2)])
def test_candidate_set_holds_brute_force_maximiser(oracle_lib, n, r, K):
    """Thm. rankr: the labellings that Alg. 2 enumerates include the maximiser
    over all K^n assignments (up to a global rotation), and the best of them
    is the brute-force optimum."""
    V = inputs.random_V(n, r, 7000 + 10 * n + r + K)
    ex = exact.solve_exact(V, K, collect_distinct=True)
    opt, zb, _ = brute.brute_force(V, K)
    classes = {bytes(oracle.canonical(np.frombuffer(b, np.uint8), K)) for b in ex["distinct_set"]}
    assert bytes(oracle.canonical(zb, K)) in classes
    Z = np.array([np.frombuffer(b, np.uint8) for b in ex["distinct_set"]], dtype=np.int64)
    assert abs(exact.objective_many(V, K, Z).max() - opt) <= 1e-12 * opt


def test_two_implies_all_and_triples(oracle_lib):
    """Cor. two_implies_all: two rows of one group force V_i c = 0;
    Lemma rank_deficiency: three rows of one group are rank deficient."""
    K = 3
    V = inputs.random_V(5, 2, 21)
    A = exact.tilde_rows(V, K)
    B = exact.boundary_count(K)
    I = [0 * B + 0, 0 * B + 1, 2 * B + 1]
    _, s, Vt = np.linalg.svd(A[I], full_matrices=True)
    v = Vt[-1]
    c = v[:2] + 1j * v[2:]
    assert abs(V[0] @ c) < 1e-12
    assert np.linalg.matrix_rank(A[[B, B + 1, B + 2]]) == 2
    # hyperplane property: a_{i,m} . c~ = Im(rho_m V_i c)
    rng = _rng(4)
    ct = rng.standard_normal(4)
    cc = ct[:2] + 1j * ct[2:]
    for i in range(5):
        for m in range(B):
            rho = np.exp(-1j * np.pi * (2 * m + 1) / K)
            assert abs(A[i * B + m] @ ct - np.imag(rho * (V[i] @ cc))) < 1e-12


def test_antipodal_boundary_count():
    """Lemma antipodal: B_K = K/2 for even K, K for odd K."""
    assert [exact.boundary_count(K) for K in (2, 3, 4, 5, 6, 8, 16)] == [1, 3, 2, 5, 3, 4, 8]


# ------------------------------------------------------------ spectral bounds

@pytest.mark.parametrize("K", [2, 3, 4])
def test_opt_spectral_bounds(oracle_lib, K):
    """OPT <= lambda_1 n (Sec. 4.2 proofs) and OPT >= lambda_1 cos^2(pi/K)
    ||u_1||_1^2 (Lemma opt_lower, rounding the top eigenvector)."""
    V = inputs.random_V(10, 2, 31 + K)
    Q = V @ V.conj().T
    lam, U = np.linalg.eigh(Q)
    opt, _, _ = brute.brute_force(V, K)
    assert opt <= lam[-1] * 10 * (1 + 1e-12)
    assert opt >= lam[-1] * np.cos(np.pi / K) ** 2 * np.sum(np.abs(U[:, -1])) ** 2 * (1 - 1e-12)


# ------------------------------------------------------------ sampled best-of-S

def test_sampled_is_best_of_its_stream(oracle_lib):
    V = inputs.random_V(50, 3, 41)
    res = oracle.sampled(V, 4, 300, seed=9)
    f = res["f"]
    assert res["best_s"] == int(np.argmax(f))
    for s in (0, 17, 299):
        c = oracle.direction(9, s, 3)
        z, _ = oracle.labels(V, 4, c)
        assert abs(f[s] - oracle.objective(V, 4, z)) <= 1e-12 * f[s]


def test_sampled_reaches_opt_small_n(oracle_lib):
    """Best-of-S never exceeds OPT and reaches it at S in the thousands for
    n <= 10 (Sec. 5.2: best-of-S reaches OPT_r by S ~ 100 at n <= 100)."""
    for seed, (n, r, K) in enumerate([(9, 2, 3), (8, 3, 3), (10, 2, 4)]):
        V = inputs.random_V(n, r, 500 + seed)
        opt, _, _ = brute.brute_force(V, K)
        res = oracle.sampled(V, K, 4000, seed=seed)
        assert res["best_f"] <= opt * (1 + 1e-12)
        assert res["best_f"] >= opt * (1 - 1e-12)
        # a single draw is at least the cos^2(pi/K)/r floor in expectation
        assert res["f"].mean() >= np.cos(np.pi / K) ** 2 / r * opt


def test_sampled_range_split_merges(oracle_lib):
    """Disjoint candidate ranges merged by max equal the whole range."""
    V = inputs.random_V(40, 2, 42)
    whole = oracle.sampled(V, 3, 1000, seed=3)
    parts = [oracle.sampled(V, 3, 250, seed=3, s0=250 * p) for p in range(4)]
    best = max(parts, key=lambda p: (p["best_f"], -p["best_s"]))
    assert best["best_s"] == whole["best_s"] and best["best_f"] == whole["best_f"]
    assert np.array_equal(np.concatenate([p["f"] for p in parts]), whole["f"])


def test_canonical_forms():
    z = np.array([2, 0, 1, 1], dtype=np.uint8)
    assert oracle.canonical(z, 3).tolist() == [0, 1, 2, 2]
    assert oracle.canonical((z + 1) % 3, 3).tolist() == [0, 1, 2, 2]
    # conjugate orbit for a real factor
    assert oracle.canonical((-z.astype(int)) % 3, 3, True).tolist() == \
        oracle.canonical(z, 3, True).tolist()


# ------------------------------------------------------------ planted mistakes

def test_pins_catch_a_dropped_half(oracle_lib):
    """A decision rule missing the +1/2 (floor instead of nearest) must be
    caught by the inner-maximisation pin (brute force over K^n)."""
    V = inputs.random_V(7, 2, 808)
    caught = 0
    for s in range(5):
        c = oracle.direction(8, s, 2)
        w = V @ c
        good = exact.decision_labels(w, 3)
        wrong = np.mod(np.floor(3 * np.angle(w) / (2 * np.pi)).astype(np.int64), 3)
        zb, _ = brute.max_assignment_for_direction(V, 3, c)
        assert np.array_equal(good, zb)
        caught += not np.array_equal(wrong, zb)
    assert caught >= 3


def test_pins_catch_swapped_columns(oracle_lib):
    """The column order [Re(rho V), Im(rho V)] as printed in eq. tildeV does
    not give the boundary condition Im(rho_m V_i c) = 0 that Lemma antipodal
    and Cor. two_implies_all use; the hyperplane identity rejects it."""
    K = 3
    V = inputs.random_V(4, 2, 909)
    A = exact.tilde_rows(V, K)
    printed = np.concatenate([A[:, 2:], A[:, :2]], axis=1)
    ct = _rng(9).standard_normal(4)
    cc = ct[:2] + 1j * ct[2:]
    B = exact.boundary_count(K)
    err_good, err_printed = 0.0, 0.0
    for i in range(4):
        for m in range(B):
            target = np.imag(np.exp(-1j * np.pi * (2 * m + 1) / K) * (V[i] @ cc))
            err_good = max(err_good, abs(A[i * B + m] @ ct - target))
            err_printed = max(err_printed, abs(printed[i * B + m] @ ct - target))
    assert err_good < 1e-12 and err_printed > 1e-3
