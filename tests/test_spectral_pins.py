"""Pins of the spectral reference (oracle/spectral.py): the Hermitian
Gaussian generator has the moments of its definition (off-diagonal N_C(0,1),
diagonal N(0,1)) and the semicircle edge 2 sqrt(n); the Laplacian's spectrum
has its textbook invariants; the factor convention reproduces the matrix."""
import numpy as np

from oracle import spectral
from paper_2602_20376_amd import inputs


def test_w_is_hermitian_with_the_stated_moments(oracle_lib):
    n = 160
    W = spectral.w_matrix(n, 77)
    assert np.array_equal(W, W.conj().T)
    off = W[np.triu_indices(n, 1)]
    d = np.real(np.diag(W))
    assert abs(np.mean(off)) < 0.03
    assert abs(np.mean(np.abs(off) ** 2) - 1.0) < 0.03
    assert abs(np.var(off.real) - 0.5) < 0.03 and abs(np.var(off.imag) - 0.5) < 0.03
    assert abs(np.mean(off.real * off.imag)) < 0.02
    assert abs(np.var(d) - 1.0) < 0.3
    assert spectral.w_entry(77, 5, 3) == np.conj(spectral.w_entry(77, 3, 5))


def test_entries_of_one_call_are_uncorrelated(oracle_lib):
    """Columns 2q and 2q + 1 of a row take the two word pairs of one Philox
    call: the pair must behave as two independent N_C(0,1) draws."""
    n = 160
    W = spectral.w_matrix(n, 91)
    a, b = [], []
    for i in range(n):
        for q in range(n // 2):
            if 2 * q > i:
                a.append(W[i, 2 * q])
                b.append(W[i, 2 * q + 1])
    a, b = np.array(a), np.array(b)
    assert len(a) > 5000
    assert abs(np.mean(a * np.conj(b))) < 0.03
    assert abs(np.mean(a * b)) < 0.03
    assert abs(np.corrcoef(np.abs(a) ** 2, np.abs(b) ** 2)[0, 1]) < 0.05


def test_semicircle_edge(oracle_lib):
    n = 300
    ev = np.linalg.eigvalsh(spectral.w_matrix(n, 5)) / np.sqrt(n)
    assert 1.85 < ev[-1] < 2.1 and -2.1 < ev[0] < -1.85


def test_laplacian_spectrum_invariants():
    n = 60
    i, j = inputs.random_edges(n, 200, 3)
    w = np.random.default_rng(1).uniform(0.5, 2.0, 200)
    L = spectral.laplacian_dense(n, (i, j, w))
    ev = np.linalg.eigvalsh(L)
    assert abs(ev[0]) < 1e-10 * ev[-1]                  # constant vector
    assert abs(np.sum(ev) - 2 * np.sum(w)) < 1e-9 * np.sum(w)   # trace = sum of weighted degrees
    assert np.all(ev > -1e-10)


def test_factor_reproduces_the_top_part():
    n, r = 40, 3
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M = A @ A.conj().T
    lam, V = spectral.top_factor(M, r)
    ev, U = np.linalg.eigh(M)
    P = U[:, -r:] @ np.diag(ev[-r:]) @ U[:, -r:].conj().T
    assert np.allclose(V @ V.conj().T, P, atol=1e-9 * ev[-1])
    for k in range(r):
        m = int(np.argmax(np.abs(V[:, k])))
        assert abs(V[m, k].imag) < 1e-12 * abs(V[m, k]) and V[m, k].real > 0


def test_w_rows_match_the_entry_definition():
    """The vectorised rows of W (numpy Philox) equal the entry-by-entry
    definition, including rows on both sides of the diagonal and 64-bit
    seeds; Q X on chosen rows equals the dense product."""
    from oracle import spectral as sp

    for n, seed in [(37, 5), (20, 2 ** 40 + 3)]:
        W = sp.w_matrix(n, seed)
        for i in range(n):
            assert np.max(np.abs(sp.w_row(seed, i, n) - W[i])) <= 1e-14
    rng = np.random.default_rng(2)
    n = 30
    U = np.exp(1j * rng.uniform(0, 2 * np.pi, (n, 3)))
    X = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    Q = sp.phase_sync_matrix(U, 2.5, 9)
    rows = [0, 7, 29]
    assert np.max(np.abs(sp.phase_sync_rows_times(U, 2.5, 9, rows, X) - (Q @ X)[rows])) < 1e-12


def test_numpy_philox_matches_c_oracle():
    import oracle
    from oracle import spectral as sp

    rng = np.random.default_rng(3)
    c = rng.integers(0, 2 ** 32, (4, 50), dtype=np.uint64).astype(np.uint32)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    o = sp.philox_np(c[0], c[1], c[2], c[3], k0, k1)
    for t in range(50):
        ref = oracle.philox4x32_10([int(c[0][t]), int(c[1][t]), int(c[2][t]), int(c[3][t])], [k0, k1])
        assert [int(o[q][t]) for q in range(4)] == ref.tolist()
