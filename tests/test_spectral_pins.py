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
