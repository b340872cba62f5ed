"""The phase-synchronisation factor is drawn from the spiked-model law of the
top eigenvectors of Q = U U^H + sigma W (U unit-modulus random phases,
W Hermitian Gaussian, sigma = 0.5 sqrt(n)) instead of an eigen-decomposition
of the dense Q, which does not fit at n = 262,144.  At a size where the dense
matrix fits, the law and the dense eigenvectors must agree on the statistics
the solver sees: the eigenvalue scale, the overlap with the planted phases and
the spread of the row norms."""
import numpy as np

from paper_2602_20376_amd import inputs


def _dense_top(n, r, seed):
    rng = np.random.default_rng(seed)
    U = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, (n, r)))
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    W = (G + G.conj().T) / np.sqrt(2.0)       # off-diagonal N_C(0,1), diagonal N(0,1)
    lam, E = np.linalg.eigh(U @ U.conj().T + 0.5 * np.sqrt(n) * W)
    lam, E = lam[::-1][:r], E[:, ::-1][:, :r]
    Uq, _ = np.linalg.qr(U)
    overlap = np.linalg.svd(Uq.conj().T @ E, compute_uv=False) ** 2
    return lam, E * np.sqrt(lam)[None, :], overlap


def _row_fourth_moment(V):
    w = np.sum(np.abs(V) ** 2, axis=1)
    return len(w) * np.sum(w ** 2) / np.sum(w) ** 2


def test_phase_sync_law_matches_dense_eigenvectors():
    n, r = 1024, 3
    lam_d, m4_d, m4_l, ov_d, lam_l = [], [], [], [], []
    for seed in range(4):
        lam, E, ov = _dense_top(n, r, seed)
        V = inputs.phase_sync_factor(n, r, 100 + seed)
        lam_d.append(lam / n)
        ov_d.append(ov)
        lam_l.append(np.sum(np.abs(V) ** 2, axis=0) / n)
        m4_d.append(_row_fourth_moment(E))
        m4_l.append(_row_fourth_moment(V))
    theta = 2.0                      # n / (sigma sqrt(n)) with sigma = 0.5 sqrt(n)
    law_lam = 0.5 * (theta + 1.0 / theta)
    law_overlap = 1.0 - 1.0 / theta ** 2
    assert abs(np.mean(lam_d) - law_lam) < 0.04
    assert abs(np.mean(lam_l) - law_lam) < 0.02
    assert abs(np.mean(ov_d) - law_overlap) < 0.04
    assert abs(np.mean(m4_d) - np.mean(m4_l)) < 0.03
    # both are delocalised: far from a factor concentrated on few rows
    assert np.mean(m4_d) < 1.3 and np.mean(m4_l) < 1.3
