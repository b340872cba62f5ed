"""GPU parity of the spectral truncation (Lanczos with full
reorthogonalisation) against oracle/spectral.py, through the C-ABI.

Laplacian: eigenvalues to 1e-10 relative and factor columns (same phase
convention) to 1e-7 of the largest entry, against numpy eigh of the dense
matrix; at full size against the cached host factor (ARPACK, stored FP32).
Phase synchronisation: the operator evaluates W in FP32 (accumulated in
FP64), so against the dense FP64 matrix of the same definition the bar is
1e-5 relative on eigenvalues and 1e-4 on the projector; at full size the
spiked-model law (eigenvalues sigma sqrt(n)(theta + 1/theta), squared overlap
with the planted phases 1 - 1/theta^2 for theta = 2) is checked."""
import numpy as np
import pytest

from oracle import spectral
from paper_2602_20376_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrqo_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20376_amd import lrqo

    lrqo.load()
    return lrqo


def _dev_graph(n, i, j, w):
    rp, col, ww = inputs.csr_adjacency(n, i, j, w)
    return (torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(),
            torch.from_numpy(ww).cuda() if ww is not None else None)


@pytest.mark.parametrize("n,m,r,weighted", [(1500, 9000, 4, True), (800, 3000, 3, False), (40, 120, 2, True)])
def test_laplacian_factor_parity(lrqo_mod, n, m, r, weighted):
    i, j = inputs.random_edges(n, m, 31 + n)
    w = np.random.default_rng(n).uniform(0.5, 2.0, m) if weighted else None
    V, res = lrqo_mod.laplacian_factor(*_dev_graph(n, i, j, w), r, tol=1e-12, max_iter=400)
    assert res.converged == 1
    L = spectral.laplacian_dense(n, (i, j, w if w is not None else np.ones(m)))
    lam, Vref = spectral.top_factor(L, r)
    assert np.allclose(np.array(res.eigenvalues[:r]), lam, rtol=1e-10, atol=0)
    Vg = V.cpu().numpy()
    scale = np.max(np.abs(Vref))
    assert np.max(np.abs(Vg - Vref)) <= 1e-7 * scale


def test_laplacian_factor_full_size(lrqo_mod):
    """Workload: the maxcut_er graph (n = 100,000, mean degree 10), r = 4,
    against the host factor of the same graph (ARPACK, tol 1e-10, FP32)."""
    inst = inputs.maxcut_er()
    i, j = inputs.maxcut_er_graph()
    V, res = lrqo_mod.laplacian_factor(*_dev_graph(inst.n, i, j, None), 4, tol=1e-11, max_iter=600)
    assert res.converged == 1
    Vh = inst.V.real
    lam_h = np.sum(Vh ** 2, axis=0)
    assert np.allclose(np.array(res.eigenvalues[:4]), lam_h, rtol=1e-6)
    Vg = V.cpu().numpy()
    assert np.max(np.abs(Vg.imag)) <= 1e-9 * np.max(np.abs(Vg.real))
    assert np.max(np.abs(Vg.real - Vh)) <= 1e-5 * np.max(np.abs(Vh))


def test_phase_sync_factor_parity(lrqo_mod):
    n, p, seed = 500, 3, 4242
    rng = np.random.default_rng(8)
    U = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, (n, p)))
    sigma = 0.5 * np.sqrt(n)
    V, res = lrqo_mod.phase_sync_factor(torch.from_numpy(U).cuda(), sigma, seed, 3, tol=1e-12, max_iter=200)
    assert res.converged == 1
    lam, Vref = spectral.top_factor(spectral.phase_sync_matrix(U, sigma, seed), 3)
    assert np.allclose(np.array(res.eigenvalues[:3]), lam, rtol=1e-5, atol=0)
    Vg = V.cpu().numpy()
    P = Vg @ Vg.conj().T
    Pref = Vref @ Vref.conj().T
    assert np.max(np.abs(P - Pref)) <= 1e-4 * np.max(np.abs(Pref))


def test_phase_sync_factor_full_size_law(lrqo_mod):
    """Workload: phase synchronisation at n = 262,144, p = r = 3,
    sigma = 0.5 sqrt(n), W matrix-free: the spiked-model law."""
    n, p = 262_144, 3
    rng = np.random.default_rng(5)
    U = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, (n, p)))
    sigma = 0.5 * np.sqrt(n)
    V, res = lrqo_mod.phase_sync_factor(torch.from_numpy(U).cuda(), sigma, 77, 3, tol=1e-8, max_iter=120)
    assert res.converged == 1
    lam = np.array(res.eigenvalues[:3]) / n
    assert np.all(np.abs(lam - 1.25) < 0.05), lam
    E = V.cpu().numpy() / np.sqrt(np.array(res.eigenvalues[:3]))[None, :]
    Uq, _ = np.linalg.qr(U)
    ov = np.linalg.svd(Uq.conj().T @ E, compute_uv=False) ** 2
    assert np.all(np.abs(ov - 0.75) < 0.05), ov


def test_spectral_rejects_bad_input(lrqo_mod):
    n = 10
    i, j = inputs.random_edges(n, 20, 5)
    rp, col, _ = inputs.csr_adjacency(n, i, j)
    bad = rp.copy()
    bad[-1] += 1
    with pytest.raises(lrqo_mod.LrqoError, match="row pointer"):
        lrqo_mod.laplacian_factor(torch.from_numpy(bad).cuda(), torch.from_numpy(col).cuda(), None, 2)
    with pytest.raises(lrqo_mod.LrqoError, match="r must be"):
        lrqo_mod.laplacian_factor(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), None, 9)


def test_phase_sync_true_factor_residual(lrqo_mod):
    """The phase-synchronisation workload factor (n = 262,144, r = 3) against
    the FP64 definition of Q = U U^H + sigma W on 32 sampled rows: each
    column satisfies (Q V_k)_i = lambda_k V_ik to 1e-4 relative (the operator
    evaluates W in FP32), the eigenvalues are the spiked-model ones to 5%,
    and the columns are orthogonal."""
    from oracle import spectral
    from paper_2602_20376_amd import phase_sync

    n = 262_144
    seed = inputs.instance_seed(5)
    V, lam, iters = phase_sync.true_factor(n, seed)
    U, sigma, w_seed = phase_sync.problem(n, seed)
    rows = np.sort(np.random.default_rng(1).choice(n, 32, replace=False))
    QV = spectral.phase_sync_rows_times(U, sigma, w_seed, rows, V)
    for k in range(3):
        res = np.linalg.norm(QV[:, k] - lam[k] * V[rows, k]) / (lam[k] * np.linalg.norm(V[rows, k]))
        assert res < 1e-4, (k, res)
    theta = n / (sigma * np.sqrt(n))
    assert np.all(np.abs(lam / (sigma * np.sqrt(n) * (theta + 1 / theta)) - 1) < 0.05), lam
    G = V.conj().T @ V
    assert np.max(np.abs(G - np.diag(np.diag(G)))) <= 1e-8 * np.max(np.abs(G))
