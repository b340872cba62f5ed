"""GPU parity of the exact rank-1 phase sweep (Alg. 1) against the FP64
reference in oracle/rank1.py, through the C-ABI.

The sweep's cells are scored by FP64 prefix sums in another order than the
reference's sequential accumulation, so cell values agree to the FP64
summation bound 4 (n + 64) 2^-53 (sum |q_i|)^2 (floored at 1e-12 relative).
Where the reference's best cell beats every other cell by more than that
bound, the chosen cell and the labels are bit-exact; otherwise the returned
labels must reach the reference's optimum within the bound.  The returned
objective is the FP64 value of the returned labels."""
import numpy as np
import pytest

import oracle
from oracle import rank1
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


def _check(lrqo_mod, q, K):
    q = np.asarray(q, dtype=np.complex128)
    n = q.size
    z, res = lrqo_mod.solve_rank1(torch.from_numpy(q).cuda(), K)
    z = z.cpu().numpy()
    f, order, k0 = rank1.rank1_cells(q, K)
    fmax = f.max()
    tol = max(1e-12 * fmax, 4.0 * (n + 64) * 2.0 ** -53 * np.sum(np.abs(q)) ** 2)
    obj_z = oracle.objective(q[:, None], K, z)
    assert abs(res.obj - obj_z) <= tol
    assert res.obj >= fmax - tol
    assert abs(res.sweep_obj - f[res.best_cell]) <= tol
    best = int(np.argmax(f))
    others = np.delete(f, best)
    if others.size == 0 or fmax - others.max() > 2 * tol:
        assert res.best_cell == best
        zo = k0.copy()
        zo[order[:best]] += 1
        assert np.array_equal(z, np.mod(zo, K).astype(np.uint8))
    return res


CASES = [(1, 3), (2, 2), (7, 5), (100, 3), (2047, 4), (2048, 8), (2049, 16), (5000, 255),
         (100_000, 3), (65_537, 7)]


@pytest.mark.parametrize("n,K", CASES)
def test_rank1_parity_random(lrqo_mod, n, K):
    q = inputs.random_V(n, 1, 500 + n + K)[:, 0]
    _check(lrqo_mod, q, K)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_rank1_real_vector_ties(lrqo_mod, K):
    """Real q: every boundary point is one of two values, so the order of
    equal points (coordinate order) decides the cells."""
    q = np.random.default_rng(K).standard_normal(3000).astype(np.complex128)
    q[::17] = 0.0
    res = _check(lrqo_mod, q, K)
    if K == 2:
        assert abs(res.obj - np.sum(np.abs(q)) ** 2) <= 1e-10 * res.obj


def _clustered(groups, size, seed, K):
    """Groups of boundary points 1e-13 apart in angle: distinct FP64 keys
    that fall in one 2^-32 step of the fixed-point image, with magnitudes
    and coordinate order shuffled so that coordinate order is not key
    order inside a group."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-np.pi, np.pi, groups)[:, None] + 1e-13 * np.arange(size)[None, :]
    q = rng.uniform(0.5, 2.0, theta.shape) * np.exp(1j * theta)
    return rng.permutation(q.ravel())


@pytest.mark.parametrize("K", [3, 5])
def test_rank1_close_points_sorted_in_place(lrqo_mod, K):
    """Runs of at most 16 equal images with distinct keys: put in key order
    after the image sort, without the 64-bit sort."""
    q = _clustered(6, 12, 11 + K, K)
    res = _check(lrqo_mod, q, K)
    assert res.sort_passes == 4


@pytest.mark.parametrize("K", [3, 5])
def test_rank1_long_close_runs_take_the_exact_sort(lrqo_mod, K):
    """A run of more than 16 equal images with distinct keys: the host sorts
    the exact 64-bit keys instead."""
    q = np.concatenate([_clustered(3, 40, 21 + K, K), inputs.random_V(500, 1, 7)[:, 0]])
    res = _check(lrqo_mod, q, K)
    assert res.sort_passes > 4


@pytest.mark.parametrize("size,exact_sort", [(16, False), (17, True)])
def test_rank1_run_length_limit(lrqo_mod, size, exact_sort):
    """The in-place limit: a run of 16 equal images with distinct keys is
    sorted in place, one of 17 sends the call to the exact-key sort."""
    q = np.concatenate([_clustered(1, size, 31 + size, 3), inputs.random_V(200, 1, 9)[:, 0]])
    res = _check(lrqo_mod, q, 3)
    assert (res.sort_passes > 4) == exact_sort


def test_rank1_equals_the_exact_path(lrqo_mod):
    q = inputs.random_V(300, 1, 42)
    z, res = lrqo_mod.solve_rank1(torch.from_numpy(q[:, 0]).cuda(), 3)
    _, ex = lrqo_mod.solve_exact(torch.from_numpy(q).cuda(), 3)
    assert abs(res.obj - ex.obj) <= 1e-11 * ex.obj


def test_rank1_rejects_bad_input(lrqo_mod):
    q = torch.zeros(10, dtype=torch.complex128, device="cuda")
    q[3] = complex(float("nan"), 0.0)
    with pytest.raises(lrqo_mod.LrqoError, match="NaN"):
        lrqo_mod.solve_rank1(q, 3)
    with pytest.raises(lrqo_mod.LrqoError, match="K must be"):
        lrqo_mod.solve_rank1(torch.ones(4, dtype=torch.complex128, device="cuda"), 1)


def test_two_eigenvector_rounding_full_size(lrqo_mod):
    """Workload: the 3-block planted partition (n = 10^6), K = 3, with
    q = v1 + i v2 from the two leading Laplacian eigenvectors (the columns
    of the factor, normalised): the two-eigenvector rounding."""
    inst = inputs.maxcut_ppm()
    V = inst.V.real
    q = V[:, 0] / np.linalg.norm(V[:, 0]) + 1j * V[:, 1] / np.linalg.norm(V[:, 1])
    _check(lrqo_mod, q, 3)
