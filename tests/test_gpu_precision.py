"""GPU parity of the precision form (BF16 MFMA for V c, FP32 recompute of
rows inside the BF16 error margin, FP64 rescore) through the C-ABI.

Bar: the same as the FP32 sampled path against the FP64 oracle (labels at
the returned direction bit-exact away from boundaries; objective equal to the
oracle's f at that direction to 1e-12; within 1e-5 of the oracle's best of
the same S), plus: every per-candidate FP32 score of the precision form
equals the plain FP32 path's score within the FP32 summation bound, which a
row labelled from a wrong BF16 value (unflagged inside its margin) would
break by a whole label flip.
"""
import numpy as np
import pytest

from paper_2602_20376_amd import inputs
from test_gpu_sampled import _check_f32, _fp32_exact, _to_dev, check_result

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrqo_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20376_amd import lrqo

    lrqo.load()
    return lrqo


def _both(lrqo_mod, V, K, S, seed, real):
    Vd = _to_dev(V, real)
    f0 = torch.empty(S, dtype=torch.float32, device="cuda")
    f1 = torch.empty(S, dtype=torch.float32, device="cuda")
    a = lrqo_mod.solve_sampled(Vd, K, S, seed, real=real, f_out=f0)
    b = lrqo_mod.solve_sampled(Vd, K, S, seed, real=real, precision=1, f_out=f1)
    return a, b, f0.cpu().numpy().astype(np.float64), f1.cpu().numpy().astype(np.float64)


def _scores_agree(V, fa, fb, max_frac=0.005):
    """FP32 scores of the two paths within the FP32 summation bound; a few
    candidates may differ where the two FP32 label computations (different
    rounding of w) split a row that sits within ~1e-7 of a boundary."""
    n = V.shape[0]
    u = 2.0 ** -24
    scale = np.sum(np.sum(np.abs(V), axis=0) ** 2)
    tol = 8.0 * (n + 16) * u * scale + 1e-6 * np.abs(fa)
    bad = np.abs(fa - fb) > tol
    assert np.mean(bad) <= max_frac, (int(bad.sum()), fa.size)


CASES = [
    # n, r, K, S, real
    (12, 2, 3, 4096, False),
    (300, 3, 3, 3000, True),
    (257, 4, 3, 2049, True),
    (1000, 1, 5, 1500, False),
    (777, 2, 8, 2500, False),
    (513, 3, 16, 2000, False),
    (200, 4, 4, 1024, False),
    (400, 2, 2, 1000, True),
    (129, 2, 2, 999, True),
]


@pytest.mark.parametrize("n,r,K,S,real", CASES)
def test_precision_parity(lrqo_mod, n, r, K, S, real):
    seed = 9100 + 7 * n + r + K
    V = _fp32_exact(inputs.random_V(n, r, seed, real=real))
    a, b, fa, fb = _both(lrqo_mod, V, K, S, seed, real)
    check_result(V, K, S, seed, b, real=real, f32=fb)
    _scores_agree(V, fa, fb)
    assert abs(b.obj - a.obj) <= 1e-5 * a.obj
    assert b.flagged_rows >= 0


def test_precision_flags_rows(lrqo_mod):
    """Rows are flagged (the BF16 margin is not vacuous) and the count is a
    small fraction of all row-candidates."""
    V = _fp32_exact(inputs.random_V(4000, 3, 5))
    _, b, _, _ = _both(lrqo_mod, V, 3, 8192, 11, False)
    total = 4000 * 8192
    assert 0 < b.flagged_rows < 0.05 * total, b.flagged_rows


def test_precision_rejects_large_r(lrqo_mod):
    V = torch.zeros((10, 5), dtype=torch.complex64, device="cuda")
    with pytest.raises(lrqo_mod.LrqoError, match="r <= 4"):
        lrqo_mod.solve_sampled(V, 3, 16, 1, precision=1)


def test_maxcut_ppm_full_size(lrqo_mod):
    """Workload: 3-block planted partition, n = 1,000,000, r = 3, K = 3,
    S = 2^20.  Both forms reach the same FP64-rescored objective within
    1e-5; the oracle scores sampled directions and the winner one by one."""
    inst = inputs.maxcut_ppm()
    V = inst.V
    a, b, fa, fb = _both(lrqo_mod, V, inst.K, inst.S, inst.seed, True)
    assert abs(b.obj - a.obj) <= 1e-5 * a.obj, (a.obj, b.obj)
    rng = np.random.default_rng(3)
    sample = np.unique(np.concatenate([rng.choice(inst.S, 24, replace=False),
                                       np.argsort(fb)[-8:]]))
    check_result(V, inst.K, inst.S, inst.seed, b, real=True, f32=fb, full_oracle=False,
                 sample=sample)
    _scores_agree(_fp32_exact(V), fa[sample], fb[sample], max_frac=0.05)
