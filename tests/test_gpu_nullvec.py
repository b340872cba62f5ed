"""GPU parity of the null-vector randomized sampler against oracle/nullvec.py,
through the C-ABI.

Complex factors are in general position: the draw statistics (valid draws,
rank-deficient draws, scored label vectors) are equal, the objective agrees
to 1e-12 relative and the labels reach it.  Real factors are not in general
position (a vertex cut out by two rows of one boundary index has every row on
a boundary line), so there only the draw statistics and the value of the
returned labels are compared."""
import numpy as np
import pytest

import oracle
from oracle import nullvec
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


CASES = [(12, 2, 3, 3000, 5), (30, 2, 4, 2000, 6), (20, 3, 3, 1200, 7), (40, 1, 5, 600, 8),
         (10, 4, 3, 400, 9), (25, 2, 8, 1000, 10),
         # r = 5 .. 8: draws of 9 to 15 rows, vertices solved by sixteen lanes
         (20, 5, 3, 300, 11), (12, 6, 4, 300, 12), (60, 7, 2, 200, 13), (50, 8, 2, 150, 14)]


@pytest.mark.parametrize("n,r,K,S,seed", CASES)
def test_nullvec_parity_complex(lrqo_mod, n, r, K, S, seed):
    V = inputs.random_V(n, r, 900 + n + r + K)
    z, res = lrqo_mod.solve_nullvec(torch.from_numpy(V).cuda(), K, S, seed)
    ref = nullvec.nullvec_sampler(V, K, S, seed)
    assert (res.index_sets, res.rank_deficient, res.candidates) == (ref["valid"], ref["rank_deficient"],
                                                                    ref["candidates"])
    assert abs(res.obj - ref["opt"]) <= 1e-12 * ref["opt"]
    zh = z.cpu().numpy()
    assert abs(oracle.objective(V, K, zh) - res.obj) <= 1e-12 * res.obj


def test_nullvec_real_factor_statistics(lrqo_mod):
    V = inputs.random_V(300, 2, 55, real=True)
    z, res = lrqo_mod.solve_nullvec(torch.from_numpy(V).cuda(), 3, 4000, 3)
    ref = nullvec.nullvec_sampler(V, 3, 4000, 3, score=False)
    assert (res.index_sets, res.rank_deficient) == (ref["valid"], ref["rank_deficient"])
    assert abs(oracle.objective(V, 3, z.cpu().numpy()) - res.obj) <= 1e-12 * res.obj


@pytest.mark.parametrize("r", [2, 4])
def test_nullvec_full_size_statistics(lrqo_mod, r):
    """The samplers comparison's configuration: the maxcut_er factor
    (n = 10^5, real, K = 3), its leading r columns, S = 65,536 draws.  The
    oracle counts the valid and the rank-deficient draws (no scoring at this
    size); the returned objective is the FP64 value of the returned labels."""
    inst = inputs.maxcut_er()
    V = np.ascontiguousarray(inst.V[:, :r])
    z, res = lrqo_mod.solve_nullvec(torch.from_numpy(V).cuda(), inst.K, inst.S, inst.seed)
    ref = nullvec.nullvec_sampler(V, inst.K, inst.S, inst.seed, score=False)
    assert (res.index_sets, res.rank_deficient) == (ref["valid"], ref["rank_deficient"])
    assert abs(oracle.objective(V, inst.K, z.cpu().numpy()) - res.obj) <= 1e-12 * res.obj


def test_nullvec_rejects_bad_arguments(lrqo_mod):
    V = torch.from_numpy(inputs.random_V(10, 2, 1)).cuda()
    with pytest.raises(lrqo_mod.LrqoError, match="S must be"):
        lrqo_mod.solve_nullvec(V, 3, 0, 1)
    with pytest.raises(lrqo_mod.LrqoError, match="no feasible draw"):
        lrqo_mod.solve_nullvec(torch.from_numpy(inputs.random_V(2, 2, 1)).cuda(), 2, 1, 5)
