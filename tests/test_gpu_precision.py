"""GPU parity of the precision form through the C-ABI.  K = 2, 3, 4: both
products on BF16 MFMA (w from six products of three-part splits, labels
taken from it directly); other K: V c on BF16 MFMA with rows inside the BF16
error margin recomputed in FP32.  FP64 rescore in both.

Bar: the sampled path's bar against the FP64 oracle (returned labels, FP64
objective at the returned direction, best of the same S within 1e-5), and:
  * every score of the precision form lies inside the oracle's interval over
    the labels its reach leaves open (plus the accumulation allowance): a row
    labelled from a wrong value would leave it;
  * for probed candidates, every row outside the reach carries the FP64
    label (REACH_PRECISION for K = 2, 3, 4, whose labels come from the split
    product; REACH otherwise); where the form recomputes rows (other K),
    every row it did not recompute carries the FP32 scorer's label bit for
    bit, and it recomputes none for K = 2, 3, 4.
"""
import numpy as np
import pytest

import oracle
import parity_helpers as PH
from paper_2602_20376_amd import inputs
from test_gpu_sampled import _fp32_exact, _to_dev, check_result

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lrqo_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20376_amd import lrqo

    lrqo.load()
    return lrqo


def _both(lrqo_mod, V, K, S, seed, real, n_probes=8):
    """FP32 and precision-form solves of the same stream with scores,
    directions and the probed candidates' labels."""
    n, r = V.shape
    Vd = _to_dev(V, real)
    runs = []
    for prec in (0, 1):
        f = torch.empty(S, dtype=torch.float32, device="cuda")
        d = torch.empty((S, 2 * r), dtype=torch.float32, device="cuda")
        out = lrqo_mod.solve_sampled(Vd, K, S, seed, real=real, precision=prec, f_out=f, dirs_out=d)
        runs.append([out, f.cpu().numpy().astype(np.float64), PH.dirs_complex(d.cpu().numpy(), r)])
    a, b = runs
    assert np.array_equal(a[2], b[2]), "both forms score the same directions"
    rng = np.random.default_rng(S + 7 * n)
    probe = sorted(set(rng.choice(S, min(S, n_probes), replace=False).tolist())
                   | {a[0].best_index, b[0].best_index} | set(np.argsort(b[1])[-4:].tolist()))[:64]
    labs = []
    for prec, run in ((0, a), (1, b)):
        lab = torch.empty((len(probe), n), dtype=torch.uint16, device="cuda")
        f = torch.empty(S, dtype=torch.float32, device="cuda")
        lrqo_mod.solve_sampled(Vd, K, S, seed, real=real, precision=prec, f_out=f, probe=probe, probe_labels=lab)
        assert np.array_equal(f.cpu().numpy().astype(np.float64), run[1]), "probed launch scores differently"
        labs.append(lab.cpu().numpy())
    return a, b, probe, labs


MFMA_K = (2, 3, 4)


def reach_of(K):
    return PH.REACH_PRECISION if K in MFMA_K else PH.REACH


def _check_probes(V, K, dirs, probe, lab32, lab16):
    """All rows outside the form's reach carry the FP64 label (both forms);
    where the precision form recomputes rows, its unflagged rows carry the
    FP32 label.  Returns (rows compared with FP32, rows recomputed, rows whose
    label differs from FP32's)."""
    V = _fp32_exact(V)
    flagged = 0
    compared = 0
    differ = 0
    for t, pos in enumerate(probe):
        fl = (lab16[t] & 0x100) != 0
        flagged += int(fl.sum())
        same = (lab16[t] & 0xFF) == (lab32[t] & 0xFF)
        differ += int((~same).sum())
        if K in MFMA_K:
            assert not np.any(fl), "the K = 2, 3, 4 form recomputes no rows"
        else:
            assert np.all(same[~fl]), (pos, np.nonzero(~same & ~fl)[0][:5].tolist())
            compared += int((~fl).sum())
        PH.check_labels(V, K, dirs[pos], lab16[t], reach=reach_of(K))
        PH.check_labels(V, K, dirs[pos], lab32[t])
    return compared, flagged, differ


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
    (3000, 3, 3, 2000, False),
    (2500, 4, 5, 1500, False),
    (600, 3, 4, 1100, True),
    (2100, 4, 2, 700, False),
    (5000, 1, 3, 300, True),
]


@pytest.mark.parametrize("n,r,K,S,real", CASES)
def test_precision_parity(lrqo_mod, n, r, K, S, real):
    seed = 9100 + 7 * n + r + K
    V = _fp32_exact(inputs.random_V(n, r, seed, real=real))
    a, b, probe, (l32, l16) = _both(lrqo_mod, V, K, S, seed, real)
    (oa, fa, dirs), (ob, fb, _) = a, b
    check_result(V, K, S, seed, ob, real=real, f32=fb, dirs=dirs, reach=reach_of(K))
    PH.check_scores(V, K, dirs, fa)
    _check_probes(V, K, dirs, probe, l32, l16)
    assert abs(ob.obj - oa.obj) <= 1e-5 * oa.obj
    assert ob.flagged_rows >= 0 and (K not in MFMA_K or ob.flagged_rows == 0)


def test_precision_flags_rows(lrqo_mod):
    """Generic K: rows are flagged (the BF16 margin is not vacuous) and the
    count is a small fraction of all row-candidates; K = 3 flags none."""
    V = _fp32_exact(inputs.random_V(4000, 3, 5))
    a, b, probe, (l32, l16) = _both(lrqo_mod, V, 5, 8192, 11, False)
    total = 4000 * 8192
    assert 0 < b[0].flagged_rows < 0.05 * total, b[0].flagged_rows
    _check_probes(V, 5, a[2], probe, l32, l16)
    a, b, probe, (l32, l16) = _both(lrqo_mod, V, 3, 8192, 11, False)
    assert b[0].flagged_rows == 0
    _check_probes(V, 3, a[2], probe, l32, l16)


@pytest.mark.parametrize("K,real", [(3, True), (3, False), (4, True), (2, False)])
def test_precision_zero_and_repeated_rows(lrqo_mod, K, real):
    """Exactly zero rows (never flagged: they add nothing to s whatever their
    label) and repeated rows, in both forms."""
    V = _fp32_exact(inputs.random_V(700, 2, 41 + K, real=real))
    V[::7] = 0
    V[1::7] = V[2::7]
    a, b, probe, (l32, l16) = _both(lrqo_mod, V, K, 1500, 43, real)
    (oa, fa, dirs), (ob, fb, _) = a, b
    check_result(V, K, 1500, 43, ob, real=real, f32=fb, dirs=dirs, reach=reach_of(K))
    PH.check_scores(V, K, dirs, fb, reach=reach_of(K))
    _check_probes(V, K, dirs, probe, l32, l16)


@pytest.mark.parametrize("K", [3, 4, 5])
def test_precision_ranges_directions_and_determinism(lrqo_mod, K):
    """The precision form over disjoint index ranges merges to the whole
    range; an explicit direction list (the stream's own directions) scores
    bit-identically to the stream; repeated calls are bit-identical."""
    V = _fp32_exact(inputs.random_V(700, 3, 71 + K))
    Vd = _to_dev(V, False)
    f_whole = torch.empty(4000, dtype=torch.float32, device="cuda")
    d_whole = torch.empty((4000, 6), dtype=torch.float32, device="cuda")
    whole = lrqo_mod.solve_sampled(Vd, K, 4000, 9, precision=1, f_out=f_whole, dirs_out=d_whole)
    parts = [lrqo_mod.solve_sampled(Vd, K, 1000, 9, precision=1, first_index=1000 * q) for q in range(4)]
    best = max(parts, key=lambda o: (o.obj, -o.best_index))
    assert best.best_index == whole.best_index and best.obj == whole.obj
    check_result(V, K, 1000, 9, parts[1], first=1000, reach=reach_of(K))
    f_list = torch.empty(4000, dtype=torch.float32, device="cuda")
    listed = lrqo_mod.solve_sampled(Vd, K, 4000, 9, precision=1, f_out=f_list, directions=d_whole)
    assert torch.equal(f_list, f_whole) and listed.best_index == whole.best_index and listed.obj == whole.obj
    again = torch.empty(4000, dtype=torch.float32, device="cuda")
    rep = lrqo_mod.solve_sampled(Vd, K, 4000, 9, precision=1, f_out=again)
    assert torch.equal(again, f_whole) and torch.equal(rep.z, whole.z)


def test_precision_rejects_large_r(lrqo_mod):
    V = torch.zeros((10, 5), dtype=torch.complex64, device="cuda")
    with pytest.raises(lrqo_mod.LrqoError, match="r <= 4"):
        lrqo_mod.solve_sampled(V, 3, 16, 1, precision=1)


def test_maxcut_ppm_full_size(lrqo_mod):
    """Workload: 3-block planted partition, n = 1,000,000, r = 3, K = 3,
    S = 2^20, both forms in the benchmark's launch configuration.  Both reach
    the same FP64-rescored objective within 1e-5; the oracle scores the
    contiguous block of the first 8,192 directions (both forms' FP32 scores
    inside its intervals; the FP64 stream's best over the block); probed
    candidates row by row."""
    inst = inputs.maxcut_ppm()
    V = _fp32_exact(inst.V)
    a, b, probe, (l32, l16) = _both(lrqo_mod, V, inst.K, inst.S, inst.seed, True)
    (oa, fa, dirs), (ob, fb, _) = a, b
    assert abs(ob.obj - oa.obj) <= 1e-5 * oa.obj, (oa.obj, ob.obj)
    blk = np.arange(8192)
    ref, stats = check_result(V, inst.K, inst.S, inst.seed, ob, real=True, f32=fb, dirs=dirs, full_oracle=False,
                              block=blk, reach=reach_of(inst.K))
    sa = PH.check_scores(V, inst.K, dirs[blk], fa[blk])
    compared, flagged, differ = _check_probes(V, inst.K, dirs, probe, l32, l16)
    print(f"maxcut_ppm: fp32 {oa.obj!r} bf16 {ob.obj!r} block oracle {ref['best_f']!r} "
          f"max |f-f64|/A fp32 {sa['max_ratio']:.3g} bf16 {stats['max_ratio']:.3g}; probed rows "
          f"{len(probe) * inst.n}, labels differing from FP32 {differ}", flush=True)
