"""The allocation-free sampled entry point (lrqo_solve_sampled_noalloc)
against lrqo_solve_sampled_ex, through the C-ABI: two calls in a row (the
second smaller, so stale contents of the static scratch would show), each
equal to the allocating entry point's result bit for bit (winner, FP64
objective, FP32 objective, labels, every FP32 score), and a call whose
scratch exceeds the static array rejected before any device work."""
import ctypes

import numpy as np
import pytest

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


def _call(lrqo_mod, entry, V, n, r, K, S, seed, real, precision=0):
    lib = lrqo_mod.load()
    z = torch.empty(n, dtype=torch.uint8, device="cuda")
    f = torch.empty(S, dtype=torch.float32, device="cuda")
    opt = lrqo_mod.SampledOptions(1 if real else 0, precision, 0, 0, 0, ctypes.c_void_p(f.data_ptr()), None,
                                  None, 0, 0, None, None)
    res = lrqo_mod.SampledResult()
    lib.lrqo_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    st = getattr(lib, entry)(ctypes.c_void_p(V.data_ptr()), n, r, K, S, seed, ctypes.byref(opt),
                             ctypes.c_void_p(z.data_ptr()), ctypes.byref(res))
    assert st == 0, lrqo_mod.last_error()
    return res, z.cpu().numpy(), f.cpu().numpy()


def _same(a, b):
    ra, za, fa = a
    rb, zb, fb = b
    assert ra.best_index == rb.best_index
    assert ra.obj == rb.obj and ra.fp32_obj == rb.fp32_obj
    assert list(ra.best_c) == list(rb.best_c)
    assert np.array_equal(za, zb)
    assert np.array_equal(fa, fb)


@pytest.mark.parametrize("real,precision", [(True, 0), (False, 0), (True, 1)])
def test_noalloc_equals_allocating_entry(lrqo_mod, real, precision):
    shapes = [(20_000, 3, 3, 40_000), (3_000, 2, 5, 5_000)]      # second call smaller
    for n, r, K, S in shapes:
        V = inputs.random_V(n, r, 31 * n + r, real=real)
        Vd = torch.from_numpy(inputs.as_real_f32(V) if real else inputs.as_interleaved_f32(V)).cuda()
        seed = 7 + n
        a = _call(lrqo_mod, "lrqo_solve_sampled_noalloc", Vd, n, r, K, S, seed, real, precision)
        b = _call(lrqo_mod, "lrqo_solve_sampled_ex", Vd, n, r, K, S, seed, real, precision)
        _same(a, b)


def test_noalloc_sliced_then_small(lrqo_mod):
    """A launch with several row slices (partial sums in the scratch), then a
    one-slice call: the second must not see the first's partial sums."""
    for n, r, K, S in [(200_000, 4, 3, 65_536), (500, 4, 3, 300)]:
        V = inputs.random_V(n, r, 5 + n, real=True)
        Vd = torch.from_numpy(inputs.as_real_f32(V)).cuda()
        a = _call(lrqo_mod, "lrqo_solve_sampled_noalloc", Vd, n, r, K, S, 11, True)
        b = _call(lrqo_mod, "lrqo_solve_sampled_ex", Vd, n, r, K, S, 11, True)
        _same(a, b)


def test_noalloc_rejects_oversized_scratch(lrqo_mod):
    n, r, S = 1000, 2, 1 << 25     # 128 MiB of FP32 scores alone
    V = torch.zeros((n, r, 2), dtype=torch.float32, device="cuda")
    z = torch.empty(n, dtype=torch.uint8, device="cuda")
    res = lrqo_mod.SampledResult()
    st = lrqo_mod.load().lrqo_solve_sampled_noalloc(ctypes.c_void_p(V.data_ptr()), n, r, 3, S, 1, None,
                                                    ctypes.c_void_p(z.data_ptr()), ctypes.byref(res))
    assert st == -4 and "static array" in lrqo_mod.last_error()
