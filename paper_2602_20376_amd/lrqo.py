"""Python binding of liblrqo (ctypes).  Argument marshalling only: every step
of the solve runs in the library's HIP kernels.  PyTorch supplies device
memory and the current stream.

The library must be built (``python -m paper_2602_20376_amd.build``); if it is
missing, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LRQO_LIBRARY") or os.path.join(HERE, "liblrqo.so")

MAX_R = 8
MAX_K = 255
MAX_TOPK = 64

STATUS = {0: "LRQO_OK", -1: "LRQO_EINVAL", -2: "LRQO_ENOMEM", -3: "LRQO_EDEVICE",
          -4: "LRQO_ETOOBIG", -5: "LRQO_ENOTFINITE", -6: "LRQO_EDEGENERATE"}

# every entry point declared in include/lrqo.h
EXPORTS = ("lrqo_version", "lrqo_last_error", "lrqo_set_stream", "lrqo_shutdown",
           "lrqo_solve_sampled", "lrqo_solve_sampled_ex", "lrqo_solve_sampled_noalloc", "lrqo_solve_exact",
           "lrqo_solve_exact_ex", "lrqo_solve_batched", "lrqo_proposal_param_count",
           "lrqo_proposal_create", "lrqo_proposal_destroy", "lrqo_proposal_get_state",
           "lrqo_proposal_set_state", "lrqo_proposal_train_step", "lrqo_proposal_sample",
           "lrqo_proposal_frame", "lrqo_solve_nullvec", "lrqo_solve_rank1", "lrqo_graph_objective",
           "lrqo_refine_greedy", "lrqo_laplacian_factor", "lrqo_phase_sync_factor")


class LrqoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class SampledOptions(ctypes.Structure):
    _fields_ = [("real_v", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rescore_topk", ctypes.c_int32), ("instance", ctypes.c_uint32),
                ("first_index", ctypes.c_uint64), ("f_out", ctypes.c_void_p),
                ("directions", ctypes.c_void_p), ("dirs_out", ctypes.c_void_p),
                ("probe_count", ctypes.c_int32), ("probe_pad", ctypes.c_int32),
                ("probe", ctypes.c_void_p), ("probe_labels", ctypes.c_void_p)]


class SampledResult(ctypes.Structure):
    _fields_ = [("best_index", ctypes.c_int64), ("obj", ctypes.c_double),
                ("fp32_obj", ctypes.c_double), ("best_c", ctypes.c_double * (2 * MAX_R)),
                ("flagged_rows", ctypes.c_int64), ("device_ms", ctypes.c_float),
                ("score_ms", ctypes.c_float), ("rescored", ctypes.c_int32),
                ("slices", ctypes.c_int32)]


class ExactResult(ctypes.Structure):
    _fields_ = [("obj", ctypes.c_double), ("index_sets", ctypes.c_int64),
                ("rank_deficient", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("device_ms", ctypes.c_float), ("warning", ctypes.c_int32)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("real_v", ctypes.c_int32), ("rescore_topk", ctypes.c_int32),
                ("cpl", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("no_graph", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("best_index", ctypes.c_void_p)]


class BatchResult(ctypes.Structure):
    _fields_ = [("device_ms", ctypes.c_float), ("cpl", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("items", ctypes.c_int32),
                ("tuned_now", ctypes.c_int32), ("graph_captured_now", ctypes.c_int32),
                ("row_candidates", ctypes.c_int64)]


class Rank1Result(ctypes.Structure):
    _fields_ = [("obj", ctypes.c_double), ("sweep_obj", ctypes.c_double),
                ("best_cell", ctypes.c_int64), ("device_ms", ctypes.c_float),
                ("sort_passes", ctypes.c_int32)]


class EigsOptions(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class EigsResult(ctypes.Structure):
    _fields_ = [("eigenvalues", ctypes.c_double * MAX_R), ("residuals", ctypes.c_double * MAX_R),
                ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("device_ms", ctypes.c_float), ("pad", ctypes.c_int32)]


class Graph(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("nnz", ctypes.c_int64)]


class RefineOptions(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class RefineResult(ctypes.Structure):
    _fields_ = [("quad_before", ctypes.c_double), ("quad_after", ctypes.c_double),
                ("cut_before", ctypes.c_double), ("cut_after", ctypes.c_double),
                ("moves", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("device_ms", ctypes.c_float),
                ("launched", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liblrqo.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblrqo.so not found at {path}: build it with "
                           "`python -m paper_2602_20376_amd.build`")
    lib = ctypes.CDLL(path)
    i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.lrqo_version.restype = i32
    lib.lrqo_last_error.restype = ctypes.c_char_p
    lib.lrqo_set_stream.argtypes = [vp]
    lib.lrqo_set_stream.restype = i32
    lib.lrqo_shutdown.restype = i32
    lib.lrqo_solve_sampled.argtypes = [vp, i64, i32, i32, i64, u64, vp, ctypes.POINTER(ctypes.c_double)]
    lib.lrqo_solve_sampled.restype = i32
    lib.lrqo_solve_sampled_ex.argtypes = [vp, i64, i32, i32, i64, u64,
                                          ctypes.POINTER(SampledOptions), vp,
                                          ctypes.POINTER(SampledResult)]
    lib.lrqo_solve_sampled_ex.restype = i32
    lib.lrqo_solve_sampled_noalloc.argtypes = lib.lrqo_solve_sampled_ex.argtypes
    lib.lrqo_solve_sampled_noalloc.restype = i32
    lib.lrqo_solve_exact.argtypes = [vp, i64, i32, i32, vp, ctypes.POINTER(ctypes.c_double)]
    lib.lrqo_solve_exact.restype = i32
    lib.lrqo_solve_exact_ex.argtypes = [vp, i64, i32, i32, i64, vp, ctypes.POINTER(ExactResult)]
    lib.lrqo_solve_exact_ex.restype = i32
    lib.lrqo_solve_batched.argtypes = [vp, i32, vp, vp, vp, i32, i64, u64,
                                       ctypes.POINTER(BatchOptions), vp, vp,
                                       ctypes.POINTER(BatchResult)]
    lib.lrqo_solve_batched.restype = i32
    lib.lrqo_proposal_param_count.restype = i32
    lib.lrqo_proposal_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.lrqo_proposal_create.restype = i32
    lib.lrqo_proposal_destroy.argtypes = [vp]
    lib.lrqo_proposal_destroy.restype = i32
    lib.lrqo_proposal_get_state.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64)]
    lib.lrqo_proposal_get_state.restype = i32
    lib.lrqo_proposal_set_state.argtypes = [vp, vp, vp, vp, i64]
    lib.lrqo_proposal_set_state.restype = i32
    lib.lrqo_proposal_train_step.argtypes = [vp, vp, i32, vp, vp, vp, ctypes.c_float, i32,
                                             ctypes.POINTER(ctypes.c_double), vp]
    lib.lrqo_proposal_train_step.restype = i32
    lib.lrqo_proposal_sample.argtypes = [vp, vp, i64, i64, u64, u32, ctypes.c_float, vp]
    lib.lrqo_proposal_sample.restype = i32
    lib.lrqo_proposal_frame.argtypes = [vp, vp, i64, vp]
    lib.lrqo_solve_nullvec.restype = i32
    lib.lrqo_solve_nullvec.argtypes = [vp, i64, i32, i32, i64, u64, vp, ctypes.POINTER(ExactResult)]
    lib.lrqo_solve_rank1.restype = i32
    lib.lrqo_solve_rank1.argtypes = [vp, i64, i32, vp, ctypes.POINTER(Rank1Result)]
    lib.lrqo_graph_objective.restype = ctypes.c_int
    lib.lrqo_graph_objective.argtypes = [ctypes.POINTER(Graph), i32, vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    lib.lrqo_laplacian_factor.restype = i32
    lib.lrqo_laplacian_factor.argtypes = [ctypes.POINTER(Graph), i32, ctypes.POINTER(EigsOptions), vp,
                                          ctypes.POINTER(EigsResult)]
    lib.lrqo_phase_sync_factor.restype = i32
    lib.lrqo_phase_sync_factor.argtypes = [vp, i64, i32, ctypes.c_double, u64, i32, ctypes.POINTER(EigsOptions),
                                           vp, ctypes.POINTER(EigsResult)]
    lib.lrqo_refine_greedy.restype = ctypes.c_int
    lib.lrqo_refine_greedy.argtypes = [ctypes.POINTER(Graph), i32, vp, ctypes.POINTER(RefineOptions),
                                       ctypes.POINTER(RefineResult)]
    lib.lrqo_proposal_frame.restype = i32
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load().lrqo_last_error().decode(errors="replace")
        raise LrqoError(status, msg)


def last_error() -> str:
    return load().lrqo_last_error().decode(errors="replace")


def _bind_stream(torch):
    load().lrqo_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@dataclass
class SampledOutput:
    z: object            # torch uint8 (n,) on the device
    obj: float
    best_index: int
    best_c: list         # complex FP64 copy of the winner's FP32 direction
    fp32_obj: float
    device_ms: float
    score_ms: float
    rescored: int
    flagged_rows: int
    slices: int


def _factor_view(V, real):
    """Return (tensor holding the FP32 layout, n, r, real flag)."""
    import torch

    if not V.is_cuda:
        raise ValueError("V must be a device tensor")
    if V.dtype == torch.complex64:
        if V.dim() != 2:
            raise ValueError("complex V must be (n, r)")
        return torch.view_as_real(V.contiguous()).contiguous(), V.shape[0], V.shape[1], False
    if V.dtype == torch.float32:
        if real or V.dim() == 2:
            if V.dim() != 2:
                raise ValueError("real V must be (n, r)")
            return V.contiguous(), V.shape[0], V.shape[1], True
        if V.dim() == 3 and V.shape[2] == 2:
            return V.contiguous(), V.shape[0], V.shape[1], False
    raise ValueError("V must be complex64 (n, r), float32 (n, r) real, or float32 (n, r, 2)")


def solve_sampled(V, K: int, S: int, seed: int, *, real: bool | None = None, precision: int = 0,
                  topk: int = 64, instance: int = 0, first_index: int = 0, f_out=None,
                  z=None, directions=None, dirs_out=None, probe=None, probe_labels=None,
                  noalloc: bool = False) -> SampledOutput:
    """Best of S sampled directions (see lrqo_solve_sampled_ex).  dirs_out
    (float32 device (S, 2r)) receives the scored FP32 directions; probe (host
    ints) and probe_labels (uint16 device (len(probe), n)) the scorer's
    per-row labels of those candidates.  noalloc: through
    lrqo_solve_sampled_noalloc (static scratch, no allocation)."""
    import numpy as np
    import torch

    lib = load()
    Vf, n, r, is_real = _factor_view(V, real)
    if z is None:
        z = torch.empty(n, dtype=torch.uint8, device=V.device)
    pr = np.ascontiguousarray(probe if probe is not None else [], dtype=np.int64)
    if pr.size and (probe_labels is None or probe_labels.dtype != torch.uint16
                    or probe_labels.numel() != pr.size * n):
        raise ValueError("probe_labels must be a uint16 device tensor of len(probe) * n entries")
    opt = SampledOptions(1 if is_real else 0, int(precision), int(topk), int(instance),
                         int(first_index), ctypes.c_void_p(f_out.data_ptr() if f_out is not None else 0),
                         ctypes.c_void_p(directions.data_ptr() if directions is not None else 0),
                         ctypes.c_void_p(dirs_out.data_ptr() if dirs_out is not None else 0),
                         int(pr.size), 0, pr.ctypes.data_as(ctypes.c_void_p) if pr.size else None,
                         ctypes.c_void_p(probe_labels.data_ptr() if pr.size else 0))
    res = SampledResult()
    with torch.cuda.device(V.device):
        _bind_stream(torch)
        entry = lib.lrqo_solve_sampled_noalloc if noalloc else lib.lrqo_solve_sampled_ex
        _check(entry(ctypes.c_void_p(Vf.data_ptr()), n, r, int(K), int(S),
                                         int(seed) & (2**64 - 1), ctypes.byref(opt),
                                         ctypes.c_void_p(z.data_ptr()), ctypes.byref(res)))
    c = [complex(res.best_c[2 * j], res.best_c[2 * j + 1]) for j in range(r)]
    return SampledOutput(z, res.obj, res.best_index, c, res.fp32_obj, res.device_ms,
                         res.score_ms, res.rescored, res.flagged_rows, res.slices)


def solve_exact(V, K: int, *, max_sets: int = 0, z=None):
    """Exact solve (see lrqo_solve_exact_ex).  V: complex128 (n, r) device."""
    import torch

    lib = load()
    if not V.is_cuda or V.dtype != torch.complex128 or V.dim() != 2:
        raise ValueError("V must be a complex128 (n, r) device tensor")
    Vc = torch.view_as_real(V.contiguous()).contiguous()
    n, r = V.shape
    if z is None:
        z = torch.empty(n, dtype=torch.uint8, device=V.device)
    res = ExactResult()
    with torch.cuda.device(V.device):
        _bind_stream(torch)
        _check(lib.lrqo_solve_exact_ex(ctypes.c_void_p(Vc.data_ptr()), n, r, int(K), int(max_sets),
                                       ctypes.c_void_p(z.data_ptr()), ctypes.byref(res)))
    return z, res


def solve_nullvec(V, K: int, S: int, seed: int, *, z=None):
    """Null-vector randomized sampler (see lrqo_solve_nullvec).  V: complex128
    (n, r) device tensor.  Returns (labels, ExactResult)."""
    import torch

    lib = load()
    if not V.is_cuda or V.dtype != torch.complex128 or V.dim() != 2:
        raise ValueError("V must be a complex128 (n, r) device tensor")
    Vc = torch.view_as_real(V.contiguous()).contiguous()
    n, r = V.shape
    if z is None:
        z = torch.empty(n, dtype=torch.uint8, device=V.device)
    res = ExactResult()
    with torch.cuda.device(V.device):
        _bind_stream(torch)
        _check(lib.lrqo_solve_nullvec(ctypes.c_void_p(Vc.data_ptr()), n, r, int(K), int(S),
                                      int(seed) & (2**64 - 1), ctypes.c_void_p(z.data_ptr()),
                                      ctypes.byref(res)))
    return z, res


@dataclass
class BatchedOutput:
    z: object             # torch uint8 (sum n,) on the device, instance t at offset sum n[:t]
    obj: object           # numpy float64 (count,)
    best_index: object    # numpy int64 (count,)
    device_ms: float
    cpl: int
    blocks_per_cu: int
    items: int
    tuned_now: bool
    graph_captured_now: bool
    row_candidates: int


def solve_batched(Vcat, v_offset, n, r, K: int, S: int, seed: int, *, real: bool = False,
                  topk: int = 0, cpl: int = 0, blocks_per_cu: int = 0, graph: bool = True,
                  z=None) -> BatchedOutput:
    """Batched sampled solve (see lrqo_solve_batched).  Vcat: float32 device
    tensor holding every factor in the library layout; v_offset, n, r: host
    integer arrays."""
    import numpy as np
    import torch

    lib = load()
    if not Vcat.is_cuda or Vcat.dtype != torch.float32:
        raise ValueError("Vcat must be a float32 device tensor")
    voff = np.ascontiguousarray(v_offset, dtype=np.int64)
    nn = np.ascontiguousarray(n, dtype=np.int32)
    rr = np.ascontiguousarray(r, dtype=np.int32)
    count = int(nn.size)
    if z is None:
        z = torch.empty(int(nn.sum()), dtype=torch.uint8, device=Vcat.device)
    obj = np.zeros(count, dtype=np.float64)
    best = np.zeros(count, dtype=np.int64)
    opt = BatchOptions(1 if real else 0, int(topk), int(cpl), int(blocks_per_cu),
                       0 if graph else 1, 0, best.ctypes.data_as(ctypes.c_void_p))
    res = BatchResult()
    with torch.cuda.device(Vcat.device):
        _bind_stream(torch)
        _check(lib.lrqo_solve_batched(ctypes.c_void_p(Vcat.data_ptr()), count,
                                      voff.ctypes.data_as(ctypes.c_void_p),
                                      nn.ctypes.data_as(ctypes.c_void_p),
                                      rr.ctypes.data_as(ctypes.c_void_p), int(K), int(S),
                                      int(seed) & (2**64 - 1), ctypes.byref(opt),
                                      ctypes.c_void_p(z.data_ptr()),
                                      obj.ctypes.data_as(ctypes.c_void_p), ctypes.byref(res)))
    return BatchedOutput(z, obj, best, res.device_ms, res.cpl, res.blocks_per_cu, res.items,
                         bool(res.tuned_now), bool(res.graph_captured_now), res.row_candidates)


class Proposal:
    """Handle of the learned direction proposal (see lrqo_proposal_* in lrqo.h)."""

    def __init__(self, init_params, K: int):
        import numpy as np

        lib = load()
        self.nparam = int(lib.lrqo_proposal_param_count())
        init = np.ascontiguousarray(init_params, dtype=np.float64)
        if init.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        h = ctypes.c_void_p()
        _check(lib.lrqo_proposal_create(init.ctypes.data_as(ctypes.c_void_p), int(K), ctypes.byref(h)))
        self._h = h
        self.K = int(K)

    def close(self):
        if getattr(self, "_h", None):
            load().lrqo_proposal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_state(self):
        import numpy as np

        th = np.zeros(self.nparam, np.float32)
        m = np.zeros(self.nparam, np.float32)
        v = np.zeros(self.nparam, np.float32)
        step = ctypes.c_int64()
        _check(load().lrqo_proposal_get_state(self._h, th.ctypes.data_as(ctypes.c_void_p),
                                              m.ctypes.data_as(ctypes.c_void_p),
                                              v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(step)))
        return {"theta": th, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, state):
        import numpy as np

        th = np.ascontiguousarray(state["theta"], np.float32)
        m = np.ascontiguousarray(state["m"], np.float32)
        v = np.ascontiguousarray(state["v"], np.float32)
        _check(load().lrqo_proposal_set_state(self._h, th.ctypes.data_as(ctypes.c_void_p),
                                              m.ctypes.data_as(ctypes.c_void_p),
                                              v.ctypes.data_as(ctypes.c_void_p), int(state["step"])))

    def train_step(self, Vcat, v_offset, n, targets, lr: float, update: bool = True,
                   want_grad: bool = False):
        """Vcat: float32 device tensor of concatenated (n_t x 3) complex64
        factors; v_offset, n: host int64 arrays; targets: host (count, 6)."""
        import numpy as np
        import torch

        voff = np.ascontiguousarray(v_offset, np.int64)
        nn = np.ascontiguousarray(n, np.int64)
        tg = np.ascontiguousarray(targets, np.float32)
        loss = ctypes.c_double()
        g = np.zeros(self.nparam, np.float32) if want_grad else None
        with torch.cuda.device(Vcat.device):
            _bind_stream(torch)
            _check(load().lrqo_proposal_train_step(
                self._h, ctypes.c_void_p(Vcat.data_ptr()), int(nn.size),
                voff.ctypes.data_as(ctypes.c_void_p), nn.ctypes.data_as(ctypes.c_void_p),
                tg.ctypes.data_as(ctypes.c_void_p), float(lr), 1 if update else 0,
                ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p) if g is not None else None))
        return float(loss.value), g

    def sample(self, V, S: int, seed: int, instance: int = 0, uniform_fraction: float = 0.0,
               out=None):
        """(S, 6) float32 device tensor of proposed directions for V
        (complex64 (n, 3) device tensor)."""
        import torch

        Vf = torch.view_as_real(V.contiguous()).contiguous()
        if out is None:
            out = torch.empty((int(S), 6), dtype=torch.float32, device=V.device)
        with torch.cuda.device(V.device):
            _bind_stream(torch)
            _check(load().lrqo_proposal_sample(self._h, ctypes.c_void_p(Vf.data_ptr()), int(V.shape[0]),
                                               int(S), int(seed) & (2**64 - 1), int(instance),
                                               float(uniform_fraction), ctypes.c_void_p(out.data_ptr())))
        return out

    def frame(self, V):
        import numpy as np
        import torch

        Vf = torch.view_as_real(V.contiguous()).contiguous()
        out = np.zeros(19, np.float64)
        with torch.cuda.device(V.device):
            _bind_stream(torch)
            _check(load().lrqo_proposal_frame(self._h, ctypes.c_void_p(Vf.data_ptr()), int(V.shape[0]),
                                              out.ctypes.data_as(ctypes.c_void_p)))
        G = (out[0:18:2] + 1j * out[1:18:2]).reshape(3, 3)
        return G, float(out[18])


def solve_rank1(q, K: int, *, z=None):
    """Exact rank-1 sweep (see lrqo_solve_rank1).  q: complex128 (n,) device
    tensor.  Returns (labels, Rank1Result)."""
    import torch

    lib = load()
    if not (q.is_cuda and q.dtype == torch.complex128 and q.dim() == 1):
        raise ValueError("q must be a complex128 (n,) device tensor")
    qc = torch.view_as_real(q.contiguous()).contiguous()
    n = int(q.numel())
    if z is None:
        z = torch.empty(n, dtype=torch.uint8, device=q.device)
    res = Rank1Result()
    with torch.cuda.device(q.device):
        _bind_stream(torch)
        _check(lib.lrqo_solve_rank1(ctypes.c_void_p(qc.data_ptr()), n, int(K), ctypes.c_void_p(z.data_ptr()),
                                    ctypes.byref(res)))
    return z, res


def _graph(row_ptr, col, w):
    """lrqo_graph of device tensors row_ptr (int64 [n+1]), col (int32
    [nnz]) and w (float64 [nnz] or None)."""
    import torch

    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.dim() == 1):
        raise ValueError("row_ptr must be an int64 device vector")
    if not (col.is_cuda and col.dtype == torch.int32 and col.dim() == 1):
        raise ValueError("col must be an int32 device vector")
    if w is not None and not (w.is_cuda and w.dtype == torch.float64 and w.shape == col.shape):
        raise ValueError("w must be a float64 device vector shaped like col")
    return Graph(ctypes.c_void_p(row_ptr.data_ptr()),
                 ctypes.c_void_p(col.data_ptr() if col.numel() else 0),
                 ctypes.c_void_p(w.data_ptr() if w is not None and w.numel() else 0),
                 int(row_ptr.numel()) - 1, int(col.numel()))


def graph_objective(row_ptr, col, w, K: int, z):
    """(z^H L z, cut weight) of device labels z on the graph (see
    lrqo_graph_objective)."""
    import torch

    lib = load()
    g = _graph(row_ptr, col, w)
    if not (z.is_cuda and z.dtype == torch.uint8 and z.numel() == g.n):
        raise ValueError("z must be a uint8 device vector of n labels")
    q, c = ctypes.c_double(), ctypes.c_double()
    with torch.cuda.device(z.device):
        _bind_stream(torch)
        _check(lib.lrqo_graph_objective(ctypes.byref(g), int(K), ctypes.c_void_p(z.data_ptr()),
                                        ctypes.byref(q), ctypes.byref(c)))
    return q.value, c.value


def refine_greedy(row_ptr, col, w, K: int, z, *, max_rounds: int = 0, check_every: int = 0):
    """Greedy local search on z^H L z, labels z updated in place (see
    lrqo_refine_greedy).  Returns the RefineResult."""
    import torch

    lib = load()
    g = _graph(row_ptr, col, w)
    if not (z.is_cuda and z.dtype == torch.uint8 and z.numel() == g.n and z.is_contiguous()):
        raise ValueError("z must be a contiguous uint8 device vector of n labels")
    opt = RefineOptions(int(max_rounds), int(check_every))
    res = RefineResult()
    with torch.cuda.device(z.device):
        _bind_stream(torch)
        _check(lib.lrqo_refine_greedy(ctypes.byref(g), int(K), ctypes.c_void_p(z.data_ptr()),
                                      ctypes.byref(opt), ctypes.byref(res)))
    return res


def laplacian_factor(row_ptr, col, w, r: int, *, max_iter: int = 0, check_every: int = 0, tol: float = 0.0,
                     seed: int = 0):
    """Top-r factor of the graph Laplacian (see lrqo_laplacian_factor).
    Returns (V complex128 (n, r) device tensor, EigsResult)."""
    import torch

    lib = load()
    g = _graph(row_ptr, col, w)
    V = torch.empty((g.n, r), dtype=torch.complex128, device=row_ptr.device)
    opt = EigsOptions(int(max_iter), int(check_every), float(tol), int(seed) & (2**64 - 1))
    res = EigsResult()
    with torch.cuda.device(row_ptr.device):
        _bind_stream(torch)
        _check(lib.lrqo_laplacian_factor(ctypes.byref(g), int(r), ctypes.byref(opt), ctypes.c_void_p(V.data_ptr()),
                                         ctypes.byref(res)))
    return V, res


def phase_sync_factor(U, sigma: float, w_seed: int, r: int, *, max_iter: int = 0, check_every: int = 0,
                      tol: float = 0.0, seed: int = 0):
    """Top-r factor of U U^H + sigma W, W from w_seed (see
    lrqo_phase_sync_factor).  U: complex128 (n, p) device tensor."""
    import torch

    lib = load()
    if not (U.is_cuda and U.dtype == torch.complex128 and U.dim() == 2):
        raise ValueError("U must be a complex128 (n, p) device tensor")
    Uc = U.contiguous()
    n, p = U.shape
    V = torch.empty((n, r), dtype=torch.complex128, device=U.device)
    opt = EigsOptions(int(max_iter), int(check_every), float(tol), int(seed) & (2**64 - 1))
    res = EigsResult()
    with torch.cuda.device(U.device):
        _bind_stream(torch)
        _check(lib.lrqo_phase_sync_factor(ctypes.c_void_p(Uc.data_ptr()), int(n), int(p), float(sigma),
                                          int(w_seed) & (2**64 - 1), int(r), ctypes.byref(opt),
                                          ctypes.c_void_p(V.data_ptr()), ctypes.byref(res)))
    return V, res
