"""FP64 CPU oracle for the low-rank K-ary quadratic maximizer.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the GPU path (no common kernels, headers, helpers or
tables); the only thing both sides read is the seeded input generator module.

Contents
  * ``lrqo_oracle.c`` (built into ``liblrqo_oracle.so`` with gcc, FP64, no
    fast-math): Philox4x32-10 direction stream, the decision rule
    (Sec. 3, eq. decision_rule), the objective ||V^H z||^2 (Sec. 2.2,
    eq. quad_max-norm) and best-of-S over sampled directions (Sec. 4.2,
    eq. def_f).  Wrapped below.
  * ``exact.py``: Alg. 2 (exact rank-r enumeration of arrangement vertices,
    Sec. 3) with the ambiguity handling read structurally.
  * ``brute.py``: the definition itself, max over all K^n assignments.
  * ``rank1.py``: Alg. 1 (exact rank-1 sweep, Sec. 2.5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lrqo_oracle.c")
_SO = os.path.join(_HERE, "liblrqo_oracle.so")
# a sanitized copy (AddressSanitizer + UndefinedBehaviorSanitizer) for the
# sanitizer tests; LRQO_ORACLE_LIBRARY selects it in their child process
_SO_SAN = os.path.join(os.path.dirname(_HERE), "_build_san", "liblrqo_oracle.so")
_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    out = _SO_SAN if sanitize else _SO
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(out), exist_ok=True)
        tmp = out + f".tmp{os.getpid()}"
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-g"] if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-Wall", *san, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LRQO_ORACLE_LIBRARY")
    if not path:
        path = build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    d, i32, i64, u32, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
    lib.oracle_uniform.argtypes = [u32]
    lib.oracle_uniform.restype = d
    lib.oracle_direction.argtypes = [u64, u64, u32, ctypes.c_int, vp]
    lib.oracle_label.argtypes = [d, d, ctypes.c_int]
    lib.oracle_label.restype = ctypes.c_int
    lib.oracle_boundary_distance.argtypes = [d, d, ctypes.c_int]
    lib.oracle_boundary_distance.restype = d
    lib.oracle_labels.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.oracle_objective.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp]
    lib.oracle_objective.restype = d
    lib.oracle_f_of_c.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.oracle_f_of_c.restype = d
    lib.oracle_sampled.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, u64, u32, u64, i64,
                                   ctypes.c_int, vp, vp, vp, vp]
    lib.oracle_sampled.restype = ctypes.c_int
    lib.oracle_score_dirs.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp, i64, d, ctypes.c_int,
                                      vp, vp, vp, vp]
    lib.oracle_score_dirs.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _V64(V: np.ndarray) -> np.ndarray:
    """(n, r) complex -> contiguous complex128 (interleaved re, im)."""
    V = np.ascontiguousarray(np.asarray(V, dtype=np.complex128))
    assert V.ndim == 2 and V.shape[1] <= 8
    return V


# ---------------------------------------------------------------- wrappers

def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(x: int) -> float:
    return _load().oracle_uniform(int(x) & 0xFFFFFFFF)


def direction(seed: int, s: int, r: int, instance: int = 0) -> np.ndarray:
    """Direction c_s in C^r of the stream (seed, instance)."""
    out = np.zeros(2 * r, dtype=np.float64)
    _load().oracle_direction(int(seed) & (2**64 - 1), int(s), int(instance), int(r), _ptr(out))
    return out[0::2] + 1j * out[1::2]


def _c_interleaved(c) -> np.ndarray:
    c = np.asarray(c, dtype=np.complex128)
    out = np.empty(2 * c.size, dtype=np.float64)
    out[0::2] = c.real
    out[1::2] = c.imag
    return out


def label(w: complex, K: int) -> int:
    return _load().oracle_label(float(np.real(w)), float(np.imag(w)), int(K))


def boundary_distance(w: complex, K: int) -> float:
    return _load().oracle_boundary_distance(float(np.real(w)), float(np.imag(w)), int(K))


def labels(V, K: int, c):
    """Decision-rule labels z(c) (uint8) and per-row boundary distance (rad)."""
    V = _V64(V)
    n, r = V.shape
    cc = _c_interleaved(c)
    z = np.zeros(n, dtype=np.uint8)
    dist = np.zeros(n, dtype=np.float64)
    _load().oracle_labels(_ptr(V), n, r, int(K), _ptr(cc), _ptr(z), _ptr(dist))
    return z, dist


def objective(V, K: int, z) -> float:
    """||V^H z||^2 for labels z (z_i = exp(2 pi i z_i / K))."""
    V = _V64(V)
    n, r = V.shape
    zz = np.ascontiguousarray(np.asarray(z, dtype=np.uint8))
    assert zz.size == n
    return _load().oracle_objective(_ptr(V), n, r, int(K), _ptr(zz))


def f_of_c(V, K: int, c):
    """(f(c), min normalised row margin) for one direction c."""
    V = _V64(V)
    n, r = V.shape
    cc = _c_interleaved(c)
    mm = np.zeros(1, dtype=np.float64)
    f = _load().oracle_f_of_c(_ptr(V), n, r, int(K), _ptr(cc), _ptr(mm))
    return f, float(mm[0])


def sampled(V, K: int, S: int, seed: int, instance: int = 0, s0: int = 0, nthreads: int = 0,
            want_f: bool = True, want_margin: bool = False) -> dict:
    """Best of directions s0..s0+S-1 of the stream (seed, instance)."""
    V = _V64(V)
    n, r = V.shape
    f = np.zeros(S, dtype=np.float64) if want_f else None
    m = np.zeros(S, dtype=np.float64) if want_margin else None
    best_s = np.zeros(1, dtype=np.int64)
    best_f = np.zeros(1, dtype=np.float64)
    used = _load().oracle_sampled(_ptr(V), n, r, int(K), int(seed) & (2**64 - 1), int(instance),
                                  int(s0), int(S), int(nthreads),
                                  _ptr(f) if f is not None else None,
                                  _ptr(m) if m is not None else None,
                                  _ptr(best_s), _ptr(best_f))
    return {"f": f, "margin": m, "best_s": int(best_s[0]), "best_f": float(best_f[0]),
            "threads": int(used)}


def score_dirs(V, K: int, dirs, reach: float, nthreads: int = 0) -> dict:
    """f at each given direction (rows of `dirs`, complex (S, r)) with the
    interval [lo, hi] holding every labelling that differs from the FP64
    decision rule only on rows within `reach` (relative to sum_j |V_ij||c_j|)
    of a decision-boundary line; `nambig` counts those rows."""
    V = _V64(V)
    n, r = V.shape
    D = np.ascontiguousarray(np.asarray(dirs, dtype=np.complex128).reshape(-1, r))
    S = D.shape[0]
    dd = np.empty((S, 2 * r), dtype=np.float64)
    dd[:, 0::2] = D.real
    dd[:, 1::2] = D.imag
    f = np.zeros(S)
    lo = np.zeros(S)
    hi = np.zeros(S)
    na = np.zeros(S, dtype=np.int64)
    used = _load().oracle_score_dirs(_ptr(V), n, r, int(K), _ptr(dd), S, float(reach), int(nthreads),
                                     _ptr(f), _ptr(lo), _ptr(hi), _ptr(na))
    return {"f": f, "lo": lo, "hi": hi, "nambig": na, "threads": int(used)}


def canonical(z, K: int, real_V: bool = False) -> np.ndarray:
    """Canonical representative of the symmetry orbit of a labelling.

    A global rotation by a K-th root leaves the objective unchanged
    (Lemma phase_equiv), so labels are shifted to make k_0 = 0; for a real V,
    conjugation (k -> -k mod K) is a symmetry too and the lexicographically
    smaller of the two shifted forms is taken.
    """
    z = np.asarray(z, dtype=np.int64)
    a = (z - z[0]) % K
    if not real_V:
        return a.astype(np.uint8)
    b = (-z - (-z[0])) % K
    for x, y in zip(a, b):
        if x != y:
            return (a if x < y else b).astype(np.uint8)
    return a.astype(np.uint8)
