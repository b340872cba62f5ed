"""Parity bars shared by the GPU tests of the sampled, precision and batched
forms (the GPU path against the FP64 oracle, both fed the same inputs).

FP32 reach.  The scorer forms w_i = V_i c in FP32 from the FP32 direction it
reports (dirs_out).  Each of Re w_i, Im w_i is a sum of at most 2r = 16
products (K = 3 pre-scales c by sqrt(3), one more rounding), so
|w_i - w_i(FP64)| <= (2r + 2) u sum_j |V_ij||c_j| (1 + O(u)) with u = 2^-24;
the generic-K quantiser adds an FP32 atan2 and one multiply-add (a few units
in the last place of the phase, below |w| 2^-20 for K <= 255).  Rows whose
Euclidean distance to a decision-boundary line exceeds REACH = 64 u times
sum_j |V_ij||c_j| therefore get the FP64 label; rows inside it may take a
neighbouring label.

Labels.  For probed candidates the scorer writes the label it used for every
row; outside the reach they must equal the oracle's FP64 labels at the same
direction, bit for bit.

Scores.  The oracle returns, for each candidate, f at the FP64 labels and an
interval [lo, hi] holding f of every labelling that differs only on rows
within the reach.  The FP32 score must lie in [lo - A, hi + A], where A
allows for the FP32 accumulation of s = V^H z: each of the 2r real
components of s is a sum of n terms; recursive summation adds a rounding
error of at most u |partial sum| per addition.  Modelling these as
independent (uniform in [-u, u] |partial sum|, standard deviation u/sqrt(3)
per addition) with partial sums bounded in root-mean-square by
|s_comp| + ||V_col|| (the final value plus the spread of a random walk of the
column's terms), the error of a component has standard deviation at most
u sqrt(n/3) (|s_comp| + ||V_col||).  A takes ten of these standard
deviations on ||s||:  eps = 10 u sqrt(n/3) (||s|| + sqrt(2) ||V||_F) and
A = 2 ||s|| eps + eps^2.  The worst-case (non-statistical) bound
n u sum_i |x_i| is thousands of times larger at n = 10^5 and could not fail.
The largest observed |f32 - f| / A is returned so that the margin is visible.
"""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24
REACH = 64.0 * U32

# Precision form (K = 2, 3, 4): w from six BF16 products of three-part
# splits of V and c.  The split drops products of order 2^-24 (about 4 u per
# term); the MFMA's sum of at most 6C = 48 products is charged one FP32 ulp
# (2u) per addition; so |w - w(FP64)| <= (2 * 48 + 5) u sum_j |V_ij||c_j|.  A
# quantiser test is a linear form in (Re w, Im w) whose zero set is a
# boundary line; its error over the distance to that line is at most
# (1 + sqrt(3))/2 (K = 3, Re w pre-scaled) or sqrt(2) (K = 4), so the
# Euclidean distance within which a label can differ from the FP64 one is
# below 1.42 * 101 u < 256 u.  The generic-K precision form recomputes such
# rows in FP32 and stays within REACH.
REACH_PRECISION = 256.0 * U32


def fp32_exact(V):
    """The FP64 values of the FP32-stored factor (what the GPU reads)."""
    return np.asarray(V).astype(np.complex64).astype(np.complex128)


def dirs_complex(d, r):
    """(S, 2r) float32 (re, im) pairs -> (S, r) complex128."""
    d = np.asarray(d, dtype=np.float64).reshape(-1, 2 * r)
    return d[:, 0::2] + 1j * d[:, 1::2]


def accumulation_allowance(V, f):
    n = V.shape[0]
    vf = np.sqrt(np.sum(np.abs(V) ** 2))
    ns = np.sqrt(np.maximum(np.asarray(f, dtype=np.float64), 0.0))
    eps = 10.0 * U32 * np.sqrt(n / 3.0) * (ns + np.sqrt(2.0) * vf)
    return 2.0 * ns * eps + eps * eps


def check_scores(V, K, dirs, f32, reach=REACH, nthreads=0):
    """Every FP32 score inside the oracle's near-boundary interval plus the
    accumulation allowance.  Returns the oracle record and the largest
    observed ratio |f32 - f| / A (over candidates with no ambiguous row)."""
    V = fp32_exact(V)
    ref = oracle.score_dirs(V, K, dirs, reach=reach, nthreads=nthreads)
    f32 = np.asarray(f32, dtype=np.float64)
    A = accumulation_allowance(V, ref["f"])
    lo, hi = ref["lo"] - A, ref["hi"] + A
    bad = np.nonzero((f32 < lo) | (f32 > hi))[0]
    assert bad.size == 0, (int(bad.size), [(int(t), float(f32[t]), float(ref["lo"][t]), float(ref["hi"][t]),
                                            float(A[t])) for t in bad[:5]])
    clean = ref["nambig"] == 0
    ratio = float(np.max(np.abs(f32[clean] - ref["f"][clean]) / A[clean])) if np.any(clean) else 0.0
    ref["allowance"] = A
    ref["max_ratio"] = ratio
    return ref


def check_labels(V, K, c, labels, reach=REACH):
    """The scorer's labels at direction c (complex (r,)) equal the FP64
    decision rule on every row farther than `reach` (relative to
    sum_j |V_ij||c_j|) from a decision-boundary line.  Returns the number of
    rows compared and the number inside the reach."""
    V = fp32_exact(V)
    c = np.asarray(c, dtype=np.complex128)
    z_or, dist = oracle.labels(V, K, c)
    w = V @ c
    scale = np.abs(V) @ np.abs(c)
    near = np.abs(w) * np.sin(np.minimum(dist, np.pi / 2)) <= reach * scale
    lab = np.asarray(labels).astype(np.int64) & 0xFF
    far = ~near
    mism = np.nonzero(lab[far] != z_or[far])[0]
    assert mism.size == 0, (int(mism.size), np.nonzero(far)[0][mism[:5]].tolist())
    return int(far.sum()), int(near.sum())


def top_sets_agree(f32, f64, A, T=64):
    """The GPU's FP32 top T (f descending, index ascending) and the oracle's
    FP64 top T may differ only by near-ties at the cut: every candidate in
    one set and not the other has an FP64 value within 2A of the oracle's
    T-th value."""
    S = f32.size
    T = min(T, S)
    g = set(np.lexsort((np.arange(S), -np.asarray(f32, dtype=np.float64)))[:T].tolist())
    o_order = np.lexsort((np.arange(S), -np.asarray(f64)))
    o = set(o_order[:T].tolist())
    cut = f64[o_order[T - 1]]
    diff = sorted(g ^ o)
    for x in diff:
        assert abs(f64[x] - cut) <= 2.0 * A[x] + 1e-12 * abs(cut), (x, f64[x], cut, A[x])
    return len(diff)
