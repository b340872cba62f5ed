"""Seeded synthetic inputs for the low-rank K-ary quadratic maximizer.

This module produces the rank-r factor V (and nothing else) for each workload
shape.  It holds none of the maximizer's arithmetic: no decision rule, no
objective, no candidate generation.  Both the CPU oracle and the GPU path read
their inputs from here, so that parity runs compare the two on identical data.

Workload shapes (instance seed = 1000 + workload number, direction seed =
2000 + workload number):

1. ``exact_small``   V in C^{12x2}, entries N_C(0,1) (real and imaginary parts
   each N(0, 1/2), the normalisation of the complex Gaussian in Sec. 4.1), FP64.
2. ``maxcut_er``     Erdos-Renyi graph, n = 100,000, mean degree 10; Laplacian
   L = D - A; top-4 (largest) eigenpairs; V = U diag(sqrt(lambda)); stored FP32.
   Max-3-Cut objective (K = 3) as in Sec. 5.
3. ``maxcut_ppm``    3-block planted partition, n = 1,000,000, p_in = 8/n,
   p_out = 2/n; Laplacian; top-3; FP32 (the spectral truncation of Alg. 4).
4. ``psk_batch``     4,096 PSK-detection-shaped instances: n ~ U{16..256},
   r ~ U{2,3,4}; Q = H^H H + 0.05 (G + G^H)/sqrt(2), H r x n and G n x n with
   N_C(0,1) entries; top-r eigenpairs of Q; V = U diag(sqrt(max(lambda,0))).
5. phase synchronisation, n = 262,144, r = 3, K = 16: the top-3 factor of
   Q = U U^H + sigma W (U unit-modulus random phases, sigma = 0.5 sqrt(n)).
   The workload factor itself is computed by the library's matrix-free
   Lanczos (paper_2602_20376_amd/phase_sync.py); this module only draws the
   surrogate ``phase_sync_factor`` from the spiked-model law of those
   eigenvectors (overlap 1 - 1/theta^2 with the planted directions,
   theta = 2), used for the proposal network's training set and for unit
   tests of the network.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np

WORKLOADS = ("exact_small", "maxcut_er", "maxcut_ppm", "psk_batch")


def instance_seed(workload_no: int) -> int:
    return 1000 + workload_no


def direction_seed(workload_no: int) -> int:
    return 2000 + workload_no


# ----------------------------------------------------------------------------
# basic random objects
# ----------------------------------------------------------------------------

def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """N_C(0,1): real and imaginary parts independent N(0, 1/2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def random_V(n: int, r: int, seed: int, real: bool = False) -> np.ndarray:
    """A general-position factor: i.i.d. N_C(0,1) (or N(0,1) when real)."""
    rng = np.random.default_rng(seed)
    if real:
        return rng.standard_normal((n, r)).astype(np.complex128)
    return complex_gaussian(rng, (n, r))


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------

def _unique_pairs(rng, n, m, draw):
    """m distinct unordered pairs {i, j}, i != j, drawn by `draw(k)` -> (i, j)."""
    got = np.empty((0,), dtype=np.int64)
    while got.size < m:
        k = int((m - got.size) * 1.15) + 64
        i, j = draw(k)
        keep = i != j
        i, j = i[keep], j[keep]
        lo, hi = np.minimum(i, j), np.maximum(i, j)
        got = np.unique(np.concatenate([got, lo * n + hi]))
    # keep a seeded subset of exactly m pairs
    sel = rng.choice(got.size, size=m, replace=False)
    keys = np.sort(got[sel])
    return keys // n, keys % n


def er_edges(n: int, mean_degree: float, seed: int):
    """G(n, p) with p = mean_degree / (n - 1): edge count ~ Binomial, then a
    uniform set of that many distinct pairs (same law as independent edges)."""
    rng = np.random.default_rng(seed)
    npairs = n * (n - 1) // 2
    p = mean_degree / (n - 1)
    m = int(rng.binomial(npairs, p))

    def draw(k):
        return rng.integers(0, n, k), rng.integers(0, n, k)

    return _unique_pairs(rng, n, m, draw)


def planted_partition_edges(n: int, p_in: float, p_out: float, seed: int, blocks: int = 3):
    """Balanced `blocks`-community planted partition; block sizes differ by <= 1."""
    rng = np.random.default_rng(seed)
    sizes = np.full(blocks, n // blocks, dtype=np.int64)
    sizes[: n % blocks] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    I, J = [], []
    for a in range(blocks):
        for b in range(a, blocks):
            na, nb = int(sizes[a]), int(sizes[b])
            if a == b:
                npairs = na * (na - 1) // 2
                p = p_in
            else:
                npairs = na * nb
                p = p_out
            m = int(rng.binomial(npairs, p))
            if m == 0:
                continue
            if a == b:
                def draw(k, na=na, sa=starts[a]):
                    return rng.integers(0, na, k) + sa, rng.integers(0, na, k) + sa
            else:
                def draw(k, na=na, nb=nb, sa=starts[a], sb=starts[b]):
                    return rng.integers(0, na, k) + sa, rng.integers(0, nb, k) + sb
            i, j = _unique_pairs(rng, n, m, draw)
            I.append(i)
            J.append(j)
    return np.concatenate(I), np.concatenate(J)


def laplacian(n: int, i: np.ndarray, j: np.ndarray):
    """Unweighted graph Laplacian L = D - A as scipy CSR (FP64)."""
    import scipy.sparse as sp

    data = np.ones(i.size, dtype=np.float64)
    A = sp.coo_matrix((data, (i, j)), shape=(n, n))
    A = (A + A.T).tocsr()
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(deg) - A).tocsr()


def csr_adjacency(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray | None = None):
    """Symmetric adjacency of the undirected edges (i, j) (each once, i != j)
    in the CSR layout of the library's graph calls: row_ptr (int64, n + 1),
    col (int32), w (float64 or None); the entries of a row sorted by column."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    src = np.concatenate([i, j])
    dst = np.concatenate([j, i])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    ww = None
    if w is not None:
        w = np.asarray(w, dtype=np.float64)
        ww = np.concatenate([w, w])[order]
    return row_ptr, dst.astype(np.int32), ww


def random_edges(n: int, m: int, seed: int):
    """m distinct undirected edges without self loops, uniform."""
    rng = np.random.default_rng(seed)

    def draw(k):
        return rng.integers(0, n, k), rng.integers(0, n, k)

    return _unique_pairs(rng, n, m, draw)


def regular_edges(n: int, d: int, seed: int):
    """A random d-regular simple graph on n vertices (n d even): the union of
    d random perfect matchings (d odd, n even), each matching drawn again
    until it shares no edge with the earlier ones."""
    if n % 2 or d < 1:
        raise ValueError("n must be even and d positive")
    rng = np.random.default_rng(seed)
    seen = set()
    ii, jj = [], []
    for _ in range(d):
        while True:
            p = rng.permutation(n)
            a, b = np.minimum(p[0::2], p[1::2]), np.maximum(p[0::2], p[1::2])
            keys = set((a.astype(np.int64) * n + b).tolist())
            if not keys & seen:
                break
        seen |= keys
        ii.append(a)
        jj.append(b)
    return np.concatenate(ii), np.concatenate(jj)


def top_factor_sparse(L, r: int, seed: int) -> np.ndarray:
    """V = U diag(sqrt(lambda)) from the r largest eigenpairs of a PSD sparse
    matrix (FP64 Lanczos via ARPACK), columns in descending eigenvalue order."""
    from scipy.sparse.linalg import eigsh

    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(L.shape[0])
    lam, U = eigsh(L, k=r, which="LA", v0=v0, tol=1e-10, ncv=max(4 * r + 1, 24))
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    # fix each eigenvector's sign: largest-magnitude entry positive
    for k in range(r):
        idx = np.argmax(np.abs(U[:, k]))
        if U[idx, k] < 0:
            U[:, k] = -U[:, k]
    return U * np.sqrt(np.maximum(lam, 0.0))[None, :]


# ----------------------------------------------------------------------------
# on-disk cache (inputs only; keyed by recipe + parameters)
# ----------------------------------------------------------------------------

def _cache_dir() -> str:
    d = os.environ.get("LRQO_INPUT_CACHE", os.path.join("/tmp", "lrqo_input_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def _cached(tag: str, fn):
    key = hashlib.sha1(tag.encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), f"{key}.npy")
    if os.path.exists(path):
        return np.load(path, allow_pickle=False)
    arr = fn()
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "wb") as fh:
        np.save(fh, arr, allow_pickle=False)
    os.replace(tmp, path)
    return arr


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclass
class Instance:
    V: np.ndarray          # complex128 (n, r); FP32-stored workloads hold FP32-exact values
    K: int
    S: int
    seed: int              # direction seed
    real: bool             # V has zero imaginary part
    name: str

    @property
    def n(self):
        return self.V.shape[0]

    @property
    def r(self):
        return self.V.shape[1]


def exact_small(n: int = 12, r: int = 2, K: int = 3) -> Instance:
    V = random_V(n, r, instance_seed(1))
    return Instance(V, K, 0, direction_seed(1), False, f"exact_small(n={n},r={r},K={K})")


def maxcut_er(n: int = 100_000, mean_degree: float = 10.0, r: int = 4, K: int = 3,
              S: int = 65_536) -> Instance:
    seed = instance_seed(2)

    def build():
        i, j = er_edges(n, mean_degree, seed)
        L = laplacian(n, i, j)
        return top_factor_sparse(L, r, seed).astype(np.float32)

    V32 = _cached(f"maxcut_er:{n}:{mean_degree}:{r}:{seed}:v1", build)
    return Instance(V32.astype(np.float64).astype(np.complex128), K, S, direction_seed(2), True,
                    f"maxcut_er(n={n},deg={mean_degree:g},r={r},K={K},S={S})")


def regular_factor(n: int, d: int = 5, r: int = 2, seed: int = 0) -> np.ndarray:
    """Max-3-Cut factor of a random d-regular graph: the top r eigenvectors
    of its Laplacian scaled by sqrt(eigenvalue), FP64."""
    i, j = regular_edges(n, d, instance_seed(10) + seed)
    return top_factor_sparse(laplacian(n, i, j), r, instance_seed(10) + seed)


def maxcut_er_graph(n: int = 100_000, mean_degree: float = 10.0):
    """The graph whose Laplacian gives the maxcut_er factor: its undirected
    edges (i, j), same seed."""
    return er_edges(n, mean_degree, instance_seed(2))


def maxcut_ppm(n: int = 1_000_000, r: int = 3, K: int = 3, S: int = 1 << 20,
               c_in: float = 8.0, c_out: float = 2.0) -> Instance:
    seed = instance_seed(3)

    def build():
        i, j = planted_partition_edges(n, c_in / n, c_out / n, seed)
        L = laplacian(n, i, j)
        return top_factor_sparse(L, r, seed).astype(np.float32)

    V32 = _cached(f"maxcut_ppm:{n}:{c_in}:{c_out}:{r}:{seed}:v1", build)
    return Instance(V32.astype(np.float64).astype(np.complex128), K, S, direction_seed(3), True,
                    f"maxcut_ppm(n={n},r={r},K={K},S={S})")


def maxcut_ppm_graph(n: int = 1_000_000, c_in: float = 8.0, c_out: float = 2.0):
    """The graph whose Laplacian gives the maxcut_ppm factor: its undirected
    edges (i, j), same seed."""
    return planted_partition_edges(n, c_in / n, c_out / n, instance_seed(3))


def psk_instance(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """One PSK-detection-shaped factor (complex, FP32-representable)."""
    H = complex_gaussian(rng, (r, n))
    G = complex_gaussian(rng, (n, n))
    Q = H.conj().T @ H + 0.05 * (G + G.conj().T) / np.sqrt(2.0)
    lam, U = np.linalg.eigh(Q)
    lam, U = lam[::-1][:r], U[:, ::-1][:, :r]
    V = U * np.sqrt(np.maximum(lam, 0.0))[None, :]
    return V.astype(np.complex64).astype(np.complex128)


@dataclass
class Batch:
    """Concatenated factors: instance t is rows[row_off[t]:row_off[t]+n[t], :r[t]]
    of the (sum n, 4) complex array `rows` (unused columns zero)."""
    rows: np.ndarray
    n: np.ndarray
    r: np.ndarray
    K: int
    S: int
    seed: int

    @property
    def count(self):
        return self.n.size

    def factor(self, t: int) -> np.ndarray:
        o = int(np.sum(self.n[:t]))
        return self.rows[o:o + self.n[t], :self.r[t]]

    def device_layout(self, real: bool = False):
        """(float32 concatenation, v_offset in floats) in the library's layout."""
        parts, offs, off = [], [], 0
        for t in range(self.count):
            V = self.factor(t)
            a = as_real_f32(V).ravel() if real else as_interleaved_f32(V).ravel()
            parts.append(a)
            offs.append(off)
            off += a.size
        return np.concatenate(parts), np.asarray(offs, dtype=np.int64)


def psk_batch(count: int = 4096, n_lo: int = 16, n_hi: int = 256, K: int = 8, S: int = 4096) -> Batch:
    """PSK-detection-shaped instances (see psk_instance), n ~ U{n_lo..n_hi},
    r ~ U{2, 3, 4}."""
    seed = instance_seed(4)
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count).astype(np.int32)
    rs = rng.integers(2, 5, count).astype(np.int32)

    def build():
        out = np.zeros((int(ns.sum()), 4), dtype=np.complex128)
        o = 0
        for t in range(count):
            sub = np.random.default_rng([seed, t])
            out[o:o + ns[t], :rs[t]] = psk_instance(sub, int(ns[t]), int(rs[t]))
            o += ns[t]
        return out

    rows = _cached(f"psk_batch:{count}:{n_lo}:{n_hi}:{seed}:v1", build)
    return Batch(rows, ns, rs, K, S, direction_seed(4))


def phase_sync_factor(n: int, r: int, seed: int, theta: float = 2.0) -> np.ndarray:
    """Top-r eigenvectors of U U^H + sigma W drawn from the spiked-model law.

    U has unit-modulus random-phase entries, sigma = 0.5 sqrt(n); in units of
    sigma sqrt(n) the planted spikes have strength theta = n / (sigma sqrt(n)) = 2.
    Above the detection threshold the leading eigenvectors carry squared
    overlap 1 - 1/theta^2 with the planted directions and are otherwise
    delocalised, with eigenvalues sigma sqrt(n) (theta + 1/theta).
    """
    rng = np.random.default_rng(seed)
    U = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, (n, r))) / np.sqrt(n)
    G = complex_gaussian(rng, (n, r))
    G -= U @ (U.conj().T @ G)
    G, _ = np.linalg.qr(G)
    a = np.sqrt(1.0 - 1.0 / theta ** 2)
    b = 1.0 / theta
    R = np.linalg.qr(complex_gaussian(rng, (r, r)))[0]      # gauge mix inside the spike
    E, _ = np.linalg.qr((a * U + b * G) @ R)
    sigma = 0.5 * np.sqrt(n)
    lam = sigma * np.sqrt(n) * (theta + 1.0 / theta) * (1.0 + 0.01 * rng.standard_normal(r))
    lam = np.sort(lam)[::-1]
    return (E * np.sqrt(lam)[None, :]).astype(np.complex64).astype(np.complex128)


def as_interleaved_f32(V: np.ndarray) -> np.ndarray:
    """(n, r) complex -> (n, r, 2) float32, the device layout of a complex64 factor."""
    out = np.empty(V.shape + (2,), dtype=np.float32)
    out[..., 0] = V.real
    out[..., 1] = V.imag
    return out


def as_real_f32(V: np.ndarray) -> np.ndarray:
    """(n, r) real-valued factor -> (n, r) float32 row-major."""
    assert np.all(V.imag == 0)
    return np.ascontiguousarray(V.real.astype(np.float32))


# ----------------------------------------------------------------------------
# learned proposal: initial weights and training instances
# ----------------------------------------------------------------------------

PROPOSAL_DIMS = {"d_in": 6, "hidden": 64, "ncomp": 32}


def proposal_init(seed: int) -> np.ndarray:
    """Initial parameters of the direction-proposal network, packed as
    [W1 (64x6), b1 (64), W2 (64x64), b2 (64), W3 (256x64), b3 (256)],
    row-major, float64.  He-normal hidden layers, a small head; the head
    bias gives every mixture component a random mean direction, equal
    weight and concentration 20."""
    d, h, c = PROPOSAL_DIMS["d_in"], PROPOSAL_DIMS["hidden"], PROPOSAL_DIMS["ncomp"]
    out_dim = c * (d + 2)
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((h, d)) * np.sqrt(2.0 / d)
    b1 = np.zeros(h)
    W2 = rng.standard_normal((h, h)) * np.sqrt(2.0 / h)
    b2 = np.zeros(h)
    W3 = rng.standard_normal((out_dim, h)) * (0.1 / np.sqrt(h))
    b3 = np.zeros((c, d + 2))
    b3[:, :d] = rng.standard_normal((c, d))
    b3[:, d] = 0.0
    b3[:, d + 1] = np.log(20.0)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3.ravel()])


def phase_sync_training_set(count: int, seed: int = 7000, n_lo: int = 1 << 10, n_hi: int = 1 << 14):
    """(list of V, list of n) phase-synchronisation factors, n ~ log-uniform in
    [n_lo, n_hi]: the training distribution of the proposal network."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).astype(np.int64)
    return [phase_sync_factor(int(ns[t]), 3, seed * 100003 + t) for t in range(count)], ns
