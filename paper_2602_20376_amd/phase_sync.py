"""Phase-synchronisation workload: Q = U U^H + sigma W and its top-r factor.

U is n x p with unit-modulus entries of uniform random phase, sigma =
0.5 sqrt(n) and W the Hermitian Gaussian matrix of the counter-based
definition in include/lrqo.h (lrqo_phase_sync_factor), seed w_seed.  The
factor V = U_r diag(sqrt(lambda)) of the r largest eigenpairs is computed by
the library's matrix-free Lanczos on the GPU (the dense matrix at
n = 262,144 would take about 1.1 TB); it is the input of the sampled solver
and of the learned proposal on this workload.
"""
from __future__ import annotations

import numpy as np

_CACHE: dict = {}


def problem(n: int, seed: int, p: int = 3):
    """(U, sigma, w_seed) of instance `seed`: U from numpy PCG64 (seed),
    w_seed derived from it."""
    rng = np.random.default_rng([seed, n])
    U = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, (n, p)))
    return U, 0.5 * np.sqrt(n), int(rng.integers(1, 2 ** 62))


def true_factor(n: int, seed: int, r: int = 3, tol: float = 1e-8, max_iter: int = 200):
    """(V complex128 (n, r) on the host, eigenvalues, Lanczos steps) of
    instance `seed`, by lrqo_phase_sync_factor; cached per process."""
    key = (n, seed, r, tol)
    if key not in _CACHE:
        import torch

        from . import lrqo

        U, sigma, w_seed = problem(n, seed)
        V, res = lrqo.phase_sync_factor(torch.from_numpy(U).cuda(), sigma, w_seed, r, tol=tol, max_iter=max_iter)
        torch.cuda.synchronize()
        if not res.converged:
            raise RuntimeError(f"phase-sync Lanczos did not converge (n={n}, seed={seed})")
        _CACHE[key] = (V.cpu().numpy(), np.array(res.eigenvalues[:r]), int(res.iterations))
    return _CACHE[key]


def fp32_factor(n: int, seed: int, r: int = 3) -> np.ndarray:
    """The factor as the solvers read it: complex64 values widened to FP64."""
    V, _, _ = true_factor(n, seed, r)
    return V.astype(np.complex64).astype(np.complex128)
