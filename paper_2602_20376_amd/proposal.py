"""Training driver of the learned direction proposal.

Host orchestration only: targets come from the plain sampled solver (HIP),
every forward, backward and Adam step runs in the library's kernels
(lrqo_proposal_train_step).  Checkpoints hold parameters and Adam state.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import inputs, lrqo


def pack_factors(Vs):
    """Concatenate complex (n_t, 3) factors into the library layout."""
    parts, offs, ns, off = [], [], [], 0
    for V in Vs:
        a = inputs.as_interleaved_f32(V).ravel()
        parts.append(a)
        offs.append(off)
        ns.append(V.shape[0])
        off += a.size
    return np.concatenate(parts), np.asarray(offs, np.int64), np.asarray(ns, np.int64)


def label_targets(Vs, K: int, S: int, seed: int):
    """Best direction of each instance under the plain uniform sampler
    (complex (count, 3)) and its objective."""
    import torch

    best_c = np.zeros((len(Vs), 3), np.complex128)
    best_f = np.zeros(len(Vs))
    for t, V in enumerate(Vs):
        out = lrqo.solve_sampled(torch.from_numpy(V.astype(np.complex64)).cuda(), K, S, seed, instance=t)
        best_c[t] = np.asarray(out.best_c)
        best_f[t] = out.obj
    return best_c, best_f


def targets_real(best_c):
    t = np.empty((best_c.shape[0], 6), np.float32)
    t[:, 0::2] = best_c.real
    t[:, 1::2] = best_c.imag
    return t


def train(prop: "lrqo.Proposal", Vs, best_c, epochs: int, batch: int, lr: float, seed: int = 0,
          log=None):
    """Mini-batch Adam over the instances; returns per-epoch mean losses."""
    import torch

    cat, offs, ns = pack_factors(Vs)
    Vd = torch.from_numpy(cat).cuda()
    tg = targets_real(best_c)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(Vs))
        losses = []
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            L, _ = prop.train_step(Vd, offs[idx], ns[idx], tg[idx], lr)
            losses.append(L)
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def save(prop: "lrqo.Proposal", path: str, meta: dict | None = None):
    st = prop.get_state()
    np.savez(path, theta=st["theta"], m=st["m"], v=st["v"], step=np.int64(st["step"]),
             meta=np.frombuffer(json.dumps(meta or {}).encode(), dtype=np.uint8))


def load_into(prop: "lrqo.Proposal", path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        prop.set_state({"theta": z["theta"], "m": z["m"], "v": z["v"], "step": int(z["step"])})
        return json.loads(bytes(z["meta"]).decode() or "{}")


def knee(f_in_order, ref: float, frac: float = 0.999):
    """Samples needed for the running best of a direction stream to reach
    frac * ref (None if it never does)."""
    best = np.maximum.accumulate(np.asarray(f_in_order, dtype=np.float64))
    hit = np.nonzero(best >= frac * ref)[0]
    return int(hit[0]) + 1 if hit.size else None


def train_default(K: int = 16, count: int = 10_000, label_S: int = 16_384, epochs: int = 30,
                  batch: int = 64, lr: float = 3e-3, seed: int = 1, log=None):
    """The proposal trained on `count` phase-synchronisation instances at
    n ~ log-uniform [2^10, 2^14], labelled by the plain sampler's best of
    label_S directions.  Returns (proposal, loss history, seconds by phase)."""
    import time

    t = time.perf_counter()
    Vs, _ = inputs.phase_sync_training_set(count, seed=7000)
    t_gen = time.perf_counter() - t
    t = time.perf_counter()
    best_c, _ = label_targets(Vs, K, label_S, 31)
    t_label = time.perf_counter() - t
    prop = lrqo.Proposal(inputs.proposal_init(seed), K)
    t = time.perf_counter()
    hist = train(prop, Vs, best_c, epochs=epochs, batch=batch, lr=lr, log=log)
    t_train = time.perf_counter() - t
    return prop, hist, {"generate_s": t_gen, "label_s": t_label, "train_s": t_train}
