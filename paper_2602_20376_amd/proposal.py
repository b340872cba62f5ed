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
