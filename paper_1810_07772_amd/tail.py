"""Driver of the learned band-tail correction: builds training pairs with the plain method and
loops the library's training step over them.  Every arithmetic step (the builds, targets,
features, forward and backward passes and the optimiser) runs in libgw.so; this module only
orders the calls and keeps the host-side bookkeeping (the training set's feature statistics)."""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from . import _lib as L


def pair_builds(psi_v, psi_c_full, e_v, e_c_full, n, a_bohr, q, miller, nc: int, precision="fp32"):
    """Plain builds with the first nc and the first 4 nc unoccupied bands, the training target
    between them and the features of the truncated build.  Returns (feat, target, p_nc, p_4nc)."""
    p_t = L.polarizability(psi_v, psi_c_full[:nc], e_v, e_c_full[:nc], n, a_bohr, q, miller, precision=precision)
    p_f = L.polarizability(psi_v, psi_c_full[:4 * nc], e_v, e_c_full[:4 * nc], n, a_bohr, q, miller,
                           precision=precision)
    target = L.tail_target(p_f, p_t)
    feat = L.tail_features(p_t, n, a_bohr, q, miller, nc, float(e_c_full[nc - 1]))
    return feat, target, p_t, p_f


def fit_norm(feats: Sequence) -> np.ndarray:
    """Feature mean, std (1 where a feature is constant) and the training box [lo, hi]."""
    x = np.concatenate([f.detach().cpu().numpy().astype(np.float64) for f in feats], axis=0)
    mean = x.mean(axis=0)
    std = x.std(axis=0)
    std[std <= 1e-12 * np.maximum(1.0, np.abs(mean))] = 1.0
    return np.concatenate([mean, std, x.min(axis=0), x.max(axis=0)]).astype(np.float32)


def mean_loss(model: "L.TailModel", entries: List[Dict]) -> float:
    """Mean loss of the current weights over the entries (no update)."""
    import torch
    out = torch.zeros(len(entries), dtype=torch.float32, device=entries[0]["feat"].device)
    for i, e in enumerate(entries):
        model.loss(e["feat"], e["target"], loss_out=out[i:i + 1])
    return float(out.cpu().numpy().astype(np.float64).mean())


def train(model: "L.TailModel", entries: List[Dict], epochs: int, seed: int = 0, val: List[Dict] = None,
          log=None) -> List[tuple]:
    """Adam over the training entries (one system per step, shuffled every epoch).  Returns per epoch
    (mean training loss during the epoch, mean validation loss after it or None)."""
    import torch
    rng = np.random.default_rng(seed)
    dev = entries[0]["feat"].device
    losses = torch.zeros(len(entries), dtype=torch.float32, device=dev)
    hist = []
    for ep in range(epochs):
        for i in rng.permutation(len(entries)):
            model.train_step(entries[i]["feat"], entries[i]["target"], loss_out=losses[i:i + 1])
        tl = float(losses.cpu().numpy().astype(np.float64).mean())
        vl = mean_loss(model, val) if val else None
        hist.append((tl, vl))
        if log:
            log(f"epoch {ep + 1}/{epochs}: training loss {tl:.4f}" + (f", validation loss {vl:.4f}" if val else ""))
    return hist
