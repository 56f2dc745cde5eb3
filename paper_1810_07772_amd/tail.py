"""Driver of the learned band-tail correction: builds training pairs with the plain method and
loops the library's training step over them.  Every arithmetic step (the builds, targets,
features, forward and backward passes and the optimiser) runs in libgw.so; this module only
orders the calls and chooses, on validation systems, the rank of the correction's U U^H term."""
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


def fit_norm(feats: Sequence):
    """Feature mean, std (1 where a feature is constant) and the training box [lo, hi], computed by the
    library over every row of the training features: a device float32 [16]."""
    return L.tail_fit_norm(list(feats))


def mean_loss(model: "L.TailModel", entries: List[Dict]) -> float:
    """Mean loss of the current weights over the entries (no update)."""
    import torch
    out = torch.zeros(len(entries), dtype=torch.float32, device=entries[0]["feat"].device)
    for i, e in enumerate(entries):
        model.loss(e["feat"], e["target"], loss_out=out[i:i + 1])
    return float(out.cpu().numpy().astype(np.float64).mean())


def residual_parts(model: "L.TailModel", entries: List[Dict]) -> np.ndarray:
    """Pooled (||offdiag(dP~ - T)||^2, ||offdiag T||^2, ||diag(dP~ - T)||^2, ||diag T||^2) over the entries."""
    import torch
    out = torch.zeros((len(entries), 4), dtype=torch.float32, device=entries[0]["feat"].device)
    for i, e in enumerate(entries):
        model.residual_parts(e["feat"], e["target"], out=out[i])
    return out.cpu().numpy().astype(np.float64).sum(axis=0)


def train(model: "L.TailModel", entries: List[Dict], epochs: int, seed: int = 0, val: List[Dict] = None,
          log=None) -> List[tuple]:
    """Adam over the training entries (one system per step, shuffled every epoch), each epoch's steps replayed
    from the library's captured training-step graphs.  Returns per epoch (mean training loss during the
    epoch, mean validation loss after it or None)."""
    import torch
    rng = np.random.default_rng(seed)
    dev = entries[0]["feat"].device
    losses = torch.zeros(len(entries), dtype=torch.float32, device=dev)
    feats = [e["feat"] for e in entries]
    targets = [e["target"] for e in entries]
    hist = []
    for ep in range(epochs):
        model.train_steps(feats, targets, rng.permutation(len(entries)), losses)
        tl = float(losses.cpu().numpy().astype(np.float64).mean())
        vl = mean_loss(model, val) if val else None
        hist.append((tl, vl))
        if log:
            log(f"epoch {ep + 1}/{epochs}: training loss {tl:.4f}" + (f", validation loss {vl:.4f}" if val else ""))
    return hist


def train_select_rank(master, norm, entries: List[Dict], val: List[Dict], epochs: int, ranks=(16, 0),
                      lr: float = 3e-4, seed: int = 0, log=None):
    """One model per candidate rank of the U U^H term, all from the same initial weights and shuffles.  A
    candidate is admissible if its pooled validation off-diagonal residual ||offdiag(dP~ - T)|| is not above
    that of no correction, ||offdiag T|| (always true at rank 0, whose correction is diagonal); among the
    admissible ones the lowest pooled validation loss wins.  Returns (model, history, {rank: parts})."""
    best = None
    report = {}
    for r in ranks:
        model = L.TailModel(master, norm, lr=lr, rank=r)
        hist = train(model, entries, epochs, seed=seed, val=val, log=log)
        parts = residual_parts(model, val)
        report[r] = parts
        admissible = parts[0] <= parts[1]
        vloss = (parts[0] + parts[2]) / (parts[1] + parts[3])
        if log:
            log(f"rank {r}: validation loss {vloss:.4f}, off-diagonal residual {np.sqrt(parts[0] / parts[1]):.4f} "
                f"of the plain one{'' if admissible else ' (rejected)'}")
        if admissible and (best is None or vloss < best[0]):
            best = (vloss, model, hist)
    return best[1], best[2], report
