"""FP64 oracle of the learned band-tail correction (TEST INFRASTRUCTURE ONLY).

The correction predicts the missing unoccupied-band tail of the truncated sum (the band
truncation of Eq.(Pstatic) that the paper lists as its first technical issue):

  T        = H(P~_{4Nc}) - H(P~_{Nc})                   target, H(X) = (X + X^H)/2
  x_G      = (|q+G|, log|Re P~_{Nc}(G,G)|, Nc/N_g, E_max)   raw per-G features
  o_G      = MLP(normalise(x_G))                        4 -> 128 -> 128 -> 33, SiLU, BF16 weights
  s_G      = |Re P~_{Nc}(G,G)|
  d_G      = softplus(o_G0) s_G,   u_Gk = (o_G,1+k + i o_G,17+k) sqrt(s_G),  k < r (r <= 16; 0 beyond)
  dP~      = -(diag(d) + U U^H)                          negative semidefinite by construction
  loss     = ||dP~ - T||_F^2 / ||T||_F^2

The rank r of the U U^H term is a model setting (16 at most, chosen on validation systems); with r = 0
the correction is diagonal.

Every function here is the plain definition in float64 (dense N_g x N_g matrices where the
definition has them); the gradients are the analytic chain rule, pinned by central finite
differences in the CPU tests.  Weights are the BF16-rounded values the GPU uses (held as
float64); the FP32 Adam master copy is rounded to BF16 after every step.
"""
from __future__ import annotations

import numpy as np

WIDTH = 128
NOUT = 33
RANK = 16
SHAPES = [("w1", (4, WIDTH)), ("b1", (WIDTH,)), ("w2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("w3", (WIDTH, NOUT)), ("b3", (NOUT,))]


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest BF16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(pt_trunc, q, miller, a_bohr, nc, e_max) -> np.ndarray:
    """Raw per-G features [N_g][4] from the truncated P~ and the sphere."""
    qm = np.asarray(miller, np.float64) + np.asarray(q, np.float64)[None, :]
    kq = (2.0 * np.pi / a_bohr) * np.sqrt((qm ** 2).sum(axis=1))
    diag = np.abs(np.real(np.diag(pt_trunc)))
    ng = len(kq)
    return np.stack([kq, np.log(np.maximum(diag, 1e-30)), np.full(ng, nc / ng), np.full(ng, e_max)], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def softplus(z):
    return np.logaddexp(0.0, z)


def forward(x, params, mean, std):
    """o = MLP((x - mean)/std) and the intermediates the backward pass needs."""
    xn = (np.asarray(x, np.float64) - mean) / std
    z1 = xn @ params["w1"] + params["b1"]
    h1 = silu(z1)
    z2 = h1 @ params["w2"] + params["b2"]
    h2 = silu(z2)
    o = h2 @ params["w3"] + params["b3"]
    return o, dict(xn=xn, z1=z1, h1=h1, z2=z2, h2=h2)


def head(o, s, rank=RANK):
    d = softplus(o[:, 0]) * s
    u = (o[:, 1:1 + RANK] + 1j * o[:, 1 + RANK:1 + 2 * RANK]) * np.sqrt(s)[:, None]
    u[:, rank:] = 0.0
    return d, u


def correction(o, s, rank=RANK):
    d, u = head(o, s, rank)
    return -(np.diag(d) + u @ np.conj(u).T)


def loss(o, s, target, rank=RANK):
    """||dP~ - T||_F^2 / ||T||_F^2 with the dense correction."""
    t = np.asarray(target, np.complex128)
    r = correction(o, s, rank) - t
    return float(np.vdot(r, r).real / np.vdot(t, t).real)


def residual_parts(o, s, target, rank=RANK):
    """(||offdiag(dP~ - T)||^2, ||offdiag T||^2, ||diag(dP~ - T)||^2, ||diag T||^2) with the dense correction."""
    t = np.asarray(target, np.complex128)
    r = correction(o, s, rank) - t
    off = ~np.eye(len(t), dtype=bool)
    sq = lambda x: float((np.abs(x) ** 2).sum())
    return sq(r[off]), sq(t[off]), sq(np.diag(r)), sq(np.diag(t))


def loss_grad_o(o, s, target, rank=RANK):
    """d loss / d o  [N_g][33] by the chain rule through the head (dense B = diag(d) + U U^H + T)."""
    t = np.asarray(target, np.complex128)
    d, u = head(o, s, rank)
    b = np.diag(d) + u @ np.conj(u).T + t
    tn = np.vdot(t, t).real
    bu = b @ u
    g = np.zeros_like(o, dtype=np.float64)
    sig = 1.0 / (1.0 + np.exp(-o[:, 0]))
    g[:, 0] = 2.0 * np.real(np.diag(b)) * sig * s / tn
    g[:, 1:1 + RANK] = 4.0 * np.real(bu) * np.sqrt(s)[:, None] / tn
    g[:, 1 + RANK:] = 4.0 * np.imag(bu) * np.sqrt(s)[:, None] / tn
    g[:, 1 + rank:1 + RANK] = 0.0                  # outputs of unused U columns do not enter the loss
    g[:, 1 + RANK + rank:] = 0.0
    return g


def backward(go, params, cache):
    """Gradients of the weights and biases from d loss / d o."""
    g = {}
    g["w3"] = cache["h2"].T @ go
    g["b3"] = go.sum(axis=0)
    dh2 = go @ params["w3"].T
    dz2 = dh2 * dsilu(cache["z2"])
    g["w2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["w2"].T
    dz1 = dh1 * dsilu(cache["z1"])
    g["w1"] = cache["xn"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def flatten(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[k], np.float64).ravel() for k, _ in SHAPES])


def unflatten(v) -> dict:
    out, i = {}, 0
    for k, shp in SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(v[i:i + n], np.float64).reshape(shp)
        i += n
    return out


def fit_norm(feats) -> np.ndarray:
    """Feature statistics of a training set: mean and (population) std of every raw feature over all rows
    of all systems (std 1 where a feature is constant to 1e-12 of max(1, |mean|)), then the training box
    [min, max] of each feature; float32 [16]."""
    x = np.concatenate([np.asarray(f, np.float64) for f in feats], axis=0)
    mean = x.mean(axis=0)
    std = np.sqrt(((x - mean) ** 2).mean(axis=0))
    std[std <= 1e-12 * np.maximum(1.0, np.abs(mean))] = 1.0
    return np.concatenate([mean, std, x.min(axis=0), x.max(axis=0)]).astype(np.float32)


def adam(master, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the FP32 master copy; returns (master, m, v, weights for the next forward)
    where the weight matrices are BF16-rounded and the biases stay FP32."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    master = (master - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32).astype(np.float64)
    p = unflatten(master)
    for k in ("w1", "w2", "w3"):
        p[k] = bf16_round(p[k])
    for k in ("b1", "b2", "b3"):
        p[k] = p[k].astype(np.float32).astype(np.float64)
    return master, m, v, p
