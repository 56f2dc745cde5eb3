"""Pins of the FP64 oracle of the learned band-tail correction (CPU)."""
import numpy as np
import pytest

import gwsynth as gs
from oracle import mlp_oracle as mo


def small_case(n=7, seed=0):
    rng = np.random.default_rng(seed)
    params = mo.unflatten(gs.mlp_init(seed).astype(np.float64))
    for k in ("w1", "w2", "w3"):
        params[k] = mo.bf16_round(params[k])
    x = np.stack([rng.uniform(0.3, 2.5, n), rng.uniform(-12, -6, n), np.full(n, 0.1), np.full(n, 0.3)], axis=1)
    mean = x.mean(axis=0)
    std = x.std(axis=0) + np.array([0, 0, 1, 1])
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    t = -(a @ a.conj().T) * 1e-5                      # Hermitian, negative semidefinite like the tail
    s = np.exp(x[:, 1])
    return params, x, mean, std, t, s


def test_bf16_rounding_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.140625, 1e-3], np.float32)
    got = mo.bf16_round(vals)
    # ties go to even: 1 + 2^-8 -> 1;  1 + 3*2^-8 -> 1 + 2^-6;  1 + 2^-7 + 2^-9 -> 1 + 2^-7 (below the tie)
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -3.140625, 0.00099945068359375])
    assert np.array_equal(got, want)


def test_loss_equals_elementwise_sum():
    params, x, mean, std, t, s = small_case()
    o, _ = mo.forward(x, params, mean, std)
    d, u = mo.head(o, s)
    n = len(s)
    num = 0.0
    for i in range(n):
        for j in range(n):
            corr = -((d[i] if i == j else 0.0) + sum(u[i, k] * np.conj(u[j, k]) for k in range(16)))
            num += abs(corr - t[i, j]) ** 2
    den = sum(abs(t[i, j]) ** 2 for i in range(n) for j in range(n))
    assert abs(mo.loss(o, s, t) - num / den) < 1e-12 * (num / den)


def test_correction_is_negative_semidefinite():
    params, x, mean, std, t, s = small_case(n=9, seed=4)
    o, _ = mo.forward(x, params, mean, std)
    c = mo.correction(o, s)
    assert np.max(np.abs(c - c.conj().T)) <= 1e-15 * np.abs(c).max()
    assert np.linalg.eigvalsh(c).max() <= 1e-12 * np.abs(c).max()


def test_grad_o_finite_differences():
    params, x, mean, std, t, s = small_case()
    o, _ = mo.forward(x, params, mean, std)
    g = mo.loss_grad_o(o, s, t)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(25):
        i, j = rng.integers(o.shape[0]), rng.integers(o.shape[1])
        op, om = o.copy(), o.copy()
        op[i, j] += h
        om[i, j] -= h
        fd = (mo.loss(op, s, t) - mo.loss(om, s, t)) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[i, j])


def test_parameter_grad_finite_differences():
    params, x, mean, std, t, s = small_case(n=6, seed=2)
    o, cache = mo.forward(x, params, mean, std)
    grads = mo.backward(mo.loss_grad_o(o, s, t), params, cache)
    rng = np.random.default_rng(3)
    h = 1e-6
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        for _ in range(6):
            idx = tuple(rng.integers(dim) for dim in params[name].shape)
            pp = {k: v.copy() for k, v in params.items()}
            pm = {k: v.copy() for k, v in params.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            lp = mo.loss(mo.forward(x, pp, mean, std)[0], s, t)
            lm = mo.loss(mo.forward(x, pm, mean, std)[0], s, t)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 2e-6 * max(1.0, abs(fd)), (name, idx, fd, grads[name][idx])


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    master = gs.mlp_init(5).astype(np.float64)
    g = rng.standard_normal(master.shape)
    new, m, v, p = mo.adam(master, np.zeros_like(master), np.zeros_like(master), g, 1, 1e-3)
    want = (master - 1e-3 * g / (np.abs(g) + 1e-8)).astype(np.float32).astype(np.float64)
    assert np.array_equal(new, want)
    assert np.array_equal(p["w2"], mo.bf16_round(new[640:640 + 16384].reshape(128, 128)))


def test_mlp_init_layout():
    v = gs.mlp_init(0)
    assert v.dtype == np.float32 and v.size == 21409
    p = mo.unflatten(v)
    assert p["b3"][0] == -2.0 and np.all(p["b1"] == 0)
