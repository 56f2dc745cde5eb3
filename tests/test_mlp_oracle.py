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


# ---------------------------------------------------------------------------------------------
# Hand values of the feature map, the activations and the output head.  The features are the
# reading of the learned tail's per-G inputs (band truncation of Eq.(Pstatic), the paper's first
# technical issue): |q+G| in 1/Bohr with G = (2 pi / a) m, log |Re P~_Nc(G,G)|, Nc / N_g and E_max.
# Every expected number below is written out from its closed form (30-digit evaluation), not from
# the oracle.
# ---------------------------------------------------------------------------------------------
def test_features_hand_values():
    a_bohr = 4.0                                  # 2 pi / a = pi / 2
    q = [0.0, 0.0, 0.5]
    miller = [[0, 0, 0], [2, 1, -1], [-1, 2, 2]]  # |q+m|^2 = 0.25, 5.25, 11.25
    pt = np.array([[-2.0 + 3.0j, 7.0 - 1.0j, 5.0 + 5.0j],
                   [7.0 + 1.0j, -0.5 - 0.25j, -9.0 + 2.0j],
                   [5.0 - 5.0j, -9.0 - 2.0j, 1e-40 + 4.0j]])
    x = mo.features(pt, q, miller, a_bohr, nc=6, e_max=0.3125)
    assert x.shape == (3, 4)
    # |q+G| = (pi/2) sqrt(0.25), (pi/2) sqrt(5.25), (pi/2) sqrt(11.25)
    np.testing.assert_allclose(x[:, 0], [0.785398163397448309615660845820, 3.59914653444810207094217103239,
                                         5.26861104828054479486728098240], rtol=1e-15)
    # log |Re P~(G,G)|: log 2, log 0.5, and the 1e-30 floor for a vanishing real part
    np.testing.assert_allclose(x[:, 1], [0.693147180559945309417232121458, -0.693147180559945309417232121458,
                                         -69.0775527898213705205397436405], rtol=1e-15)
    # Nc / N_g = 6 / 3 and E_max on every row
    assert np.array_equal(x[:, 2], [2.0, 2.0, 2.0])
    assert np.array_equal(x[:, 3], [0.3125, 0.3125, 0.3125])


def test_activation_hand_values():
    z = np.array([0.0, 1.0, -2.0, 3.0])
    # silu(z) = z / (1 + e^-z): 0, e/(1+e), -2/(1+e^2), 3/(1+e^-3)
    np.testing.assert_allclose(mo.silu(z), [0.0, 0.731058578630004879251159241822,
                                            -0.238405844044235111880541717395, 2.85772238046729965736345554468],
                               rtol=1e-15, atol=0)
    # silu'(z) = sigma(z) (1 + z (1 - sigma(z))): 1/2 at 0
    np.testing.assert_allclose(mo.dsilu(np.array([0.0, 1.0, -2.0])),
                               [0.5, 0.927670511871486731788583975408, -0.0907842487848954787569775108232],
                               rtol=1e-14)
    # softplus(z) = log(1 + e^z): log 2, log(1+e), log(1+e^-3), e^-30 to first order, 40 (+4e-18)
    np.testing.assert_allclose(mo.softplus(np.array([0.0, 1.0, -3.0, -30.0, 40.0])),
                               [0.693147180559945309417232121458, 1.31326168751822283404899549497,
                                0.0485873515737420587589259198547, 9.35762296883973677414241121536e-14, 40.0],
                               rtol=1e-14)


def test_head_hand_values():
    """d = softplus(o_0) s and u_k = (o_{1+k} + i o_{17+k}) sqrt(s) on one G row."""
    o = np.zeros((1, 33))
    o[0, 0] = 0.0
    o[0, 1], o[0, 17] = 3.0, -4.0      # u_0 = (3 - 4i) sqrt(s)
    o[0, 16], o[0, 32] = 0.5, 0.25     # u_15 = (0.5 + 0.25i) sqrt(s)
    s = np.array([4.0])
    d, u = mo.head(o, s)
    np.testing.assert_allclose(d, [4.0 * 0.693147180559945309417232121458], rtol=1e-15)
    assert u.shape == (1, 16)
    assert u[0, 0] == 6.0 - 8.0j and u[0, 15] == 1.0 + 0.5j and np.all(u[0, 1:15] == 0)
    # the correction is -(d + |u|^2) on the diagonal: -(4 log 2 + 100 + 1.25)
    np.testing.assert_allclose(mo.correction(o, s), [[-(2.77258872223978123766892848583 + 101.25)]], rtol=1e-15)


def test_rank_zero_correction_is_diagonal_and_rank_masks_columns():
    params, x, mean, std, t, s = small_case(n=6, seed=8)
    o, _ = mo.forward(x, params, mean, std)
    c0 = mo.correction(o, s, rank=0)
    assert np.array_equal(c0, np.diag(np.diag(c0)))
    np.testing.assert_allclose(np.diag(c0).real, -mo.softplus(o[:, 0]) * s, rtol=1e-15)
    # rank 3: exactly the first three columns of U, by an explicit sum
    d, u = mo.head(o, s)
    want = -(np.diag(d) + sum(np.outer(u[:, k], np.conj(u[:, k])) for k in range(3)))
    assert np.max(np.abs(mo.correction(o, s, rank=3) - want)) <= 1e-15 * np.abs(want).max()


def test_residual_parts_elementwise():
    params, x, mean, std, t, s = small_case(n=5, seed=6)
    o, _ = mo.forward(x, params, mean, std)
    for rank in (16, 2, 0):
        d, u = mo.head(o, s)
        parts = [0.0, 0.0, 0.0, 0.0]
        for i in range(5):
            for j in range(5):
                corr = -((d[i] if i == j else 0.0) + sum(u[i, k] * np.conj(u[j, k]) for k in range(rank)))
                k = 2 if i == j else 0
                parts[k] += abs(corr - t[i, j]) ** 2
                parts[k + 1] += abs(t[i, j]) ** 2
        got = mo.residual_parts(o, s, t, rank)
        np.testing.assert_allclose(got, parts, rtol=1e-12)
        assert abs((got[0] + got[2]) / (got[1] + got[3]) - mo.loss(o, s, t, rank)) <= 1e-12 * mo.loss(o, s, t, rank)


def test_grad_o_finite_differences_reduced_rank():
    params, x, mean, std, t, s = small_case(seed=11)
    o, _ = mo.forward(x, params, mean, std)
    g = mo.loss_grad_o(o, s, t, rank=5)
    assert np.all(g[:, 6:17] == 0) and np.all(g[:, 22:] == 0)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(25):
        i, j = rng.integers(o.shape[0]), rng.integers(o.shape[1])
        op, om = o.copy(), o.copy()
        op[i, j] += h
        om[i, j] -= h
        fd = (mo.loss(op, s, t, 5) - mo.loss(om, s, t, 5)) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[i, j])


def test_fit_norm_hand_values():
    a = np.array([[1.0, 2.0, 0.5, 3.0], [3.0, 2.0, 0.5, 3.0]])
    b = np.array([[5.0, 2.0, 0.5, 3.0]])
    nm = mo.fit_norm([a, b])
    # feature 0: values 1, 3, 5 -> mean 3, population std sqrt(8/3); the constant features get std 1
    np.testing.assert_allclose(nm[:4], [3.0, 2.0, 0.5, 3.0], rtol=1e-7)
    np.testing.assert_allclose(nm[4:8], [1.632993161855452, 1.0, 1.0, 1.0], rtol=1e-7)
    np.testing.assert_array_equal(nm[8:12], [1.0, 2.0, 0.5, 3.0])
    np.testing.assert_array_equal(nm[12:], [5.0, 2.0, 0.5, 3.0])
    assert nm.dtype == np.float32
