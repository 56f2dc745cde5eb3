"""The Python binding checks every buffer's shape and every host array's length against the sizes
it passes to the C ABI, before any device or library call (CPU tensors suffice: a mismatch raises
ValueError; a consistent call passes the shape checks and fails later, at the device or context
step, with another error)."""
import numpy as np
import pytest
import torch

import paper_1810_07772_amd as gw

N = (4, 3, 2)
NR = 24
MILLER = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.int32)
NG = 3
Q = [0.0, 0.0, 0.0]


def c64(*shape):
    return torch.zeros(shape, dtype=torch.complex64)


def c128(*shape):
    return torch.zeros(shape, dtype=torch.complex128)


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


EV, EC = [-0.3, -0.2], [0.1, 0.2, 0.3]


def raises_value(fn, match):
    with pytest.raises(ValueError, match=match):
        fn()


def reaches_device_check(fn):
    with pytest.raises(Exception) as e:
        fn()
    assert not isinstance(e.value, ValueError), e.value


def test_pair_products_shapes():
    reaches_device_check(lambda: gw.pair_products(c64(2, NR), c64(3, NR), EV, EC))
    raises_value(lambda: gw.pair_products(c64(2, NR), c64(3, NR + 1), EV, EC), "grid points")
    raises_value(lambda: gw.pair_products(c64(2, NR), c64(3, NR), EV[:1], EC), "e_v")
    raises_value(lambda: gw.pair_products(c64(2, NR), c64(3, NR), EV, EC + [0.4]), "e_c")
    raises_value(lambda: gw.pair_products(c64(2, NR), c64(3, NR), EV, EC, out=c64(5, NR)), "f_out")
    raises_value(lambda: gw.pair_products(c64(2 * NR), c64(3, NR), EV, EC), "dimensions")


def test_polarizability_r_shapes():
    reaches_device_check(lambda: gw.polarizability_r(c64(2, NR), c64(3, NR), EV, EC))
    raises_value(lambda: gw.polarizability_r(c64(2, NR), c64(3, NR), EV, EC, out=c64(NR, NR - 1)), "p_rr")
    raises_value(lambda: gw.polarizability_r(c64(2, NR), c64(3, NR), [-0.3, -0.2, -0.1], EC), "e_v")


def test_polarizability_shapes():
    call = lambda pv=c64(2, NR), pc=c64(3, NR), ev=EV, ec=EC, n=N, q=Q, m=MILLER, **kw: \
        gw.polarizability(pv, pc, ev, ec, n, 5.0, q, m, **kw)
    reaches_device_check(call)
    reaches_device_check(lambda: call(p_rr=c64(NR, NR), out=c64(NG, NG)))
    raises_value(lambda: call(n=(4, 3, 3)), "grid")
    raises_value(lambda: call(pv=c64(2, NR + 2), pc=c64(3, NR + 2)), "grid")
    raises_value(lambda: call(ec=EC[:2]), "e_c")
    raises_value(lambda: call(q=[0.0, 0.0]), "q")
    raises_value(lambda: call(m=MILLER[:, :2]), r"\[ng\]\[3\]")
    raises_value(lambda: call(p_rr=c64(NR, NR + 1)), "p_rr")
    raises_value(lambda: call(out=c64(NG + 1, NG + 1)), "p_gg")


def test_transform_and_epsilon_shapes():
    reaches_device_check(lambda: gw.sphere_transform(c64(NR, NR), N, MILLER))
    raises_value(lambda: gw.sphere_transform(c64(NR - 1, NR - 1), N, MILLER), "p_rr")
    raises_value(lambda: gw.sphere_transform(c64(NR, NR), N, MILLER, out=c64(NG, NG + 1)), "p_gg")
    for fn in (gw.epsilon, gw.eps_inverse):
        reaches_device_check(lambda: fn(c64(NG, NG), N, 5.0, Q, MILLER))
        raises_value(lambda: fn(c64(NG + 1, NG + 1), N, 5.0, Q, MILLER), "p_gg")
        raises_value(lambda: fn(c64(NG, NG), N, 5.0, Q, MILLER, out=c128(NG, NG - 1)), "eps")
        raises_value(lambda: fn(c64(NG, NG), N, 5.0, [0.0], MILLER), "q")
    raises_value(lambda: gw.eps_inverse_newton(c64(NG, NG + 1), N, 5.0, Q, MILLER), "p_gg")
    raises_value(lambda: gw.hpd_inverse(c128(3, 4)), "a")
    raises_value(lambda: gw.hpd_inverse(c128(3, 3), out=c128(4, 4)), "out")
    raises_value(lambda: gw.newton_inverse(c128(3, 3), out=c128(3, 2)), "out")


def test_batched_shapes():
    job = dict(psi_c=c64(3, NR), e_c=EC, q=[0.1, 0.0, 0.0], miller=MILLER, p_gg=c64(NG, NG))
    reaches_device_check(lambda: gw.polarizability_batched(c64(2, NR), EV, N, 5.0, [job]))
    raises_value(lambda: gw.polarizability_batched(c64(2, NR), EV, N, 5.0, [dict(job, e_c=EC[:1])]), "e_c")
    raises_value(lambda: gw.polarizability_batched(c64(2, NR), EV, N, 5.0, [dict(job, psi_c=c64(3, 7))]),
                 "grid points")
    raises_value(lambda: gw.polarizability_batched(c64(2, NR), EV, N, 5.0, [dict(job, p_gg=c64(2, 2))]), "p_gg")
    raises_value(lambda: gw.polarizability_batched(c64(2, NR), EV, N, 5.0,
                                                   [dict(job, eps_inv=c128(NG, 1))]), "eps_inv")
    raises_value(lambda: gw.polarizability_batched(c64(2, NR), EV[:1], N, 5.0, [job]), "e_v")


def test_other_entry_point_shapes():
    raises_value(lambda: gw.orbitals_to_grid(c64(2, 3), N, MILLER, out=c64(2, NR + 1)), "psi")
    raises_value(lambda: gw.orbitals_to_grid(c64(2, 4), N, MILLER), "coefficients")
    raises_value(lambda: gw.tail_features(c64(NG, NG + 1), N, 5.0, Q, MILLER, 4, 0.3), "p_gg")
    raises_value(lambda: gw.tail_features(c64(NG, NG), N, 5.0, Q, MILLER, 4, 0.3, out=f32(NG, 3)), "feat")
    raises_value(lambda: gw.tail_target(c64(NG, NG), c64(NG, NG + 1)), "p_trunc")
    raises_value(lambda: gw.plasmon_pole(c128(NG, NG), N, 5.0, Q, MILLER, c64(2, NR + 1)), "grid points")
    raises_value(lambda: gw.plasmon_pole(c128(NG, NG + 1), N, 5.0, Q, MILLER, c64(2, NR)), "eps_inv")
    modes, sig = c128(NG, 2), torch.zeros(2, dtype=torch.float64)
    raises_value(lambda: gw.pp_eps_inverse(c128(NG, NG), N, 5.0, Q, MILLER, modes, sig,
                                           torch.zeros(3, dtype=torch.float64), [0.1]), "omega")
    raises_value(lambda: gw.pp_eps_inverse(c128(NG, NG), N, 5.0, Q, MILLER, c128(NG + 1, 2), sig, sig, [0.1]),
                 "modes")
    raises_value(lambda: gw.sigma_static(c64(2, NR), c64(3, NR - 1), N, 5.0, Q, MILLER), "grid points")
    raises_value(lambda: gw.sigma_static(c64(2, NR), c64(3, NR), N, 5.0, Q, MILLER, eps_inv=c128(2, 2)), "eps_inv")
    raises_value(lambda: gw.sigma_sex_modes(c64(2, NR), c64(3, NR), N, MILLER, modes, torch.zeros(3)), "sigma")
