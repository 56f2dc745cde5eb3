"""Pins of the plasmon-pole oracle: hand-computed densities, the homogeneous-gas closed form of the
mode strengths and frequencies, the eigen-structure of S, and the limits of the pole form."""
import numpy as np
import pytest

import gwsynth as gs
import oracle as orc
from oracle import pp_oracle as pp


def two_wave_density(n, occ, phase):
    """psi = (exp(i g1.r) + phase * exp(i g2.r)) / sqrt(2 N_r), g1 = (1,0,0), g2 = (0,1,0)."""
    psi = (gs.plane_wave_orbitals(n, np.array([[1, 0, 0]]))[0]
           + phase * gs.plane_wave_orbitals(n, np.array([[0, 1, 0]]))[0]) / np.sqrt(2.0)
    return pp.density_r(psi[None, :], occ)


def test_density_hand_values():
    n = (4, 4, 4)
    occ = 2.0
    # phase 1: |psi|^2 = (1 + cos((g1-g2).r)) / N_r, so rho_0 = occ, rho_{+-(1,-1,0)} = occ/2
    rho = two_wave_density(n, occ, 1.0)
    assert abs(rho[0] - 2 * occ / 64) < 1e-16                        # r = 0: cos 0 = 1
    assert abs(rho[16] - occ / 64) < 1e-16                           # r = (1,0,0): cos(pi/2) = 0
    g = pp.density_g(rho, n, np.array([[0, 0, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 0], [5, -1, 0]]))
    assert np.max(np.abs(g - [occ, occ / 2, occ / 2, 0, occ / 2])) < 1e-14   # (5,-1,0) = (1,-1,0) mod 4
    # phase i: |psi|^2 = (1 + sin((g1-g2).r)) / N_r, so rho_{g1-g2} = -i occ/2 and rho_{g2-g1} = +i occ/2
    rho = two_wave_density(n, occ, 1j)
    g = pp.density_g(rho, n, np.array([[1, -1, 0], [-1, 1, 0]]))
    assert np.max(np.abs(g - [-0.5j * occ, 0.5j * occ])) < 1e-14


def test_density_electron_count_and_reality():
    s = gs.make_system(6, 5, 7, r2_psi=4.0, seed=1)
    rho = pp.density_r(s.psi_v, 2.0)
    assert abs(rho.sum() - 10.0) < 1e-12
    m = gs.sphere(s.n, r2=3.0)
    g = pp.density_g(rho, s.n, m)
    gm = pp.density_g(rho, s.n, -m)
    assert abs(g[0] - 10.0) < 1e-12
    assert np.max(np.abs(gm - np.conj(g))) < 1e-13


def test_density_on_the_grid_equals_the_direct_sum():
    s = gs.make_system(6, 5, 7, r2_psi=4.0, seed=2)
    rho = pp.density_r(s.psi_v, 1.0)
    m = gs.sphere(s.n, r2=8.0)
    full = pp.density_g_grid(rho, s.n)
    idx = ((m[:, 0] % 6) * 6 + m[:, 1] % 6) * 6 + m[:, 2] % 6
    assert np.max(np.abs(full[idx] - pp.density_g(rho, s.n, m))) < 1e-13


def test_sum_rule_matrix_orientation():
    """M(g1, g2) carries rho_{g1-g2}: with the phase-i density above that is -i occ/2, not +i occ/2."""
    n = (4, 4, 4)
    a = 5.0
    q = np.array([0.1, 0.2, 0.3])
    miller = np.array([[1, 0, 0], [0, 1, 0]])
    sv = orc.coulomb_sqrt(n, a, q, miller)
    rho = two_wave_density(n, 1.0, 1j)
    mm = pp.sum_rule_matrix(n, a, q, miller, sv, rho)
    b = 2 * np.pi / a
    k1, k2 = b * (miller[0] + q), b * (miller[1] + q)
    v1, v2 = 4 * np.pi / (a ** 3 * k1 @ k1), 4 * np.pi / (a ** 3 * k2 @ k2)
    assert abs(mm[0, 1] - v1 * v2 * (k1 @ k2) * (-0.5j)) < 1e-14 * abs(mm[0, 1])
    assert abs(mm[0, 0] - v1 * v1 * (k1 @ k1) * 1.0) < 1e-14 * abs(mm[0, 0])
    assert np.max(np.abs(mm - np.conj(mm).T)) < 1e-16


def plane_wave_case():
    n = (6, 6, 6)
    q = np.array([0.13, 0.07, 0.03])
    mv = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0]])
    mc = np.array([[1, 1, 0], [-1, 0, 2], [0, 0, 1], [2, -1, 1], [0, 2, -1], [-2, 1, 0], [1, -2, 2]])
    e_v = np.array([-0.31, -0.22, -0.12])
    e_c = np.array([0.15, 0.21, 0.33, 0.41, 0.52, 0.6, 0.75])
    a = gs.cell_side(6)
    miller = gs.sphere(n, r2=5.0, q=q)
    pv, pc = gs.plane_wave_orbitals(n, mv), gs.plane_wave_orbitals(n, mc)
    pt = orc.to_sphere(orc.polarizability_r(pv, pc, e_v, e_c), n, miller)
    sv = orc.coulomb_sqrt(n, a, q, miller)
    ei = orc.eps_inverse(orc.epsilon(pt, sv))
    return n, q, a, miller, pv, sv, pt, ei


def test_homogeneous_gas_closed_form():
    """Plane-wave orbitals: P~ and eps are diagonal and the density is uniform (rho_g = occ Nv delta_g0),
    so sigma_g = V_g (1/eps_gg - 1) and omega_g^2 = (4 pi / Omega) occ Nv / (1 - 1/eps_gg)."""
    n, q, a, miller, pv, sv, pt, ei = plane_wave_case()
    assert np.max(np.abs(pt - np.diag(np.diag(pt)))) < 1e-12 * np.max(np.abs(pt))
    occ, nmod = 2.0, 6
    sigma, omega, modes = pp.plasmon_pole(ei, n, a, q, miller, sv, pv, occ, nmod)
    eps_d = 1.0 - sv ** 2 * np.real(np.diag(pt))
    sig_closed = sv ** 2 * (1.0 / eps_d - 1.0)
    order = np.argsort(sig_closed)
    assert np.max(np.abs(sigma - sig_closed[order[:nmod]])) < 1e-12 * np.max(np.abs(sig_closed))
    idx = np.argmax(np.abs(modes), axis=0)
    assert list(idx) == list(order[:nmod])
    w2 = 4 * np.pi / a ** 3 * occ * len(pv) / (1.0 - 1.0 / eps_d[idx])
    assert np.max(np.abs(omega ** 2 - w2) / w2) < 1e-12


def test_modes_structure_and_pole_form_limits():
    s = gs.make_system(8, 6, 40, r2_psi=6.0, q=(0.2, 0.1, 0.05), seed=3)
    pt = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    sv = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
    ei = orc.eps_inverse(orc.epsilon(0.5 * (pt + pt.conj().T), sv))
    ng = len(sv)
    sigma, omega, a = pp.plasmon_pole(ei, s.n, s.a_bohr, s.q, s.miller, sv, s.psi_v, 1.0, ng)
    S = pp.screening_part(ei, sv)
    assert np.all(sigma <= 1e-14 * np.max(np.abs(sigma)))                 # S is negative semidefinite
    assert np.max(np.abs(a.conj().T @ a - np.eye(ng))) < 1e-12
    assert np.max(np.abs((a * sigma) @ a.conj().T - S)) < 1e-13 * np.max(np.abs(S))
    assert np.all(np.isfinite(omega)) and np.all(omega > 0)
    # w = 0 with every mode gives back the static eps^-1; large w gives I
    e0 = pp.pp_eps_inverse(ei, sigma, omega, a, sv, [0.0])[0]
    assert np.max(np.abs(e0 - ei)) < 1e-12
    big = pp.pp_eps_inverse(ei, sigma, omega, a, sv, [1e6])[0]
    assert np.max(np.abs(big - np.eye(ng))) < 1e-6
    # a few modes already carry most of the static screening of the most screened diagonal element
    # (the head carries none here: with one orbital set for k and k+q the pair densities at G = 0 vanish)
    g = int(np.argmax(np.abs(1.0 - np.diag(ei))))
    s5 = pp.pp_eps_inverse(ei, sigma[:5], omega[:5], a[:, :5], sv, [0.0])[0]
    assert abs(s5[g, g] - ei[g, g]) < 0.5 * abs(1.0 - ei[g, g])
