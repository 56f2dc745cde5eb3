"""Pins of the static self-energy oracle: the paper's real-space route for the bare exchange, the
plane-wave (Fock) closed form, completeness, the sign structure of both terms, and the agreement of
the T and eigen (zeta) forms of the screened exchange."""
import numpy as np

import gwsynth as gs
import oracle as orc
from oracle import pp_oracle as pp
from oracle import sigma_oracle as so


def test_real_space_route_equals_g_space():
    n = (5, 4, 3)
    rng = np.random.default_rng(0)
    psi = gs.random_unitary_orbitals(rng, 60)
    pn, pv = psi[:3], psi[3:7]
    q = np.array([0.15, -0.1, 0.2])
    miller = gs.sphere(n, r2=2.0, q=q)
    sv = orc.coulomb_sqrt(n, gs.cell_side(4), q, miller)
    ft = so.pair_transform(pn, pv, n, miller)
    a = so.sigma_x(ft, sv)
    b = so.sigma_x_real_space(pn, pv, n, miller, sv)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_plane_wave_fock_closed_form():
    """u_n, u_v plane waves: f~_g^{nv} = 1 where m_g = m_v - m_n, so Sigma_x is diagonal with
    -sum_v V(q + m_v - m_n) over the v whose difference lies in the sphere."""
    n = (8, 8, 8)
    q = np.array([0.11, 0.07, -0.05])
    a = gs.cell_side(8)
    mn = np.array([[0, 0, 0], [1, 0, 0], [0, 1, -1]])
    mv = np.array([[0, 0, 0], [-1, 0, 0], [1, 1, 0], [0, 0, 2], [3, 0, 0]])
    miller = gs.sphere(n, r2=5.0, q=q)
    sv = orc.coulomb_sqrt(n, a, q, miller)
    ft = so.pair_transform(gs.plane_wave_orbitals(n, mn), gs.plane_wave_orbitals(n, mv), n, miller)
    sx = so.sigma_x(ft, sv)
    inside = {tuple(m) for m in miller}
    b = 2 * np.pi / a
    for i, m1 in enumerate(mn):
        ref = 0.0
        for m2 in mv:
            d = m2 - m1
            if tuple(d) in inside:
                k = b * (q + d)
                ref -= 4 * np.pi / (a ** 3 * k @ k)
        assert abs(sx[i, i] - ref) < 1e-13 * abs(ref)
    assert np.max(np.abs(sx - np.diag(np.diag(sx)))) < 1e-13 * np.max(np.abs(sx))


def test_completeness():
    """With a complete occupied set, sum_v |f~_g^{nv}|^2 = 1, so Sigma_x = -(sum_g V_g) I."""
    n = (4, 4, 4)
    rng = np.random.default_rng(5)
    psi = gs.random_unitary_orbitals(rng, 64)
    q = np.array([0.2, 0.1, 0.05])
    miller = gs.sphere(n, r2=2.0, q=q)
    sv = orc.coulomb_sqrt(n, gs.cell_side(4), q, miller)
    sx = so.sigma_x(so.pair_transform(psi[:5], psi, n, miller), sv)
    assert np.max(np.abs(sx + np.sum(sv ** 2) * np.eye(5))) < 1e-12 * np.sum(sv ** 2)


def _screened_case():
    s = gs.make_system(8, 6, 40, r2_psi=6.0, q=(0.2, 0.1, 0.05), seed=3)
    pt = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    sv = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
    ei = orc.eps_inverse(orc.epsilon(0.5 * (pt + pt.conj().T), sv))
    return s, sv, ei


def test_signs_and_forms_of_the_screened_exchange():
    s, sv, ei = _screened_case()
    bands = np.concatenate([s.psi_v[-3:], s.psi_c[:3]])          # a band window around the gap
    ft = so.pair_transform(bands, s.psi_v, s.n, s.miller)
    sx = so.sigma_x(ft, sv)
    S = pp.screening_part(ei, sv)
    sse = so.sigma_sex(ft, S)
    assert np.max(np.abs(sx - sx.conj().T)) < 1e-14 * np.max(np.abs(sx))
    assert np.max(np.linalg.eigvalsh(sx)) < 1e-12 * np.max(np.abs(sx))          # bare exchange NSD
    assert np.max(np.abs(sse - sse.conj().T)) < 1e-14 * np.max(np.abs(sse))
    assert np.min(np.linalg.eigvalsh(sse)) > -1e-12 * np.max(np.abs(sse))       # S NSD makes it PSD
    # screening weakens exchange: the screened total Sigma_x + Sigma_sex lies between Sigma_x and 0
    tot = np.real(np.diag(sx + sse))
    assert np.all(tot < 0) and np.all(tot > np.real(np.diag(sx)))
    # S = diag(V) turns the screened form into the bare one
    assert np.max(np.abs(so.sigma_sex(ft, np.diag(sv ** 2)) - sx)) < 1e-13 * np.max(np.abs(sx))
    # the eigen form with every mode equals the T form; with a few modes it approaches it
    w, a = np.linalg.eigh(0.5 * (S + S.conj().T))
    assert np.max(np.abs(so.sigma_sex_modes(ft, a, w) - sse)) < 1e-12 * np.max(np.abs(sse))
    e8 = np.max(np.abs(so.sigma_sex_modes(ft, a[:, :8], w[:8]) - sse))
    e2 = np.max(np.abs(so.sigma_sex_modes(ft, a[:, :2], w[:2]) - sse))
    assert e8 < e2
