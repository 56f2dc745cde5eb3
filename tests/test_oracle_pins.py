"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: a
brute-force sum of a different equation, an independent route, a closed form,
an invariant or a physical constant.  Each names the passage it pins.
"""
import json
import os

import numpy as np
import pytest
from scipy.special import erfc

import gwsynth as gs
import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_system(n=3, nv=2, nc=3, r2=2.0, seed=7, q=(0.0, 0.0, 0.0)):
    return gs.make_system(n, nv, nc, r2_psi=r2, seed=seed, q=q)


# --- P1: literal quadruple sum of Eq.(staticpol) -----------------------------------------
def test_p1_literal_staticpol_quadruple_loop():
    """Eq.(staticpol) summed literally (N_k = 1, prefactor p in place of 2): pins orientation and scale."""
    for n, p in ((3, 1.0), (4, 2.0)):
        s = gs.make_system(n, 2, 3, r2_psi=3.0, seed=11 + n)
        nr = s.nr
        lit = np.zeros((nr, nr), dtype=np.complex128)
        for r in range(nr):
            for rp in range(nr):
                acc = 0.0 + 0.0j
                for v in range(s.nv):
                    for c in range(s.nc):
                        acc += (np.conj(s.psi_c[c, r]) * s.psi_v[v, r] * np.conj(s.psi_v[v, rp]) * s.psi_c[c, rp]
                                / (s.e_c[c] - s.e_v[v]))
                lit[r, rp] = -p * acc
        got = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=p)
        assert orc.rel_f(got, lit) < 1e-13


def test_p1_pair_products_literal():
    """Eq.(fdef) element by element."""
    s = tiny_system()
    f = orc.pair_products(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=2.0)
    for v in range(s.nv):
        for c in range(s.nc):
            for r in range(s.nr):
                want = np.conj(s.psi_v[v, r]) * s.psi_c[c, r] * np.sqrt(2.0 / (s.e_c[c] - s.e_v[v]))
                assert abs(f[v * s.nc + c, r] - want) <= 1e-15 * max(1.0, abs(want))


# --- P2: r-space route == Adler-Wiser (Eq.(gpsaceP)) --------------------------------------
@pytest.mark.parametrize("n,nv,nc,r2,q", [(6, 3, 7, 4.0, (0, 0, 0)), (8, 4, 9, 6.0, (0.1, -0.2, 0.05)),
                                          (12, 8, 64, 10.0, (0, 0, 0))])
def test_p2_rspace_equals_adler_wiser(n, nv, nc, r2, q):
    s = gs.make_system(n, nv, nc, r2_psi=r2, seed=3, q=q)
    p = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    pt = orc.to_sphere(p, s.n, s.miller)
    aw = orc.adler_wiser(s.psi_v, s.psi_c, s.e_v, s.e_c, s.n, s.miller)
    assert orc.rel_f(pt, aw) < 1e-13


def test_p2_selected_entries_equal_full_route():
    """The direct-sum Adler-Wiser on a subset of G equals the FFT-based full route on that subset."""
    s = gs.make_system(8, 3, 10, r2_psi=6.0, seed=23, q=(0.05, 0.0, -0.1))
    sel = np.array([0, 3, 7, 20, len(s.miller) - 1])
    full = orc.adler_wiser(s.psi_v, s.psi_c, s.e_v, s.e_c, s.n, s.miller)
    part = orc.adler_wiser_selected(s.psi_v, s.psi_c, s.e_v, s.e_c, s.n, s.miller[sel])
    assert np.max(np.abs(part - full[np.ix_(sel, sel)])) < 1e-13 * np.max(np.abs(full))


# --- P3: plane-wave closed form -------------------------------------------------------
def test_p3_plane_wave_closed_form():
    """Plane-wave orbitals: P~ is diagonal with P~(g,g) = -p sum_{vc: m_v - m_c = m_g (mod n)} 1/(E_c-E_v).
    Pins the exponent signs, the absence of N_r factors and the conjugation orientation."""
    n = (6, 6, 6)
    mv = np.array([[0, 0, 0], [1, 0, 0], [0, 2, -1]])
    mc = np.array([[1, 1, 0], [-1, 0, 2], [2, -1, 1], [0, 0, 1], [-2, 1, 1]])
    psi_v = gs.plane_wave_orbitals(n, mv)
    psi_c = gs.plane_wave_orbitals(n, mc)
    rng = np.random.default_rng(5)
    e_v = -rng.uniform(0.1, 0.5, len(mv))
    e_c = rng.uniform(0.1, 0.9, len(mc))
    p = 2.0
    mill = gs.sphere(n, r2=12.0)
    pt = orc.to_sphere(orc.polarizability_r(psi_v, psi_c, e_v, e_c, prefactor=p), n, mill)
    want = np.zeros(len(mill), dtype=np.complex128)
    for iv, a in enumerate(mv):
        for ic, b in enumerate(mc):
            d = (a - b) % 6
            for g, m in enumerate(mill):
                if np.all(m % 6 == d):
                    want[g] += -p / (e_c[ic] - e_v[iv])
    assert np.count_nonzero(np.abs(want) > 0) >= 8           # the case is not trivial
    assert np.max(np.abs(pt - np.diag(want))) < 1e-12
    # the opposite assignment (m_c - m_v) must NOT match: the pin can tell orientation apart
    wrong = np.zeros(len(mill), dtype=np.complex128)
    for iv, a in enumerate(mv):
        for ic, b in enumerate(mc):
            for g, m in enumerate(mill):
                if np.all(m % 6 == (b - a) % 6):
                    wrong[g] += -p / (e_c[ic] - e_v[iv])
    assert np.max(np.abs(pt - np.diag(wrong))) > 1e-3


# --- P4: completeness closed form -----------------------------------------------------
def test_p4_completeness_closed_form():
    """All N_r grid bands, one common gap D: P = -(p/D)(rho(r) delta_rr' - |rho(r,r')|^2)."""
    n = 4
    nr = n ** 3
    rng = np.random.default_rng(21)
    u = gs.random_unitary_orbitals(rng, nr)
    nv = 13
    psi_v, psi_c = u[:nv], u[nv:]
    gap, p = 0.37, 1.5
    e_v = np.full(nv, -0.2)
    e_c = np.full(nr - nv, -0.2 + gap)
    got = orc.polarizability_r(psi_v, psi_c, e_v, e_c, prefactor=p)
    rho = psi_v.T @ np.conj(psi_v)                     # rho(r, r') = sum_v psi_v(r) psi_v(r')^*
    want = -(p / gap) * (np.diag(np.diag(rho).real) - np.abs(rho) ** 2)
    assert np.max(np.abs(got - want)) < 1e-14 * nr
    assert orc.rel_f(got, want) < 1e-12


# --- P5: trace identity ---------------------------------------------------------------
def test_p5_trace_identity():
    s = gs.make_system(6, 3, 11, r2_psi=4.0, seed=9)
    p = 2.0
    got = np.trace(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=p))
    want = 0.0
    for v in range(s.nv):
        for c in range(s.nc):
            want += p * np.sum(np.abs(np.conj(s.psi_v[v]) * s.psi_c[c]) ** 2) / (s.e_v[v] - s.e_c[c])
    assert abs(got.imag) < 1e-15 * abs(want)
    assert abs(got.real - want) < 1e-13 * abs(want)


# --- P6: Hermitian, negative semidefinite ---------------------------------------------
def test_p6_hermitian_nsd():
    s = gs.make_system(8, 4, 20, r2_psi=6.0, seed=2, q=(0.05, 0.1, -0.1))
    p = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    assert np.max(np.abs(p - np.conj(p).T)) <= 1e-15 * np.max(np.abs(p))
    assert np.linalg.eigvalsh(p).max() <= 1e-12 * np.max(np.abs(p))
    pt = orc.to_sphere(p, s.n, s.miller)
    assert np.max(np.abs(pt - np.conj(pt).T)) <= 1e-13 * np.max(np.abs(pt))
    assert np.linalg.eigvalsh(0.5 * (pt + np.conj(pt).T)).max() <= 1e-12 * np.max(np.abs(pt))


# --- P7: Parseval with the full grid as the sphere -----------------------------------------
def test_p7_parseval_full_grid():
    n = (5, 5, 5)                                     # odd n: every Miller triple obeys |m| < n/2
    s = gs.make_system(5, 3, 9, r2_psi=3.0, seed=4)
    full = gs.sphere(n, r2=1e9)
    assert len(full) == 125
    p = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    pt = orc.to_sphere(p, n, full)
    assert abs(np.trace(pt) - 125 * np.trace(p)) < 1e-12 * abs(125 * np.trace(p))
    assert abs(np.linalg.norm(pt) - 125 * np.linalg.norm(p)) < 1e-12 * 125 * np.linalg.norm(p)


# --- P8: head and wings vanish at q = 0 -------------------------------------------------
def test_p8_head_wings_zero_at_q0():
    s = gs.make_system(8, 4, 12, r2_psi=6.0, seed=8)
    assert np.all(s.miller[0] == 0)
    pt = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    scale = np.max(np.abs(pt))
    assert np.max(np.abs(pt[0, :])) < 1e-14 * scale
    assert np.max(np.abs(pt[:, 0])) < 1e-14 * scale


# --- P9 / P10: linearity and energy handling -----------------------------------------------
def test_p9_linearity_over_occupied_sets():
    s = gs.make_system(6, 5, 8, r2_psi=4.0, seed=12)
    full = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    a = orc.polarizability_r(s.psi_v[:2], s.psi_c, s.e_v[:2], s.e_c)
    b = orc.polarizability_r(s.psi_v[2:], s.psi_c, s.e_v[2:], s.e_c)
    assert orc.rel_f(a + b, full) < 1e-14
    c1 = orc.polarizability_r(s.psi_v, s.psi_c[:3], s.e_v, s.e_c[:3])
    c2 = orc.polarizability_r(s.psi_v, s.psi_c[3:], s.e_v, s.e_c[3:])
    assert orc.rel_f(c1 + c2, full) < 1e-14


def test_p10_energy_scale_and_shift():
    s = gs.make_system(6, 3, 7, r2_psi=4.0, seed=13)
    base = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    scaled = orc.polarizability_r(s.psi_v, s.psi_c, 2.5 * s.e_v, 2.5 * s.e_c)
    shifted = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v + 0.3, s.e_c + 0.3)
    assert orc.rel_f(scaled * 2.5, base) < 1e-14
    assert orc.rel_f(shifted, base) < 1e-13


def test_invalid_energies_rejected():
    s = tiny_system()
    with pytest.raises(ValueError):
        orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, np.full(s.nc, s.e_v.max()))


# --- Coulomb kernel: Madelung constant of the simple-cubic lattice ---------------------------
def test_coulomb_kernel_madelung():
    """sum_{G!=0} V(G) exp(-s^2 G^2) = 1/(s sqrt(pi)) - xi/L + 4 pi s^2/Omega - sum_{R!=0} erfc(R/2s)/R
    (Ewald split of the periodic Coulomb potential with background; xi is the simple-cubic Madelung constant).
    Pins 4 pi, Omega, the 2 pi / a reciprocal scale and the square of |q+G| in the Coulomb form."""
    xi = json.load(open(os.path.join(GOLDEN, "constants.json")))["madelung_simple_cubic_with_background"]["value"]
    n = (23, 23, 23)
    mill = gs.sphere(n, r2=1e9)
    for a in (7.3, 10.26):
        sv = orc.coulomb_sqrt(n, a, (0.0, 0.0, 0.0), mill)
        g2 = (2 * np.pi / a) ** 2 * (mill.astype(np.float64) ** 2).sum(axis=1)
        for sig in (a / 10.0, a / 8.0):
            s_sum = np.sum(sv ** 2 * np.exp(-sig ** 2 * g2))
            ax = np.arange(-2, 3)
            img = a * np.sqrt((np.stack(np.meshgrid(ax, ax, ax, indexing="ij")) ** 2).sum(axis=0)).ravel()
            img = img[img > 0]
            real_space = np.sum(erfc(img / (2 * sig)) / img)
            want = 1.0 / (sig * np.sqrt(np.pi)) - xi / a + 4 * np.pi * sig ** 2 / a ** 3 - real_space
            assert abs(s_sum - want) < 1e-12 * abs(want), (a, sig, s_sum, want)


def test_coulomb_head_rule():
    n = (8, 8, 8)
    mill = gs.sphere(n, r2=4.0)
    sv = orc.coulomb_sqrt(n, 6.84, (0, 0, 0), mill)
    assert sv[0] == 0.0 and np.all(sv[1:] > 0)
    sv_q = orc.coulomb_sqrt(n, 6.84, (0.0, 0.0, 0.001), gs.sphere(n, r2=4.0, q=(0, 0, 0.001)))
    assert np.all(sv_q > 0)


# --- P11: epsilon and its inverse ------------------------------------------------------
def _eps_case(q=(0.0, 0.0, 0.0), head=1.0):
    s = gs.make_system(8, 4, 24, r2_psi=6.0, seed=31, q=q)
    pt = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    sv = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
    return s, pt, sv, orc.epsilon(pt, sv, head)


@pytest.mark.parametrize("q", [(0.0, 0.0, 0.0), (0.0, 0.0, 0.001), (0.2, 0.1, 0.05)])
def test_p11_epsilon_structure_and_inverse(q):
    s, pt, sv, eps = _eps_case(q)
    # (at tiny |q| the head carries V(q) ~ 1/|q|^2 times rounding noise of P~(0,0))
    assert np.max(np.abs(eps - np.conj(eps).T)) < 1e-12 * np.max(np.abs(eps))
    w = np.linalg.eigvalsh(0.5 * (eps + np.conj(eps).T))
    assert w.min() >= 1.0 - 1e-12
    # the symmetric form of Sec. 5.1 is similar to the RPA form of Sec. 2, eps = 1 - V P~
    ok = sv > 0
    ns = np.eye(ok.sum()) - (sv[ok] ** 2)[:, None] * pt[np.ix_(ok, ok)]
    w_ns = np.sort(np.linalg.eigvals(ns).real)
    w_sym = np.sort(np.linalg.eigvalsh(eps[np.ix_(ok, ok)]))
    assert np.max(np.abs(w_ns - w_sym)) < 1e-11 * w_sym.max()
    inv = orc.eps_inverse(eps)
    assert np.max(np.abs(eps @ inv - np.eye(len(eps)))) < 1e-12
    assert orc.rel_f(orc.eps_inverse_cholesky(eps), inv) < 1e-13
    x, it, hist = orc.newton_schulz_inverse(eps, tol=1e-11)
    assert hist[-1] < 1e-11 and it < 60
    assert np.max(np.abs(x - inv)) < 1e-10
    wi = np.linalg.eigvalsh(0.5 * (inv + np.conj(inv).T))
    assert wi.max() <= 1.0 + 1e-12 and wi.min() > 0.0


def test_p11_head_value_and_wings():
    s, pt, sv, eps = _eps_case((0.0, 0.0, 0.0), head=2.5)
    assert sv[0] == 0.0
    assert eps[0, 0] == 2.5
    assert np.all(eps[0, 1:] == 0) and np.all(eps[1:, 0] == 0)
    inv = orc.eps_inverse(eps)
    assert abs(inv[0, 0] - 1 / 2.5) < 1e-15


def test_plane_wave_epsilon_diagonal():
    """With plane-wave orbitals P~ is diagonal, so eps and eps^-1 are diagonal: 1/(1 - V(g) P~(g,g))."""
    n = (6, 6, 6)
    mv = np.array([[0, 0, 0], [1, 0, 0]])
    mc = np.array([[1, 1, 0], [-1, 0, 2], [0, 0, 1]])
    e_v, e_c = np.array([-0.3, -0.1]), np.array([0.2, 0.4, 0.5])
    mill = gs.sphere(n, r2=6.0, q=(0.0, 0.0, 0.01))
    pt = orc.to_sphere(orc.polarizability_r(gs.plane_wave_orbitals(n, mv), gs.plane_wave_orbitals(n, mc),
                                            e_v, e_c), n, mill)
    sv = orc.coulomb_sqrt(n, 5.13, (0, 0, 0.01), mill)
    inv = orc.eps_inverse(orc.epsilon(pt, sv))
    d = 1.0 / (1.0 - sv ** 2 * np.diag(pt).real)
    assert np.max(np.abs(inv - np.diag(d))) < 1e-12


# --- generator facts the workloads rely on -----------------------------------------------
def test_generator_orthonormal_and_sphere_counts():
    s = gs.make_system(12, 8, 64, r2_psi=10.0, seed=0)
    psi = np.concatenate([s.psi_v, s.psi_c])
    assert np.max(np.abs(psi @ np.conj(psi).T - np.eye(72))) < 1e-13
    assert s.ng == 147
    # brute-force lattice-point counts of the spheres used by the workloads
    for r2, want in ((10, 147), (36, 925), (81, 3071), (98, 4067)):
        k = int(np.floor(np.sqrt(r2)))
        ax = np.arange(-k, k + 1)
        cnt = sum(1 for a in ax for b in ax for c in ax if a * a + b * b + c * c <= r2)
        assert cnt == want
    assert s.e_c.min() - s.e_v.max() >= 1.0 / gs.HARTREE_EV - 1e-15
    again = gs.make_system(12, 8, 64, r2_psi=10.0, seed=0)
    assert np.array_equal(again.psi_c, s.psi_c)


def test_sphere_order_and_count_rule():
    q = (0.0625, 0.03125, 0.015625)
    m = gs.sphere((32, 32, 32), q=q, count=2500)
    d2 = ((m + np.array(q)) ** 2).sum(axis=1)
    assert len(m) == 2500 and np.all(np.diff(d2) >= 0)
    assert len({tuple(x) for x in m}) == 2500


def test_orbitals_on_grid_hand_values():
    """One plane wave m = (1, 0, 0) on a 4^3 grid: psi(i1, i2, i3) = i^{i1} / 8 (exp(+i pi/2 i1) / sqrt(64))."""
    c = np.array([[1.0 + 0j]])
    psi = orc.orbitals_on_grid(c, np.array([[1, 0, 0]]), (4, 4, 4))[0]
    assert abs(psi[0] - 1 / 8) < 1e-16
    assert abs(psi[16] - 1j / 8) < 1e-16           # r = (1, 0, 0)
    assert abs(psi[32] + 1 / 8) < 1e-16            # r = (2, 0, 0)
    assert abs(psi[1] - 1 / 8) < 1e-16             # r = (0, 0, 1): m3 = 0, no phase
    # m = (0, 1, -1) on 4 x 5 x 6, r = (0, 2, 3): exp(2 pi i (2/5 - 3/6)) / sqrt(120)
    psi = orc.orbitals_on_grid(c, np.array([[0, 1, -1]]), (4, 5, 6), points=[2 * 6 + 3])[0, 0]
    assert abs(psi - np.exp(2j * np.pi * (0.4 - 0.5)) / np.sqrt(120)) < 1e-15


def test_orbitals_on_grid_equals_inverse_fft_on_a_non_cubic_grid():
    """Special case that reduces to a library routine: numpy's inverse FFT times sqrt(N_r); the
    6 x 5 x 4 grid catches a swapped axis, and the sign of the exponent a conjugation."""
    n = (6, 5, 4)
    rng = np.random.default_rng(3)
    mp = gs.sphere(n, r2=3.0)
    c = rng.standard_normal((3, len(mp))) + 1j * rng.standard_normal((3, len(mp)))
    box = np.zeros((3,) + n, dtype=np.complex128)
    for j, m in enumerate(mp):
        box[:, m[0] % n[0], m[1] % n[1], m[2] % n[2]] = c[:, j]
    ref = np.fft.ifftn(box, axes=(1, 2, 3)).reshape(3, -1) * np.sqrt(120)
    got = orc.orbitals_on_grid(c, mp, n)
    assert np.max(np.abs(got - ref)) < 1e-14
    # sampled points equal the full transform's columns
    pts = [0, 7, 119]
    assert np.max(np.abs(orc.orbitals_on_grid(c, mp, n, points=pts) - got[:, pts])) < 1e-15


def test_orbitals_on_grid_orthonormal_and_equal_to_generator():
    """Orthonormal coefficient vectors give grid-orthonormal orbitals (Parseval), and the
    direct sum equals the generator's numpy-FFT orbitals for the same draws."""
    s = gs.make_system(8, 4, 12, r2_psi=6.0, seed=5)
    psi = orc.orbitals_on_grid(s.coeff, s.pw_miller, s.n)
    assert np.max(np.abs(psi @ psi.conj().T - np.eye(16))) < 1e-13
    assert np.max(np.abs(psi[:4] - s.psi_v)) < 1e-14 and np.max(np.abs(psi[4:] - s.psi_c)) < 1e-14


# --- both transforms of a factored P (sampled-entry route for large grids) --------------------
def test_to_sphere_factored_plane_wave_closed_form():
    """P(r,r') = exp(+i G_a.r) exp(-i G_b.r'): the two transforms of Sec. 4.1 give N_r^2 at (g, g') =
    (a, b) and zero elsewhere.  Pins the exponent signs of both sides and the absence of any
    normalisation, independently of the FFT route."""
    n = (5, 4, 6)
    nr = 120
    mill = gs.sphere(n, r2=3.0, q=(0.1, 0.0, -0.2))
    ia, ib = 4, 9
    i1, i2, i3 = np.meshgrid(*(np.arange(x) for x in n), indexing="ij")
    def pw(m):
        return np.exp(2j * np.pi * (m[0] * i1 / n[0] + m[1] * i2 / n[1] + m[2] * i3 / n[2])).ravel()
    pt = orc.to_sphere_factored(pw(mill[ia])[None, :], pw(mill[ib])[None, :], n, mill)
    want = np.zeros((len(mill), len(mill)), dtype=np.complex128)
    want[ia, ib] = nr * nr
    assert np.max(np.abs(pt - want)) < 1e-9


def test_to_sphere_factored_equals_dense_route():
    """On a non-cubic grid with q != 0, the factored direct sums equal the FFT route applied to the dense
    P = sum_k a_k b_k^H, on a rectangular block of rows and columns."""
    n = (6, 5, 4)
    rng = np.random.default_rng(31)
    a = rng.standard_normal((3, 120)) + 1j * rng.standard_normal((3, 120))
    b = rng.standard_normal((3, 120)) + 1j * rng.standard_normal((3, 120))
    mill = gs.sphere(n, r2=4.0, q=(0.0, 0.3, 0.1))
    dense = orc.to_sphere(a.T @ np.conj(b), n, mill)
    rows, cols = np.array([0, 2, 5, len(mill) - 1]), np.array([1, 3, 4, 7, 11])
    got = orc.to_sphere_factored(a, b, n, mill[rows], mill[cols])
    assert np.max(np.abs(got - dense[np.ix_(rows, cols)])) < 1e-12 * np.max(np.abs(dense))
