"""GPU parity of the plasmon-pole model against the FP64 oracle: mode strengths, vectors and sum-rule
frequencies from the block iteration (small, full-space and 410-vector cases), the homogeneous-gas
closed form, the pole-form eps^-1(w) with its mode convergence (the synthetic analogue of the
paper's 410 x 410 silicon figure), and the iteration limit."""
import numpy as np
import pytest

import gwsynth as gs
import oracle as orc
from oracle import pp_oracle as pp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_07772_amd as gw
    gw.load()
    return gw


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def gpu_eps_inv(gw, s):
    """eps^-1 by the library, for a system whose orbitals are already complex64-exact."""
    pv, pc = dev(s.psi_v.astype(np.complex64)), dev(s.psi_c.astype(np.complex64))
    pgg = gw.polarizability(pv, pc, s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)
    return gw.eps_inverse(pgg, s.n, s.a_bohr, s.q, s.miller), pv


def compare(gw, s, ei, pv, n_modes, occ=1.0, tol=1e-10):
    sig, om, a, its, res = gw.plasmon_pole(ei, s.n, s.a_bohr, s.q, s.miller, pv, occ, n_modes, tol=tol)
    torch.cuda.synchronize()
    sv = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
    e = ei.cpu().numpy()
    s_ref, o_ref, a_ref = pp.plasmon_pole(e, s.n, s.a_bohr, s.q, s.miller, sv, s.psi_v, occ, n_modes)
    sig, om, a = sig.cpu().numpy(), om.cpu().numpy(), a.cpu().numpy()
    e_sig = np.max(np.abs(sig - s_ref)) / abs(s_ref[0])
    e_om = np.max(np.abs(om - o_ref) / o_ref)
    overlap = np.abs(np.sum(np.conj(a_ref) * a, axis=0))         # |<a_ref, a>| per mode (phases are free)
    print(f"ng={len(sv)} modes={n_modes}: {its} iterations, residual {res:.1e}; sigma {e_sig:.1e}, "
          f"omega {e_om:.1e}, 1-overlap {np.max(1 - overlap):.1e}")
    return e_sig, e_om, overlap, its, (sig, om, a, s_ref, o_ref, a_ref, sv, e)


def test_small_system_modes(gw):
    s = gs.make_system(8, 6, 40, r2_psi=6.0, q=(0.2, 0.1, 0.05), seed=4).as_c64()
    ei, pv = gpu_eps_inv(gw, s)
    for nm in (1, 5, 8, 16):
        e_sig, e_om, ov, its, _ = compare(gw, s, ei, pv, nm, occ=2.0)
        # the residual bound 1e-10 gives eigenvalues to about its square and vectors to about 1e-10 / gap
        assert e_sig < 1e-12 and e_om < 1e-8 and np.min(ov) > 1 - 1e-8


def test_full_space_block_is_exact_in_one_iteration(gw):
    s = gs.make_system(6, 4, 20, r2_psi=4.0, q=(0.1, 0.2, 0.3), ng=30, seed=2).as_c64()
    ei, pv = gpu_eps_inv(gw, s)
    e_sig, e_om, ov, its, _ = compare(gw, s, ei, pv, 12)
    assert its == 1 and e_sig < 1e-13 and e_om < 1e-10 and np.min(ov) > 1 - 1e-10


def test_homogeneous_gas_closed_form(gw):
    n = (6, 6, 6)
    q = np.array([0.13, 0.07, 0.03])
    mv = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0]])
    mc = np.array([[1, 1, 0], [-1, 0, 2], [0, 0, 1], [2, -1, 1], [0, 2, -1], [-2, 1, 0], [1, -2, 2]])
    e_v = np.array([-0.31, -0.22, -0.12])
    e_c = np.array([0.15, 0.21, 0.33, 0.41, 0.52, 0.6, 0.75])
    a = gs.cell_side(6)
    miller = gs.sphere(n, r2=5.0, q=q)
    pv = dev(gs.plane_wave_orbitals(n, mv).astype(np.complex64))
    pc = dev(gs.plane_wave_orbitals(n, mc).astype(np.complex64))
    pgg = gw.polarizability(pv, pc, e_v, e_c, n, a, q, miller)
    ei = gw.eps_inverse(pgg, n, a, q, miller)
    occ, nm = 2.0, 6
    sig, om, modes, its, _ = gw.plasmon_pole(ei, n, a, q, miller, pv, occ, nm)
    sv = orc.coulomb_sqrt(n, a, q, miller)
    ptd = np.real(np.diag(pgg.cpu().numpy().astype(np.complex128)))
    eps_d = 1.0 - sv ** 2 * ptd
    sig_closed = np.sort(sv ** 2 * (1.0 / eps_d - 1.0))[:nm]
    sig = sig.cpu().numpy()
    assert np.max(np.abs(sig - sig_closed)) < 1e-10 * np.max(np.abs(sig_closed))
    idx = np.argmax(np.abs(modes.cpu().numpy()), axis=0)
    w2 = 4 * np.pi / a ** 3 * occ * 3 / (1.0 - 1.0 / eps_d[idx])
    # the density comes from complex64 orbitals: relative error at the FP32 level
    assert np.max(np.abs(om.cpu().numpy() ** 2 - w2) / w2) < 1e-6


def test_silicon_analogue_410_pole_form(gw):
    """410 G, q = pi/a (1,1,-1): modes and eps^-1(w) of the pole form with 1 and 5 modes against all
    410 (the oracle's full eigendecomposition), at frequencies below, between and above the poles."""
    s = gs.make_system(12, 8, 64, r2_psi=10.0, r2_p=25.0, q=(0.5, 0.5, -0.5), ng=410, seed=4).as_c64()
    ei, pv = gpu_eps_inv(gw, s)
    e_sig, e_om, ov, its, (sig, om, a, s_ref, o_ref, a_ref, sv, e) = compare(gw, s, ei, pv, 5)
    assert e_sig < 1e-12 and e_om < 1e-8 and np.min(ov) > 1 - 1e-8
    freqs = np.array([0.0, 0.3 * o_ref.min(), 0.5 * (o_ref[0] + o_ref[1]), 3.0 * o_ref.max()])
    got = gw.pp_eps_inverse(ei, s.n, s.a_bohr, s.q, s.miller, dev(a), dev(sig), dev(om), freqs).cpu().numpy()
    ref = pp.pp_eps_inverse(e, sig, om, a, sv, freqs)          # the same modes through the oracle's formula
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    s_all, o_all, a_all = pp.plasmon_pole(e, s.n, s.a_bohr, s.q, s.miller, sv, s.psi_v, 1.0, len(sv))
    g = int(np.argmax(np.abs(1.0 - np.diag(e))))
    lo = freqs[:2]
    all_modes = pp.pp_eps_inverse(e, s_all, o_all, a_all, sv, lo)[:, g, g]
    one = pp.pp_eps_inverse(e, s_ref[:1], o_ref[:1], a_ref[:, :1], sv, lo)[:, g, g]
    five = got[:2, g, g]
    print(f"eps^-1(w)[{g},{g}] at w = {lo}: all {all_modes.real}, 1 mode {one.real}, 5 modes {five.real}")
    assert np.all(np.abs(five - all_modes) < np.abs(one - all_modes) + 1e-15)
    assert abs(got[0, g, g] - e[g, g]) < 0.5 * abs(1.0 - e[g, g])      # 5 modes hold most of the static screening


def test_iteration_limit(gw):
    s = gs.make_system(8, 6, 40, r2_psi=6.0, q=(0.2, 0.1, 0.05), seed=4).as_c64()
    ei, pv = gpu_eps_inv(gw, s)
    with pytest.raises(gw.GwError, match="did not reach tol"):
        gw.plasmon_pole(ei, s.n, s.a_bohr, s.q, s.miller, pv, 1.0, 8, tol=1e-14, max_iter=2)
