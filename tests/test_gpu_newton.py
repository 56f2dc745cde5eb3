"""GPU tests of eps^-1 by the Newton iteration of Sec. 5.1 on the FP64 MFMA GEMM: a synthetic analogue
of the paper's 410 x 410 silicon case (q = pi/a (1,1,-1), tol 1e-11), a general complex matrix with a
ragged size, the iteration limit and the 1 x 1 case.  The oracle runs the same iteration in numpy
(iteration counts and histories must agree) and LU gives the exact inverse."""
import numpy as np
import pytest

import gwsynth as gs
import oracle as orc

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


def test_silicon_analogue_410(gw):
    """410 sphere vectors, q = pi/a (1,1,-1) = (1/2, 1/2, -1/2) in crystal units, tol 1e-11."""
    s = gs.make_system(12, 8, 64, r2_psi=10.0, r2_p=25.0, q=(0.5, 0.5, -0.5), ng=410, seed=4).as_c64()
    assert len(s.miller) == 410
    pv, pc = dev(s.psi_v.astype(np.complex64)), dev(s.psi_c.astype(np.complex64))
    pgg = gw.polarizability(pv, pc, s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)
    x, it, hist = gw.eps_inverse_newton(pgg, s.n, s.a_bohr, s.q, s.miller, tol=1e-11)
    chol = gw.eps_inverse(pgg, s.n, s.a_bohr, s.q, s.miller)
    torch.cuda.synchronize()
    pt = pgg.cpu().numpy().astype(np.complex128)
    eps = orc.epsilon(0.5 * (pt + pt.conj().T), orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller))
    x_ref, it_ref, hist_ref = orc.newton_schulz_inverse(eps, tol=1e-11)
    inv = orc.eps_inverse(eps)
    xg = x.cpu().numpy()
    print(f"Newton: {it} iterations (oracle {it_ref}), last change {hist[-1]:.1e}; "
          f"max|X - LU| {np.max(np.abs(xg - inv)):.1e}")
    assert abs(it - it_ref) <= 1 and hist[-1] < 1e-11
    # the early iterates are far from rounding level, so their changes must agree closely
    k = min(len(hist), len(hist_ref)) - 3
    assert np.allclose(hist[:k], hist_ref[:k], rtol=1e-8, atol=0)
    assert np.max(np.abs(xg - x_ref)) < 1e-11
    assert np.max(np.abs(xg - inv)) < 1e-10
    assert np.max(np.abs(xg - chol.cpu().numpy())) < 1e-10


@pytest.mark.parametrize("n", [1, 300])
def test_general_complex_matrix(gw, n):
    rng = np.random.default_rng(n)
    a = (3.0 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n))
    x, it, hist = gw.newton_inverse(dev(a), tol=1e-12)
    torch.cuda.synchronize()
    x_ref, it_ref, _ = orc.newton_schulz_inverse(a, tol=1e-12)
    xg = x.cpu().numpy()
    print(f"n={n}: {it} iterations (oracle {it_ref})")
    assert abs(it - it_ref) <= 1
    assert np.max(np.abs(xg - np.linalg.inv(a))) < 1e-11
    assert np.max(np.abs(a @ xg - np.eye(n))) < 1e-11


def test_iteration_limit_reports_and_keeps_last_iterate(gw):
    rng = np.random.default_rng(7)
    n = 130
    a = 2.0 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    out = torch.empty((n, n), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(gw.GwError, match="did not reach tol"):
        gw.newton_inverse(dev(a), tol=1e-12, max_iter=3, out=out)
    torch.cuda.synchronize()
    # three iterations from X_0 = alpha A^H, done by the oracle's own loop
    x3, it3, _ = orc.newton_schulz_inverse(a, tol=1e-300, max_iter=3)
    assert it3 == 3
    assert np.max(np.abs(out.cpu().numpy() - x3)) < 1e-12 * max(1.0, np.max(np.abs(x3)))
