"""Plain FP64 oracle of the static polarizability build (complex128 / float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function is the
plain definition from the paper, with numpy's matmul, FFT and dense linear
algebra as the only library steps, and no blocking, fusion or reordering
beyond what the definition states.

Readings of the paper used here (each one is also pinned by a CPU test):

* Prefactor p: Eq.(fdef) carries sqrt(2/(E_c - E_v)) (spin factor 2); the
  library takes p as an argument, default 1.
* Orientation: P(r,r') = -sum conj(f(r)) f(r'), as printed in the outer
  product below Eq.(fdef) with N_k = 1.  This is the orientation under which
  the real-space route equals the Adler-Wiser form Eq.(gpsaceP).
* Transform signs: the rows go to g with exp(-i G.r), the columns with
  exp(+i G'.r'), both as unnormalised sums over grid-normalised orbitals
  (Sec. 4.1 names both steps "IFFT", which read literally gives P(g,-g');
  with the paper's FFT being g -> r with exp(+i g.r), its inverse carries
  exp(-i g.r)).
* Coulomb: V(q+G) = 4 pi / (Omega |q+G|^2) in Hartree atomic units (e^2 = 1),
  Sec. 5.1.  Where |q+G| vanishes, sqrt(V) is taken as 0 and the head of
  epsilon is set to a caller-supplied value (default 1), which zeroes the
  wings; the paper avoids this case with a small nonzero q.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

__all__ = [
    "pair_products", "polarizability_r", "row_transform", "to_sphere", "coulomb_sqrt",
    "epsilon", "eps_inverse", "eps_inverse_cholesky", "newton_schulz_inverse", "adler_wiser",
    "rel_f", "grid_phase_index", "adler_wiser_selected", "orbitals_on_grid", "to_sphere_factored",
]


def rel_f(x, ref) -> float:
    """Relative Frobenius error ||x - ref||_F / ||ref||_F, in float64."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def _scales(e_v, e_c, prefactor):
    de = np.asarray(e_c, np.float64)[None, :] - np.asarray(e_v, np.float64)[:, None]   # [nv][nc]
    if np.any(de <= 0):
        raise ValueError("every E_c - E_v must be positive")
    return np.sqrt(prefactor / de)


def orbitals_on_grid(coeff, miller, n: Sequence[int], points=None) -> np.ndarray:
    """Sec. 4.1, the step from plane-wave coefficients to the orbitals' periodic parts on the
    real-space grid (Table 1's first row), as the direct sum
        psi_n(r) = N_r^(-1/2) sum_m c_nm exp(+2 pi i (m1 i1/n1 + m2 i2/n2 + m3 i3/n3)),
    r = (i1*n2 + i2)*n3 + i3.  coeff complex [nb][npw], miller int [npw][3].  Returns
    complex128 [nb][N_r], or [nb][len(points)] for the grid indices in `points`."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    r = np.arange(nr) if points is None else np.asarray(points, np.int64)
    i1, i2, i3 = r // (n[1] * n[2]), (r // n[2]) % n[1], r % n[2]
    m = np.asarray(miller, np.float64)
    phase = (np.outer(m[:, 0], i1) / n[0] + np.outer(m[:, 1], i2) / n[1] + np.outer(m[:, 2], i3) / n[2])
    return np.asarray(coeff, np.complex128) @ np.exp(2j * np.pi * phase) / np.sqrt(nr)


def pair_products(psi_v, psi_c, e_v, e_c, prefactor: float = 1.0) -> np.ndarray:
    """Eq.(fdef): f_vc(r) = conj(u_v(r)) u_c(r) sqrt(p / (E_c - E_v)).

    Returns complex128 [nv*nc][nr] with row index v*nc + c.
    """
    psi_v = np.asarray(psi_v, np.complex128)
    psi_c = np.asarray(psi_c, np.complex128)
    s = _scales(e_v, e_c, prefactor)
    f = np.conj(psi_v)[:, None, :] * psi_c[None, :, :] * s[:, :, None]
    return f.reshape(-1, psi_v.shape[1])


def polarizability_r(psi_v, psi_c, e_v, e_c, prefactor: float = 1.0,
                     rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Outer-product form below Eq.(fdef), N_k = 1: P(r,r') = -sum_{vc} conj(f_vc(r)) f_vc(r').

    The sum runs over v one occupied band at a time (the c-sum of each band is
    one matrix product).  With `rows`, only P[rows, :] is formed.
    """
    psi_v = np.asarray(psi_v, np.complex128)
    psi_c = np.asarray(psi_c, np.complex128)
    s = _scales(e_v, e_c, prefactor)
    nr = psi_v.shape[1]
    sel = np.arange(nr) if rows is None else np.asarray(rows)
    p = np.zeros((len(sel), nr), dtype=np.complex128)
    for v in range(psi_v.shape[0]):
        fv = np.conj(psi_v[v])[None, :] * psi_c * s[v][:, None]          # [nc][nr]
        p -= np.conj(fv[:, sel]).T @ fv
    return p


def grid_phase_index(n: Sequence[int], miller) -> np.ndarray:
    """Flat grid index of each Miller triple after wrapping m mod n (numpy FFT output order)."""
    m = np.asarray(miller, np.int64)
    return ((m[:, 0] % n[0]) * n[1] + (m[:, 1] % n[1])) * n[2] + (m[:, 2] % n[2])


def row_transform(p, n: Sequence[int], miller) -> np.ndarray:
    """First transform of Sec. 4.1: P^(g, r') = sum_r exp(-i G_g.r) P(r, r'), rows on the sphere."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    x = np.asarray(p, np.complex128).reshape(n + (nr,))
    xh = np.fft.fftn(x, axes=(0, 1, 2)).reshape(nr, nr)
    return xh[grid_phase_index(n, miller), :]


def to_sphere(p, n: Sequence[int], miller) -> np.ndarray:
    """Both transforms of Sec. 4.1:
    P~(g, g') = sum_{r, r'} exp(-i G_g.r) P(r, r') exp(+i G_g'.r'), on the ordered sphere."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    ph = row_transform(p, n, miller)                                          # [ng][nr]
    ng = ph.shape[0]
    y = np.fft.ifftn(ph.reshape((ng,) + n), axes=(1, 2, 3)).reshape(ng, nr) * nr
    return y[:, grid_phase_index(n, miller)]


def coulomb_sqrt(n: Sequence[int], a_bohr: float, q, miller) -> np.ndarray:
    """sqrt(V(q+G)) with V = 4 pi / (Omega |q+G|^2), Sec. 5.1, cubic cell of side a.

    |q+G| = (2 pi / a) |q + m| with q and m in crystal units.  Where |q+G| is
    below 1e-10 * 2pi/a the value is 0 (head handled by `epsilon`).
    """
    qm = np.asarray(miller, np.float64) + np.asarray(q, np.float64)[None, :]
    b = 2.0 * np.pi / a_bohr
    k2 = (b * b) * (qm ** 2).sum(axis=1)
    omega = a_bohr ** 3
    out = np.zeros(len(qm))
    ok = np.sqrt(k2) >= 1e-10 * b
    out[ok] = np.sqrt(4.0 * np.pi / (omega * k2[ok]))
    return out


def epsilon(ptilde, sqrtv, head: float = 1.0) -> np.ndarray:
    """Sec. 5.1: eps(g,g') = delta - sqrt(V(q+g)) P~(g,g') sqrt(V(q+g')), with the head rule."""
    sv = np.asarray(sqrtv, np.float64)
    eps = np.eye(len(sv), dtype=np.complex128) - sv[:, None] * np.asarray(ptilde, np.complex128) * sv[None, :]
    zero = np.nonzero(sv == 0.0)[0]
    for g in zero:
        eps[g, g] = head
    return eps


def eps_inverse(eps) -> np.ndarray:
    """epsilon^-1 by LU (numpy.linalg.inv)."""
    return np.linalg.inv(np.asarray(eps, np.complex128))


def eps_inverse_cholesky(eps) -> np.ndarray:
    """epsilon^-1 = L^-H L^-1 from the Cholesky factor eps = L L^H (eps Hermitian PD)."""
    l = np.linalg.cholesky(np.asarray(eps, np.complex128))
    y = np.linalg.solve(l, np.eye(l.shape[0], dtype=np.complex128))      # L^-1 (triangular, dense solve)
    return np.conj(y).T @ y


def newton_schulz_inverse(a, tol: float = 1e-11, max_iter: int = 200):
    """Newton iteration of Sec. 5.1: X_{n+1} = X_n (2I - A X_n), X_0 = alpha A^H,
    alpha = 1 / max_i sum_j |(A A^H)_ij|; stop when max |X_{n+1} - X_n| < tol.

    Returns (X, iterations, history of the max-abs change).  For complex A the
    start uses A^H (for Hermitian eps it is A itself), and the row sums take
    absolute values so that alpha <= 1 / sigma_max^2 and the iteration converges.
    """
    a = np.asarray(a, np.complex128)
    n = a.shape[0]
    aah = a @ np.conj(a).T
    alpha = 1.0 / np.max(np.abs(aah).sum(axis=1))
    x = alpha * np.conj(a).T
    hist = []
    eye2 = 2.0 * np.eye(n, dtype=np.complex128)
    for it in range(1, max_iter + 1):
        xn = x @ (eye2 - a @ x)
        d = float(np.max(np.abs(xn - x)))
        hist.append(d)
        x = xn
        if d < tol:
            return x, it, hist
    return x, max_iter, hist


def adler_wiser(psi_v, psi_c, e_v, e_c, n: Sequence[int], miller, prefactor: float = 1.0) -> np.ndarray:
    """Eq.(gpsaceP) with N_k = 1 and p in place of 2:
    P~(g,g') = p sum_{vc} M_vc(g) conj(M_vc(g')) / (E_v - E_c),
    M_vc(g) = sum_r exp(-i G_g.r) conj(u_c(r)) u_v(r)   (the transform of the pair product)."""
    n = tuple(int(x) for x in n)
    psi_v = np.asarray(psi_v, np.complex128)
    psi_c = np.asarray(psi_c, np.complex128)
    idx = grid_phase_index(n, miller)
    ng = len(idx)
    out = np.zeros((ng, ng), dtype=np.complex128)
    de = np.asarray(e_c, np.float64)[None, :] - np.asarray(e_v, np.float64)[:, None]
    for v in range(psi_v.shape[0]):
        prod = np.conj(psi_c) * psi_v[v][None, :]                              # [nc][nr]
        m = np.fft.fftn(prod.reshape((-1,) + n), axes=(1, 2, 3)).reshape(len(psi_c), -1)[:, idx]  # [nc][ng]
        w = prefactor / (-de[v])                                                # p / (E_v - E_c)
        out += (m * w[:, None]).T @ np.conj(m)
    return out


def adler_wiser_selected(psi_v, psi_c, e_v, e_c, n: Sequence[int], miller_sel, prefactor: float = 1.0) -> np.ndarray:
    """Eq.(gpsaceP) on a subset of sphere vectors: P~(g, g') for g, g' in `miller_sel`, with
    M_vc(g) = sum_r exp(-i G_g.r) conj(u_c(r)) u_v(r) summed directly over the grid (no FFT),
    one occupied band at a time.  For checks at sizes where the full P(r, r') is out of reach."""
    n = tuple(int(x) for x in n)
    psi_v = np.asarray(psi_v)
    psi_c = np.asarray(psi_c)
    m = np.asarray(miller_sel, np.float64)
    i1, i2, i3 = np.meshgrid(*(np.arange(x) for x in n), indexing="ij")
    ph = (np.multiply.outer(m[:, 0], i1.ravel()) / n[0] + np.multiply.outer(m[:, 1], i2.ravel()) / n[1]
          + np.multiply.outer(m[:, 2], i3.ravel()) / n[2])
    e = np.exp(-2j * np.pi * ph).T                                          # [nr][nsel]
    de = np.asarray(e_c, np.float64)[None, :] - np.asarray(e_v, np.float64)[:, None]
    out = np.zeros((len(m), len(m)), dtype=np.complex128)
    for v in range(psi_v.shape[0]):
        prod = np.conj(psi_c).astype(np.complex128) * psi_v[v].astype(np.complex128)[None, :]   # [nc][nr]
        mm = prod @ e                                                         # [nc][nsel]
        w = prefactor / (-de[v])
        out += (mm * w[:, None]).T @ np.conj(mm)
    return out


def to_sphere_factored(a, b, n: Sequence[int], miller_rows, miller_cols=None) -> np.ndarray:
    """Both transforms of Sec. 4.1 for a matrix given by factors, P(r, r') = sum_k a_k(r) conj(b_k(r'))
    (a, b complex [R][N_r]), on selected sphere vectors:
        P~(g, g') = sum_{r, r'} exp(-i G_g.r) P(r, r') exp(+i G_g'.r')
                  = sum_k [sum_r exp(-i G_g.r) a_k(r)] conj[sum_r' exp(-i G_g'.r') b_k(r')],
    with every grid sum written out directly (no FFT), for sizes where P itself is out of reach.
    Rows g run over miller_rows, columns g' over miller_cols (default: the same list)."""
    n = tuple(int(x) for x in n)
    mc = miller_rows if miller_cols is None else miller_cols
    i1, i2, i3 = np.meshgrid(*(np.arange(x) for x in n), indexing="ij")
    i1, i2, i3 = i1.ravel(), i2.ravel(), i3.ravel()

    def kernel(miller):                                   # exp(-i G_g.r) as [N_r][len(miller)]
        m = np.asarray(miller, np.float64)
        ph = (np.multiply.outer(i1, m[:, 0]) / n[0] + np.multiply.outer(i2, m[:, 1]) / n[1]
              + np.multiply.outer(i3, m[:, 2]) / n[2])
        return np.exp(-2j * np.pi * ph)

    ah = np.asarray(a, np.complex128) @ kernel(miller_rows)     # [R][n_rows]
    bh = np.asarray(b, np.complex128) @ kernel(mc)              # [R][n_cols]
    return ah.T @ np.conj(bh)
