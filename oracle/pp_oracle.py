"""FP64 oracle of the plasmon-pole model of the dynamic inverse dielectric matrix.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's CPU
baseline, never by the library.  Each function is the plain definition of the paper's
section on the dynamic inverse dielectric matrix (vdLH-type plasmon poles), with LAPACK's
dense Hermitian eigensolver (through scipy), numpy's FFT and matrix product as the only
library steps.

Readings used here:

* Density: rho(r) = occ sum_v |psi_v(r)|^2 for grid-normalised orbitals, and
  rho_g = sum_r rho(r) exp(-i G_g.r), so rho_0 = occ * Nv is the electron count of the cell
  (this is the normalisation under which the printed sum rule, with V = 4 pi / (Omega |q+g|^2),
  reduces to the homogeneous-gas plasma frequency 4 pi n_e).  occ plays the role of the
  polarizability's prefactor p (1 spinless, 2 spin-degenerate).
* Mode frequency: the printed Eq.(ppfreq) divides by sigma_alpha, but S is negative
  semidefinite (eig(eps^-1) in (0, 1]) while the sum-rule matrix M below is positive
  semidefinite, so the printed ratio is <= 0.  Carrying the sum rule through the pole form
  Eq.(ppform) with a retarded pole gives sigma_alpha omega_alpha^2 = -(A^H M A)_aa, i.e.
  omega_alpha^2 = (A^H M A)_aa / |sigma_alpha|, which is what is used.
* Modes: the n_modes most negative eigenvalues of S (the largest screening strengths).
* Differences g - g' are taken on the grid (Miller indices modulo n), as every grid
  transform in this package is.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def density_r(psi_v, occupation: float = 1.0) -> np.ndarray:
    """rho(r) = occ sum_v |psi_v(r)|^2, float64 [N_r]."""
    psi_v = np.asarray(psi_v, np.complex128)
    return occupation * (np.abs(psi_v) ** 2).sum(axis=0)


def density_g(rho_r, n: Sequence[int], miller) -> np.ndarray:
    """rho_g = sum_r rho(r) exp(-i 2 pi (m1 i1/n1 + m2 i2/n2 + m3 i3/n3)) for each Miller triple
    (any integers: the grid makes them periodic), as a direct sum."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    r = np.arange(nr)
    i1, i2, i3 = r // (n[1] * n[2]), (r // n[2]) % n[1], r % n[2]
    m = np.asarray(miller, np.float64).reshape(-1, 3)
    out = np.empty(len(m), dtype=np.complex128)
    for s in range(0, len(m), 512):
        mm = m[s:s + 512]
        ph = np.outer(mm[:, 0], i1) / n[0] + np.outer(mm[:, 1], i2) / n[1] + np.outer(mm[:, 2], i3) / n[2]
        out[s:s + 512] = np.exp(-2j * np.pi * ph) @ np.asarray(rho_r, np.float64)
    return out


def density_g_grid(rho_r, n: Sequence[int]) -> np.ndarray:
    """rho_g for every grid frequency (index m mod n), by numpy's forward FFT: the same sum as
    density_g, evaluated for all m at once."""
    n = tuple(int(x) for x in n)
    return np.fft.fftn(np.asarray(rho_r, np.float64).reshape(n)).ravel()


def screening_part(eps_inv, sqrtv) -> np.ndarray:
    """S = sqrt(V) (eps^-1 - I) sqrt(V): the polarization part of the static W (W - V)."""
    sv = np.asarray(sqrtv, np.float64)
    e = np.asarray(eps_inv, np.complex128)
    return sv[:, None] * (e - np.eye(len(sv))) * sv[None, :]


def sum_rule_matrix(n: Sequence[int], a_bohr: float, q, miller, sqrtv, rho_r) -> np.ndarray:
    """M(g,g') = V(q+g) V(q+g') [(q+g).(q+g')] rho_{g-g'}, the right side of the Johnson sum rule
    without its -pi/2; (q+g) in 1/Bohr, V = sqrtv^2."""
    m = np.asarray(miller, np.int64)
    qm = (m + np.asarray(q, np.float64)[None, :]) * (2.0 * np.pi / a_bohr)
    v = np.asarray(sqrtv, np.float64) ** 2
    n = tuple(int(x) for x in n)
    rg = density_g_grid(rho_r, n)
    d = [(m[:, None, k] - m[None, :, k]) % n[k] for k in range(3)]
    rho = rg[(d[0] * n[1] + d[1]) * n[2] + d[2]]
    return v[:, None] * v[None, :] * (qm @ qm.T) * rho


def plasmon_pole(eps_inv, n: Sequence[int], a_bohr: float, q, miller, sqrtv, psi_v, occupation: float = 1.0,
                 n_modes: int = 8):
    """Eq.(eigdecomp) and Eq.(ppfreq): the n_modes most negative eigenpairs (sigma_a, A[:, a]) of S
    and their frequencies omega_a.  Returns (sigma [n_modes], omega [n_modes], A [ng][n_modes])."""
    import scipy.linalg
    s = screening_part(eps_inv, sqrtv)
    # ascending eigenvalues, so the first n_modes are the most negative
    w, a = scipy.linalg.eigh(0.5 * (s + np.conj(s).T), subset_by_index=[0, n_modes - 1])
    mm = sum_rule_matrix(n, a_bohr, q, miller, sqrtv, density_r(psi_v, occupation))
    num = np.real(np.sum(np.conj(a) * (mm @ a), axis=0))
    return w, np.sqrt(num / np.abs(w)), a


def pp_eps_inverse(eps_inv_static, sigma, omega, modes, sqrtv, freqs) -> np.ndarray:
    """Eq.(ppform) turned back into eps^-1(w) = I + V^-1/2 S(w) V^-1/2 for each frequency w, with
    S(w) = sum_a A_a sigma_a omega_a^2 / (omega_a^2 - w^2) A_a^H.  Rows and columns where
    sqrt(V) = 0 keep their static values.  Returns complex128 [len(freqs)][ng][ng]."""
    sv = np.asarray(sqrtv, np.float64)
    ok = sv > 0
    inv_sv = np.where(ok, 1.0 / np.where(ok, sv, 1.0), 0.0)
    a = np.asarray(modes, np.complex128)
    out = []
    for w in np.atleast_1d(freqs):
        c = np.asarray(sigma) * np.asarray(omega) ** 2 / (np.asarray(omega) ** 2 - w * w)
        sw = (a * c[None, :]) @ np.conj(a).T
        e = np.eye(len(sv), dtype=np.complex128) + inv_sv[:, None] * sw * inv_sv[None, :]
        e[~ok, :] = eps_inv_static[~ok, :]
        e[:, ~ok] = eps_inv_static[:, ~ok]
        out.append(e)
    return np.array(out)
