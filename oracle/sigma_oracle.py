"""FP64 oracle of the static self-energy matrix elements in g-space: bare exchange and static screened
exchange.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.  Each function is the plain
definition from the paper's self-energy section (g-space approach for the bare exchange, the
T-matrix and the eigen (zeta) forms for the screened exchange), with numpy's FFT and matrix product
as the only library steps; `sigma_x_real_space` is the paper's second (real-space) route, kept as
an independent cross-check.

Conventions: orbitals are grid-normalised, so an integral over the cell of a product of two
orbitals is the plain grid sum; f~_g^{nv} = sum_r exp(-i G_g.r) conj(u_n(r)) u_v(r) (the transform
direction of the polarizability's row transform); V = 4 pi / (Omega |q+g|^2) (sqrtv squared).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .gw_oracle import grid_phase_index


def pair_transform(psi_n, psi_v, n: Sequence[int], miller) -> np.ndarray:
    """f~[n][v][g] = sum_r exp(-i G_g.r) conj(u_n(r)) u_v(r), on the ordered sphere."""
    n = tuple(int(x) for x in n)
    psi_n = np.asarray(psi_n, np.complex128)
    psi_v = np.asarray(psi_v, np.complex128)
    idx = grid_phase_index(n, miller)
    prod = np.conj(psi_n)[:, None, :] * psi_v[None, :, :]                     # [nn][nv][nr]
    ft = np.fft.fftn(prod.reshape(prod.shape[:2] + n), axes=(2, 3, 4)).reshape(prod.shape[:2] + (-1,))
    return ft[:, :, idx]


def sigma_x(ft, sqrtv) -> np.ndarray:
    """Bare exchange, g-space form: Sigma_x(n,n') = -sum_g V(q+g) sum_v f~_g^{nv} conj(f~_g^{n'v})."""
    v = np.asarray(sqrtv, np.float64) ** 2
    ft = np.asarray(ft, np.complex128)
    return -np.einsum("avg,g,bvg->ab", ft, v, np.conj(ft))


def sigma_sex(ft, s_gg) -> np.ndarray:
    """Static screened exchange, T form: Sigma_sex(n,n') = sum_v sum_g f~_g^{nv} T_g^{n'v} with
    T_g^{n'v} = -sum_g' S(g,g') conj(f~_g'^{n'v})."""
    ft = np.asarray(ft, np.complex128)
    nn, nv, ng = ft.shape
    t = -(np.conj(ft).reshape(nn * nv, ng) @ np.asarray(s_gg, np.complex128).T).reshape(nn, nv, ng)
    return np.einsum("avg,bvg->ab", ft, t)


def sigma_sex_modes(ft, modes, sigma) -> np.ndarray:
    """Static screened exchange, eigen form: zeta_a^{nv} = sum_g f~_g^{nv} A(g,a);
    Sigma_sex(n,n') = -sum_a sigma_a sum_v zeta_a^{nv} conj(zeta_a^{n'v})."""
    zeta = np.einsum("avg,gk->avk", np.asarray(ft, np.complex128), np.asarray(modes, np.complex128))
    return -np.einsum("k,avk,bvk->ab", np.asarray(sigma, np.float64), zeta, np.conj(zeta))


def sigma_x_real_space(psi_n, psi_v, n: Sequence[int], miller, sqrtv) -> np.ndarray:
    """The paper's real-space route for the bare exchange: B(r,r') = sum_v u_v(r) conj(u_v(r')),
    Vq(r,r') = sum_g V(q+g) exp(-i G.(r - r')), C = B * Vq entry by entry, J = C u_n',
    Sigma_x(n,n') = -sum_r conj(u_n(r)) J(r, n')."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    r = np.arange(nr)
    i = np.stack([r // (n[1] * n[2]), (r // n[2]) % n[1], r % n[2]], axis=1).astype(np.float64)
    m = np.asarray(miller, np.float64)
    ph = np.exp(-2j * np.pi * (i / np.array(n, np.float64)) @ m.T)          # [nr][ng]: exp(-i G.r)
    v = np.asarray(sqrtv, np.float64) ** 2
    vq = (ph * v[None, :]) @ np.conj(ph).T                                  # sum_g V exp(-iG.r) exp(+iG.r')
    psi_v = np.asarray(psi_v, np.complex128)
    b = psi_v.T @ np.conj(psi_v)                                            # [nr][nr]
    c = b * vq
    j = c @ np.asarray(psi_n, np.complex128).T                              # [nr][nn]
    return -np.conj(np.asarray(psi_n, np.complex128)) @ j
