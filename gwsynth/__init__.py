"""Seeded synthetic inputs for the static polarizability build.

This module only *draws inputs*: plane-wave orbitals on an FFT grid, band
energies, q-vectors and the ordered G-sphere (Miller list) on which the
caller wants the output.  It holds none of the method's arithmetic (no pair
products, no rank-k update, no transforms of P, no Coulomb kernel), so both
the FP64 oracle and the GPU library can take their inputs from here without
sharing any computation.

Conventions (shared input format, stated once):

* Grid index of a real-space point: r = (i1*n2 + i2)*n3 + i3.
* Miller indices m = (m1, m2, m3) with |m_d| < n_d/2 (no Nyquist plane).
* Orbitals are grid-normalised: sum_r |psi_n(r)|^2 = 1, with
  psi_n(r) = N_r^(-1/2) sum_m c_nm exp(+i 2pi m.i/n), i.e. the plane-wave to
  real-space transform of the paper's Sec. 4.1 (periodic parts u_nk built from
  their plane-wave coefficients) written on the grid.  Grid orbitals handed
  out here come from numpy's inverse FFT of the drawn coefficients; systems also
  carry the coefficients themselves, for the library's own transform of them.
* Energies are returned in Hartree.
* Cubic cell of side a = 0.855 * n Bohr, Omega = a^3 (the paper gives no cell
  size; this makes a 12^3 grid a 10.26 Bohr cell, close to bulk Si).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

HARTREE_EV = 27.211386245988
CELL_BOHR_PER_POINT = 0.855


# ---------------------------------------------------------------------------
# G-spheres (ordered Miller lists)
# ---------------------------------------------------------------------------
def _all_miller(n: Tuple[int, int, int]) -> np.ndarray:
    """Every Miller triple with |m_d| < n_d/2, as an int array [M][3]."""
    axes = []
    for nd in n:
        half = (nd - 1) // 2          # |m| <= half  <=>  |m| < nd/2 for the Nyquist rule
        axes.append(np.arange(-half, half + 1))
    m1, m2, m3 = np.meshgrid(*axes, indexing="ij")
    return np.stack([m1.ravel(), m2.ravel(), m3.ravel()], axis=1).astype(np.int64)


def sphere(n: Sequence[int], r2: Optional[float] = None, q: Sequence[float] = (0.0, 0.0, 0.0),
           count: Optional[int] = None) -> np.ndarray:
    """Ordered G-sphere as int32 Miller triples [Ng][3].

    Membership: |q + m|^2 <= r2 (crystal units, cubic cell), or, when `count`
    is given, the `count` smallest |q + m|.  Order: ascending (|q+m|^2, m1, m2,
    m3), which is also the tie-break for `count`.
    """
    n = tuple(int(x) for x in n)
    m = _all_miller(n)
    qv = np.asarray(q, dtype=np.float64)
    d2 = ((m + qv[None, :]) ** 2).sum(axis=1)
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], d2))
    m, d2 = m[order], d2[order]
    if count is not None:
        if count > len(m):
            raise ValueError("sphere count exceeds the grid's Miller set")
        m = m[:count]
    else:
        if r2 is None:
            raise ValueError("give r2 or count")
        m = m[d2 <= r2 + 1e-9]
    return np.ascontiguousarray(m.astype(np.int32))


def cell_side(n: int) -> float:
    return CELL_BOHR_PER_POINT * float(n)


# ---------------------------------------------------------------------------
# Orbitals and energies
# ---------------------------------------------------------------------------
def orbital_coefficients(rng: np.random.Generator, n: Sequence[int], r2_psi: float,
                         nbands: int) -> Tuple[np.ndarray, np.ndarray]:
    """Orthonormal random plane-wave coefficients on the sphere |m|^2 <= r2_psi.

    Returns (Miller list int32 [N_pw][3] in sphere order, coefficients complex128
    [nbands][N_pw]).  Draw order: real parts then imaginary parts of the block
    [N_pw][nbands] (standard normal, /sqrt(2)), Gaussian envelope
    exp(-|m|^2 / r2_psi) (sigma^2 = r2_psi/2), reduced QR with the phase of
    diag(R) removed so diag(R) > 0.
    """
    n = tuple(int(x) for x in n)
    mp = sphere(n, r2=r2_psi)
    npw = len(mp)
    if nbands > npw:
        raise ValueError(f"{nbands} bands need at least as many plane waves (have {npw})")
    re = rng.standard_normal((npw, nbands))
    im = rng.standard_normal((npw, nbands))
    c = (re + 1j * im) / np.sqrt(2.0)
    env = np.exp(-(mp.astype(np.float64) ** 2).sum(axis=1) / float(r2_psi))
    c *= env[:, None]
    qm, rm = np.linalg.qr(c, mode="reduced")
    d = np.diag(rm)
    qm = qm * (d / np.abs(d))[None, :]
    return mp, np.ascontiguousarray(qm.T)


def coefficients_on_grid(n: Sequence[int], mp: np.ndarray, coeff: np.ndarray) -> np.ndarray:
    """Grid orbitals from plane-wave coefficients by numpy's inverse FFT times sqrt(N_r)
    (the input convention above), complex128 [nbands][N_r]."""
    n = tuple(int(x) for x in n)
    nr = n[0] * n[1] * n[2]
    box = np.zeros((coeff.shape[0],) + n, dtype=np.complex128)
    box[:, mp[:, 0] % n[0], mp[:, 1] % n[1], mp[:, 2] % n[2]] = coeff
    psi = np.fft.ifftn(box, axes=(1, 2, 3)) * np.sqrt(nr)
    return np.ascontiguousarray(psi.reshape(coeff.shape[0], nr))


def orbitals(rng: np.random.Generator, n: Sequence[int], r2_psi: float, nbands: int) -> np.ndarray:
    """Grid-orthonormal random orbitals, complex128 [nbands][N_r]: the coefficients of
    orbital_coefficients placed on the grid by coefficients_on_grid."""
    mp, c = orbital_coefficients(rng, n, r2_psi, nbands)
    return coefficients_on_grid(n, mp, c)


def energies(rng: np.random.Generator, nv: int, nc: int) -> Tuple[np.ndarray, np.ndarray]:
    """E_v sorted U[-15, 0] eV, E_c sorted 1 + U[0, 30] eV; returned in Hartree."""
    ev = np.sort(rng.uniform(-15.0, 0.0, nv)) / HARTREE_EV
    ec = np.sort(1.0 + rng.uniform(0.0, 30.0, nc)) / HARTREE_EV
    return ev, ec


def plane_wave_orbitals(n: Sequence[int], millers: np.ndarray) -> np.ndarray:
    """psi_m(r) = exp(+i 2pi m.i/n) / sqrt(N_r) for each Miller triple, complex128 [len][N_r]."""
    n = tuple(int(x) for x in n)
    i1, i2, i3 = np.meshgrid(*(np.arange(x) for x in n), indexing="ij")
    ph = (np.multiply.outer(millers[:, 0], i1) / n[0] + np.multiply.outer(millers[:, 1], i2) / n[1]
          + np.multiply.outer(millers[:, 2], i3) / n[2])
    nr = n[0] * n[1] * n[2]
    return (np.exp(2j * np.pi * ph) / np.sqrt(nr)).reshape(len(millers), nr)


def random_unitary_orbitals(rng: np.random.Generator, nr: int) -> np.ndarray:
    """A complete grid basis: N_r orthonormal orbitals from the QR of a Gaussian matrix."""
    a = (rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))) / np.sqrt(2.0)
    qm, rm = np.linalg.qr(a)
    d = np.diag(rm)
    return np.ascontiguousarray((qm * (d / np.abs(d))[None, :]).T)


# ---------------------------------------------------------------------------
# Whole systems
# ---------------------------------------------------------------------------
@dataclass
class System:
    n: Tuple[int, int, int]
    a_bohr: float
    psi_v: np.ndarray          # complex128 [nv][nr]
    psi_c: np.ndarray          # complex128 [nc][nr]
    e_v: np.ndarray            # float64 [nv], Hartree
    e_c: np.ndarray            # float64 [nc], Hartree
    q: np.ndarray              # float64 [3], crystal units
    miller: np.ndarray         # int32 [ng][3], ordered sphere
    meta: dict = field(default_factory=dict)
    pw_miller: Optional[np.ndarray] = None   # int32 [npw][3], the orbitals' plane-wave sphere
    coeff: Optional[np.ndarray] = None       # complex128 [nv + nc][npw], occupied bands first

    @property
    def nr(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nv(self) -> int:
        return self.psi_v.shape[0]

    @property
    def nc(self) -> int:
        return self.psi_c.shape[0]

    @property
    def ng(self) -> int:
        return self.miller.shape[0]

    def as_c64(self) -> "System":
        """The same system with orbitals rounded to complex64 and back (what the GPU receives)."""
        return System(self.n, self.a_bohr,
                      self.psi_v.astype(np.complex64).astype(np.complex128),
                      self.psi_c.astype(np.complex64).astype(np.complex128),
                      self.e_v.copy(), self.e_c.copy(), self.q.copy(), self.miller.copy(), dict(self.meta))


def make_system(n: int, nv: int, nc: int, r2_psi: float, r2_p: Optional[float] = None, seed: int = 0,
                q: Sequence[float] = (0.0, 0.0, 0.0), ng: Optional[int] = None) -> System:
    """One seeded system: bands 0..nv-1 of the QR'd set are occupied, nv..nv+nc-1 unoccupied."""
    rng = np.random.default_rng(seed)
    grid = (n, n, n)
    mp, coeff = orbital_coefficients(rng, grid, r2_psi, nv + nc)
    psi = coefficients_on_grid(grid, mp, coeff)
    ev, ec = energies(rng, nv, nc)
    mill = sphere(grid, r2=(r2_psi if r2_p is None else r2_p), q=q, count=ng)
    return System(grid, cell_side(n), psi[:nv].copy(), psi[nv:].copy(), ev, ec,
                  np.asarray(q, dtype=np.float64), mill, {"seed": seed, "r2_psi": r2_psi}, mp, coeff)


def truncate(sys_: System, nc: int) -> System:
    """The same system keeping only the first nc unoccupied bands."""
    return System(sys_.n, sys_.a_bohr, sys_.psi_v, sys_.psi_c[:nc].copy(), sys_.e_v, sys_.e_c[:nc].copy(),
                  sys_.q, sys_.miller, dict(sys_.meta))


# Workload shapes (the five synthetic workloads of this library).  r2 values are
# in squared Miller-index units.
WORKLOADS = {
    # 12^3 grid, Nv=8, Nc=64, 147-vector sphere, q = 0
    "si12": dict(n=12, nv=8, nc=64, r2_psi=10.0),
    # 36^3 grid, Nv=128, Nc=1024, 4067-vector sphere, q = 0
    "si36": dict(n=36, nv=128, nc=1024, r2_psi=98.0),
}


def batched_q_vectors(nq: int = 8) -> np.ndarray:
    """q_j = ((j+1)/16) * (1, 1/2, 1/4), crystal units: nonzero, never on a G."""
    return np.array([[(j + 1) / 16.0, (j + 1) / 32.0, (j + 1) / 64.0] for j in range(nq)])


def batched_q_sizes(nq: int = 8) -> list:
    """Uneven sphere sizes 2500 .. 4500 for the q batch."""
    return [2500 + int(round(2000.0 * j / (nq - 1))) for j in range(nq)]


def make_batched_q(n: int = 32, nv: int = 96, nc: int = 768, r2_psi: float = 81.0, nq: int = 8,
                   sizes: Optional[Sequence[int]] = None):
    """Occupied set from seed 0; unoccupied set of q_j from seed 1+j (its own orbital set)."""
    grid = (n, n, n)
    rng0 = np.random.default_rng(0)
    psi0 = orbitals(rng0, grid, r2_psi, nv + nc)
    ev, _ = energies(rng0, nv, nc)
    qs = batched_q_vectors(nq)
    sizes = batched_q_sizes(nq) if sizes is None else list(sizes)
    jobs = []
    for j in range(nq):
        rng = np.random.default_rng(1 + j)
        psij = orbitals(rng, grid, r2_psi, nv + nc)
        _, ecj = energies(rng, nv, nc)
        jobs.append(dict(psi_c=psij[nv:].copy(), e_c=ecj, q=qs[j], miller=sphere(grid, q=qs[j], count=sizes[j])))
    return dict(n=grid, a_bohr=cell_side(n), psi_v=psi0[:nv].copy(), e_v=ev, jobs=jobs)


# ---------------------------------------------------------------------------
# Learned band tail: seeded initial parameters and the training / evaluation systems
# ---------------------------------------------------------------------------
TAIL_SHAPES = [("w1", (4, 128)), ("b1", (128,)), ("w2", (128, 128)), ("b2", (128,)), ("w3", (128, 33)),
               ("b3", (33,))]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Flat float32 initial parameters (W1, b1, W2, b2, W3, b3): weights N(0, 1/fan_in), the last
    layer scaled by 0.1, biases zero except b3[0] = -2 (a small initial diagonal correction)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in TAIL_SHAPES:
        if name.startswith("w"):
            a = rng.standard_normal(shp) / np.sqrt(shp[0])
            if name == "w3":
                a *= 0.1
        else:
            a = np.zeros(shp)
            if name == "b3":
                a[0] = -2.0
        parts.append(a.ravel())
    return np.concatenate(parts).astype(np.float32)


def tail_train_system(seed: int, n: int = 16, nv: int = 32, nc_full: int = 512, r2: float = 36.0) -> System:
    """A training system: 16^3 grid, 925-vector sphere, the full unoccupied set of 512 bands."""
    return make_system(n, nv, nc_full, r2_psi=r2, seed=seed)


def tail_eval_system(seed: int, n: int = 24, nv: int = 32, nc_full: int = 1024, r2: float = 81.0) -> System:
    """An evaluation system: 24^3 grid, 3071-vector sphere, 1024 unoccupied bands."""
    return make_system(n, nv, nc_full, r2_psi=r2, seed=seed)
