"""GPU parity: every entry point of the C ABI against the FP64 oracle on the same seeded inputs.

Inputs are the complex64-rounded orbitals the GPU receives (the oracle upcasts them), so the
reported errors are those of the kernels.  Tolerances (relative Frobenius unless stated):
FP32 path 1e-5 for P, P~ and eps^-1; split BF16 / FP16 1e-4."""
import numpy as np
import pytest

import gwsynth as gs
import oracle as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def gw():
    _need_gpu()
    import paper_1810_07772_amd as gw
    gw.load()
    return gw


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def c64(x):
    return dev(np.asarray(x).astype(np.complex64))


def sys_c64(n, nv, nc, r2, seed=0, q=(0.0, 0.0, 0.0)):
    s = gs.make_system(n, nv, nc, r2_psi=r2, seed=seed, q=q).as_c64()
    print(f"[case] n={n} nv={nv} nc={nc} r2={r2} seed={seed} q={q} ng={s.ng}", flush=True)
    return s


# --- pair products --------------------------------------------------------------------------
@pytest.mark.parametrize("n,nv,nc,r2", [(12, 8, 64, 10.0),
                                        (5, 3, 7, 3.0),       # odd nr, fewer bands than one block of each
                                        (6, 11, 13, 4.0),     # two occupied and two unoccupied blocks, ragged
                                        (12, 11, 13, 10.0),   # the same raggedness where whole 1024-point chunks exist
                                        (11, 3, 9, 8.0)])     # odd nr above one chunk: every workgroup on the general path
def test_pair_products(gw, n, nv, nc, r2):
    s = sys_c64(n, nv, nc, r2)
    f = gw.pair_products(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, prefactor=2.0)
    torch.cuda.synchronize()
    ref = orc.pair_products(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=2.0)
    got = f.cpu().numpy()
    err = np.abs(got - ref) / np.max(np.abs(ref))
    assert err.max() < 2e-7, err.max()


# --- P(r, r') --------------------------------------------------------------------------------
@pytest.mark.parametrize("n,nv,nc,r2,tile", [
    (12, 8, 64, 10.0, -1),        # 12^3 workload: several 128-tiles, exact chunk multiples
    (10, 3, 37, 6.0, -1),         # ragged: nr = 1000 (not a tile multiple), nc not a chunk multiple
    (12, 8, 64, 10.0, 1),         # the single-level FP32 tile
    (4, 1, 1, 1.0, -1),           # degenerate: one pair, nr = 64 (one partial tile)
])
def test_polarizability_r_fp32(gw, n, nv, nc, r2, tile):
    s = sys_c64(n, nv, nc, r2)
    p = gw.polarizability_r(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, tile=tile)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    got = p.cpu().numpy()
    e = orc.rel_f(got, ref)
    print(f"rel_F(P) = {e:.3e}")
    assert e < 1e-5
    # Hermitian and negative semidefinite as written (both triangles)
    assert np.max(np.abs(got - got.conj().T)) <= 1e-6 * np.max(np.abs(got))


def test_polarizability_r_accumulate_and_prefactor(gw):
    s = sys_c64(8, 6, 24, 6.0, seed=3)
    pv, pc = c64(s.psi_v), c64(s.psi_c)
    p = gw.polarizability_r(pv[:2].contiguous(), pc, s.e_v[:2], s.e_c, prefactor=2.0)
    gw.polarizability_r(pv[2:].contiguous(), pc, s.e_v[2:], s.e_c, prefactor=2.0, accumulate=True, out=p)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=2.0)
    assert orc.rel_f(p.cpu().numpy(), ref) < 1e-5


# --- sphere transforms -------------------------------------------------------------------------
@pytest.mark.parametrize("n,r2,q", [(12, 10.0, (0, 0, 0)), (8, 6.0, (0.1, -0.2, 0.05)), (6, 4.0, (0, 0, 0)),
                                    (9, 9.0, (0.25, 0.0, 0.0)), (16, 30.0, (0, 0, 0)), (5, 1e9, (0, 0, 0))])
def test_sphere_transform(gw, n, r2, q):
    rng = np.random.default_rng(7)
    nr = n ** 3
    a = (rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))).astype(np.complex64)
    mill = gs.sphere((n, n, n), r2=r2, q=q)
    print(f"[case] n={n} ng={len(mill)} q={q}", flush=True)
    out = gw.sphere_transform(dev(a), (n, n, n), mill)
    torch.cuda.synchronize()
    ref = orc.to_sphere(a.astype(np.complex128), (n, n, n), mill)
    e = orc.rel_f(out.cpu().numpy(), ref)
    print(f"rel_F = {e:.3e}")
    assert e < 2e-6


# Each long transform length (24 = 4 x 6, 32 = 4 x 8, 36 = 6 x 6) on every axis of a grid small enough
# for the dense oracle, pruned to a sphere at q = 0 and unpruned (every non-Nyquist vector) at q != 0.
LONG_GRIDS = [(L, 5, 6) for L in (24, 32, 36)] + [(6, L, 5) for L in (24, 32, 36)] + [(5, 6, L) for L in (24, 32, 36)]


@pytest.mark.parametrize("n", LONG_GRIDS)
@pytest.mark.parametrize("r2,q", [(20.0, (0.0, 0.0, 0.0)), (1e9, (0.15, -0.05, 0.3))])
def test_sphere_transform_long_axes(gw, n, r2, q):
    rng = np.random.default_rng(sum(n))
    nr = n[0] * n[1] * n[2]
    a = (rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))).astype(np.complex64)
    mill = gs.sphere(n, r2=r2, q=q)
    print(f"[case] n={n} ng={len(mill)} q={q}", flush=True)
    out = gw.sphere_transform(dev(a), n, mill)
    torch.cuda.synchronize()
    ref = orc.to_sphere(a.astype(np.complex128), n, mill)
    e = orc.rel_f(out.cpu().numpy(), ref)
    print(f"rel_F = {e:.3e}")
    assert e < 2e-6


# Grids with n2 = n3 take the row-contiguous transform (one wave per (row, i1) plane, then the i1 axis per
# row); every other grid the strided passes.  Both the general form and the Hermitian form, which reads
# only the upper triangle of P, are checked against the dense oracle, at q = 0 with a pruned sphere and at
# q != 0 with every non-Nyquist vector.
PLANE_GRIDS = [(5, 24, 24), (6, 32, 32), (4, 36, 36), (12, 12, 12), (9, 8, 8), (10, 5, 5)]
# every other supported length: as n2 = n3 (the in-plane kernel, its planes per wave chosen per length and
# sphere) and as n1 (the i1 kernel); (5, 48, 48) with the whole grid's sphere has 8836 vectors, more than the
# i1 kernel stages in LDS, so it also takes that kernel's direct-store path
PLANE_GRIDS += [(5, 48, 48), (4, 40, 40), (4, 30, 30), (4, 27, 27), (4, 20, 20), (4, 18, 18), (4, 15, 15),
                (4, 10, 10), (5, 4, 4), (48, 4, 4), (40, 4, 4), (36, 4, 4), (32, 4, 4), (30, 4, 4), (27, 4, 4),
                (24, 4, 4), (20, 4, 4), (18, 4, 4), (16, 4, 4), (15, 4, 4), (8, 4, 4)]


def hermitian_c64(nr, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))
    h = (a + a.conj().T).astype(np.complex64)
    iu = np.triu_indices(nr, 1)
    h.T[iu] = np.conj(h[iu])                # exactly Hermitian after the rounding
    h[np.diag_indices(nr)] = h[np.diag_indices(nr)].real
    return h


@pytest.mark.parametrize("n", PLANE_GRIDS)
@pytest.mark.parametrize("r2,q", [(20.0, (0.0, 0.0, 0.0)), (1e9, (0.15, -0.05, 0.3))])
def test_sphere_transform_plane_path(gw, n, r2, q):
    nr = n[0] * n[1] * n[2]
    mill = gs.sphere(n, r2=r2, q=q)
    print(f"[case] plane path n={n} ng={len(mill)} q={q}", flush=True)
    h = hermitian_c64(nr, sum(n))
    rng = np.random.default_rng(sum(n) + 3)
    a = (rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))).astype(np.complex64)
    out_g = gw.sphere_transform(dev(a), n, mill)
    out_h = gw.sphere_transform(dev(h), n, mill, hermitian=True)
    # below the diagonal the Hermitian form must read nothing: garbage there changes no output bit
    hg = h.copy()
    hg[np.tril_indices(nr, -1)] = 1e30
    out_hg = gw.sphere_transform(dev(hg), n, mill, hermitian=True)
    torch.cuda.synchronize()
    ref_g = orc.to_sphere(a.astype(np.complex128), n, mill)
    ref_h = orc.to_sphere(h.astype(np.complex128), n, mill)
    e_g = orc.rel_f(out_g.cpu().numpy(), ref_g)
    got_h = out_h.cpu().numpy()
    e_h = orc.rel_f(got_h, ref_h)
    print(f"general rel_F = {e_g:.3e}, hermitian rel_F = {e_h:.3e}")
    assert e_g < 2e-6 and e_h < 2e-6
    assert np.array_equal(got_h, out_hg.cpu().numpy())
    assert np.array_equal(got_h, got_h.conj().T)              # X + X^H is Hermitian exactly


# --- the whole build to P~ -----------------------------------------------------------------------
@pytest.mark.parametrize("n,nv,nc,r2,q", [(12, 8, 64, 10.0, (0, 0, 0)), (8, 4, 20, 6.0, (0.0, 0.0, 0.001))])
def test_polarizability_end_to_end(gw, n, nv, nc, r2, q):
    s = sys_c64(n, nv, nc, r2, q=q)
    prr = torch.empty((s.nr, s.nr), dtype=torch.complex64, device="cuda:0")
    pgg = gw.polarizability(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller, p_rr=prr)
    pgg2 = gw.polarizability(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)  # internal P
    torch.cuda.synchronize()
    p_ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    pt_ref = orc.to_sphere(p_ref, s.n, s.miller)
    assert orc.rel_f(prr.cpu().numpy(), p_ref) < 1e-5
    e = orc.rel_f(pgg.cpu().numpy(), pt_ref)
    print(f"rel_F(P~) = {e:.3e}")
    assert e < 1e-5
    assert np.array_equal(pgg.cpu().numpy(), pgg2.cpu().numpy())


# --- eps and eps^-1 ------------------------------------------------------------------------------
def test_epsilon_build(gw):
    s = sys_c64(8, 4, 24, 6.0, seed=5)
    rng = np.random.default_rng(1)
    pt = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    pt32 = (pt + 1e-3 * np.abs(pt).max() * rng.standard_normal(pt.shape)).astype(np.complex64)  # not Hermitian
    eps = gw.epsilon(dev(pt32), s.n, s.a_bohr, s.q, s.miller, head=1.7)
    torch.cuda.synchronize()
    h = 0.5 * (pt32.astype(np.complex128) + pt32.astype(np.complex128).conj().T)
    ref = orc.epsilon(h, orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller), head=1.7)
    got = eps.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    assert got[0, 0] == 1.7


@pytest.mark.parametrize("n", [1, 31, 32, 100, 257, 450])
def test_hpd_inverse(gw, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = x @ x.conj().T / n + np.eye(n)
    inv = gw.hpd_inverse(dev(a))
    torch.cuda.synchronize()
    ref = np.linalg.inv(a)
    e = orc.rel_f(inv.cpu().numpy(), ref)
    print(f"n={n} rel_F = {e:.3e}")
    assert e < 1e-12


def test_hpd_inverse_not_pd(gw):
    n = 70
    a = np.eye(n, dtype=np.complex128)
    a[40, 40] = -1.0
    with pytest.raises(gw.GwError) as ei:
        gw.hpd_inverse(dev(a))
    assert ei.value.status == 4 and "pivot 41" in str(ei.value)


def test_hpd_inverse_not_pd_in_a_later_panel(gw):
    # A = Lu D Lu^H with a dense unit lower triangular Lu: the factorisation's pivots are D's entries, so the
    # first non-positive one is pivot 201 (the third 32-wide step of the second 128-column panel, where the
    # panel's earlier columns are applied before the pivot is seen)
    n = 300
    rng = np.random.default_rng(3)
    lu = np.eye(n) + np.tril(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1) * (0.3 / np.sqrt(n))
    d = np.ones(n)
    d[200] = -0.5
    a = (lu * d) @ lu.conj().T
    with pytest.raises(gw.GwError) as ei:
        gw.hpd_inverse(dev(a))
    assert ei.value.status == 4 and "pivot 201" in str(ei.value)


@pytest.mark.parametrize("q,head", [((0, 0, 0), 1.0), ((0.0, 0.0, 0.001), 1.0), ((0.2, 0.1, 0.05), 1.0)])
def test_eps_inverse_end_to_end(gw, q, head):
    s = sys_c64(12, 8, 64, 10.0, q=q)
    pgg = gw.polarizability(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)
    einv = gw.eps_inverse(pgg, s.n, s.a_bohr, s.q, s.miller, head=head)
    torch.cuda.synchronize()
    pt_ref = orc.to_sphere(orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c), s.n, s.miller)
    ref = orc.eps_inverse(orc.epsilon(pt_ref, orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller), head))
    got = einv.cpu().numpy()
    e = orc.rel_f(got, ref)
    # eps^-1 - I: at tiny |q| the head row and column carry V(q) ~ 1/|q|^2 times the single-precision
    # rounding of P~(0, .), which is conditioning of the input, so they are left out of this measure.
    tiny = 0 < np.linalg.norm(q) < 1e-2
    body = slice(1, None) if tiny else slice(0, None)
    eye = np.eye(len(ref))
    e2 = orc.rel_f((got - eye)[body, body], (ref - eye)[body, body])
    # The whole matrix can be no more accurate than P~ in single precision allows: to first order
    # d(eps^-1) = eps^-1 V^1/2 dP~ V^1/2 eps^-1 (eps = I - V^1/2 P~ V^1/2), and an FP32 P~ carries
    # ||dP~||_F ~ 2^-24 ||P~||_F, so ||d(eps^-1)||_F <= ||eps^-1||_2^2 max(v)^2 2^-24 ||P~||_F.
    v = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
    cond = np.linalg.norm(ref, 2) ** 2 * np.max(np.abs(v)) ** 2 * 2.0 ** -24 * np.linalg.norm(pt_ref)
    cond /= np.linalg.norm(ref)
    print(f"rel_F(eps^-1) = {e:.3e}, rel_F(eps^-1 - I) = {e2:.3e}, FP32 conditioning bound {cond:.3e}")
    assert e < max(1e-5, cond) and e2 < 1e-4


# --- precision variants (workload 3: the 12^3 system, rows r = 0 mod 8 of P) -------------------------
@pytest.mark.parametrize("prec,tol", [("bf16", 1e-4), ("fp16", 1e-4), ("fp32", 1e-5)])
def test_precision_variants(gw, prec, tol):
    s = sys_c64(12, 8, 64, 10.0)
    prr = torch.empty((s.nr, s.nr), dtype=torch.complex64, device="cuda:0")
    pgg = gw.polarizability(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller,
                            precision=prec, p_rr=prr)
    einv = gw.eps_inverse(pgg, s.n, s.a_bohr, s.q, s.miller)
    torch.cuda.synchronize()
    rows = np.arange(0, s.nr, 8)
    p_full = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    pt_ref = orc.to_sphere(p_full, s.n, s.miller)
    ei_ref = orc.eps_inverse(orc.epsilon(pt_ref, orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)))
    ep = orc.rel_f(prr.cpu().numpy()[rows], p_full[rows])
    ept = orc.rel_f(pgg.cpu().numpy(), pt_ref)
    eei = orc.rel_f(einv.cpu().numpy(), ei_ref)
    print(f"{prec}: rel_F P(rows)={ep:.3e} P~={ept:.3e} eps^-1={eei:.3e}")
    assert ep < tol and ept < tol and eei < tol


# --- errors and workspace --------------------------------------------------------------------------
def test_invalid_arguments_raise(gw):
    s = sys_c64(4, 2, 3, 2.0)
    with pytest.raises(gw.GwError) as ei:
        gw.polarizability_r(c64(s.psi_v), c64(s.psi_c), s.e_v, np.full(3, -1.0))
    assert ei.value.status == 1
    bad = s.miller.copy()
    bad[1] = bad[0]
    with pytest.raises(gw.GwError) as ei:
        gw.sphere_transform(torch.zeros((64, 64), dtype=torch.complex64, device="cuda:0"), (4, 4, 4), bad)
    assert ei.value.status == 1
    with pytest.raises(gw.GwError) as ei:
        gw.sphere_transform(torch.zeros((343, 343), dtype=torch.complex64, device="cuda:0"), (7, 7, 7),
                            gs.sphere((7, 7, 7), r2=2.0))
    assert ei.value.status == 5


def test_workspace_cap(gw):
    s = sys_c64(8, 2, 8, 4.0)
    ctx = gw.Context(0, workspace_cap=1 << 16)
    with pytest.raises(gw.GwError) as ei:
        gw.polarizability(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller, ctx=ctx)
    assert ei.value.status == 2
    ctx.close()


# --- every tile configuration of the update ------------------------------------------------------
def _tiles():
    import paper_1810_07772_amd as gw
    try:
        return list(enumerate(gw.tile_names()))
    except Exception:
        return [(i, f"tile{i}") for i in range(6)]


@pytest.mark.parametrize("n,nv,nc,r2", [(12, 8, 64, 10.0), (10, 3, 37, 6.0),
                                        (4, 1, 1, 1.0),       # one pair, one partial tile
                                        (6, 1, 40, 6.0)])     # one occupied band over several chunks
@pytest.mark.parametrize("tile,name", _tiles())
def test_every_tile(gw, tile, name, n, nv, nc, r2):
    prec = "fp32" if name.startswith("fp32") else ("bf16" if name.startswith("bf16") else "fp16")
    tol = 1e-5 if prec == "fp32" else 1e-4
    s = sys_c64(n, nv, nc, r2, seed=11)
    p = gw.polarizability_r(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, precision=prec, tile=tile)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c)
    e = orc.rel_f(p.cpu().numpy(), ref)
    print(f"tile {name}: rel_F(P) = {e:.3e}")
    assert e < tol


def test_fp16_scaled_tiles_agree_with_wide_band_exponents(gw):
    """Occupied energies spread over 400 eV give per-band exponents several units apart, so the
    wave-specialised FP16 tile rescales its accumulators between bands; it must agree with the
    per-band-fold tile and with the oracle."""
    s = sys_c64(12, 8, 64, 10.0, seed=5)
    e_v = np.linspace(-400.0, -0.5, 8) / 27.211386245988
    names = gw.tile_names()
    t_old = names.index("fp16split_t128_scaled_vouter")
    pv, pc = c64(s.psi_v), c64(s.psi_c)
    a = gw.polarizability_r(pv, pc, e_v, s.e_c, precision="fp16", tile=t_old).cpu().numpy()
    ref = orc.polarizability_r(s.psi_v, s.psi_c, e_v, s.e_c)
    ea = orc.rel_f(a, ref)
    for ws in ("fp16split_t128_ws_k32_scaled", "fp16split_t128_ws2_k32_scaled", "fp16split_t128x256_wide_k16_scaled",
               "fp16split_t128x256_planar_k16_scaled"):
        b = gw.polarizability_r(pv, pc, e_v, s.e_c, precision="fp16", tile=names.index(ws)).cpu().numpy()
        eb, eab = orc.rel_f(b, ref), orc.rel_f(b, a)
        print(f"fp16 per-band fold {ea:.2e}, {ws} with rescaling {eb:.2e}, between them {eab:.2e}")
        # an FP16 hi + lo pair carries 22 bits: the wave-specialised tiles reach that level; the
        # older single-role tile stays within the split-precision bound
        assert eb < 1e-6 and ea < 1e-4 and eab < 1e-4


@pytest.mark.parametrize("prec,tile_name,tol", [("bf16", "bf16split_t128_ws_k32", 1e-4),
                                                ("bf16", "bf16split_t128_ws", 1e-4),
                                                ("bf16", "bf16split_t128_ws2_k32", 1e-4),
                                                ("bf16", "bf16split_t128x256_wide_k16", 1e-4),
                                                ("bf16", "bf16split_t128x256_planar_k16", 1e-4),
                                                ("fp16", "fp16split_t128_ws_k32_scaled", 2e-5),
                                                ("fp16", "fp16split_t128_ws2_k32_scaled", 2e-5),
                                                ("fp16", "fp16split_t128x256_wide_k16_scaled", 2e-5),
                                                ("fp16", "fp16split_t128x256_planar_k16_scaled", 2e-5)])
@pytest.mark.parametrize("nv,nc", [(32, 1024), (64, 600), (64, 1024)])
def test_split_two_level_sum(gw, prec, tile_name, tol, nv, nc):
    """K = nv*nc of 32768 (no fold), 38400 (one fold, ragged) and 65536 (a fold between two full blocks)
    on an 8^3 grid with random (non-orthogonal) orbitals: the wave-specialised kernels add their
    partial sums into P every 32768 pairs.  Also accumulating onto an existing P, and the written
    mirror half."""
    rng = np.random.default_rng(nv * nc)
    nr = 512
    pv = ((rng.standard_normal((nv, nr)) + 1j * rng.standard_normal((nv, nr))) / np.sqrt(2 * nr)).astype(np.complex64)
    pc = ((rng.standard_normal((nc, nr)) + 1j * rng.standard_normal((nc, nr))) / np.sqrt(2 * nr)).astype(np.complex64)
    e_v, e_c = gs.energies(rng, nv, nc)
    tile = gw.tile_names().index(tile_name)
    print(f"[case] {tile_name} nv={nv} nc={nc} K={nv * nc}", flush=True)
    p = gw.polarizability_r(c64(pv), c64(pc), e_v, e_c, precision=prec, tile=tile)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(pv, pc, e_v, e_c)
    got = p.cpu().numpy()
    e = orc.rel_f(got, ref)
    herm = np.max(np.abs(got - got.conj().T)) / np.max(np.abs(got))
    print(f"rel_F(P) = {e:.2e}, |P - P^H| / max|P| = {herm:.1e}")
    assert e < tol and herm < 0.1 * tol
    # accumulate: P holds the first half of the occupied bands, the call adds the second half
    h = nv // 2
    gw.polarizability_r(c64(pv[:h]), c64(pc), e_v[:h], e_c, precision=prec, tile=tile, out=p)
    gw.polarizability_r(c64(pv[h:]), c64(pc), e_v[h:], e_c, precision=prec, tile=tile, accumulate=True, out=p)
    torch.cuda.synchronize()
    e2 = orc.rel_f(p.cpu().numpy(), ref)
    print(f"accumulated in two calls: rel_F(P) = {e2:.2e}")
    assert e2 < tol


def test_mfma_rate_reference_runs_its_products(gw):
    """The MFMA-only rate kernel does the products it counts: the sum of all accumulator entries of a
    wave equals sum over iterations of 3 (v_a.v_b + v_a.v_c + v_c.v_b + v_b.v_a), where v_X[k] sums
    operand set X over the lanes holding K index k (lanes 0-31: k = 0..7, lanes 32-63: k = 8..15)."""
    rng = np.random.default_rng(3)
    halves = ((127 << 7) | rng.integers(0, 128, 8192)).astype(np.uint32)   # BF16 in [1, 2): no cancellation
    words = torch.from_numpy((halves[0::2] | (halves[1::2] << 16)).view(np.int32).copy()).to("cuda:0")
    grid, n_iter = 3, 20
    out = gw.mfma_rate(words, n_iter, grid).cpu().numpy().astype(np.float64)
    sets = (halves.astype(np.uint32) << 16).view(np.float32).astype(np.float64).reshape(16, 64, 8)
    v = np.concatenate([sets[:, :32, :].sum(axis=1), sets[:, 32:, :].sum(axis=1)], axis=1)   # [set][k]
    per_wg = 0.0
    for w in range(8):
        for it in range(n_iter):
            a = (2 * it + w) & 15
            b, c = (a + 5) & 15, (a + 9) & 15
            per_wg += 3 * (v[a] @ v[b] + v[a] @ v[c] + v[c] @ v[b] + v[b] @ v[a])
    got = out.reshape(grid, 512).sum(axis=1)
    print(f"per-workgroup sums {got}, expected {per_wg:.6e}")
    assert np.all(np.abs(got - per_wg) < 1e-5 * per_wg)
