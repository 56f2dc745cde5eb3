"""The allocation-free update (gw_polarizability_r_noalloc) against the allocating entry point
(gw_polarizability_r) with the same tile: bit-identical output, and within the oracle's tolerance,
on two calls in a row (the second smaller), in every precision; its scratch limit is enforced on
the host before anything runs."""
import ctypes as C

import numpy as np
import pytest

import gwsynth as gs
import oracle as orc

torch = pytest.importorskip("torch")


def _gw():
    import paper_1810_07772_amd as gw
    gw.load()
    return gw


def test_noalloc_limit_on_dry_run_context():
    gw = _gw()
    ctx = gw.Context(-1)
    o = gw._lib._opts("bf16")
    nv, nc = 128, 16384                            # scale table alone 8 MiB: above the limit
    ev = np.linspace(-0.5, -0.1, nv)
    ec = np.linspace(0.1, 1.0, nc)
    st = ctx.lib.gw_polarizability_r_noalloc(ctx.handle, C.c_void_p(16), nv, C.c_void_p(16), nc, 1000,
                                             ev.ctypes.data_as(C.c_void_p), ec.ctypes.data_as(C.c_void_p),
                                             C.byref(o), C.c_void_p(16), None)
    assert st == 1 and "limit" in ctx.lib.gw_last_error(ctx.handle).decode()
    st = ctx.lib.gw_polarizability_r_noalloc(ctx.handle, C.c_void_p(16), nv, C.c_void_p(16), 1024, 1000,
                                             ev.ctypes.data_as(C.c_void_p), ec[:1024].ctypes.data_as(C.c_void_p),
                                             C.byref(o), C.c_void_p(16), None)
    assert st == 0


@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-4), ("fp16", 1e-4)])
def test_noalloc_matches_allocating_entry_point(prec, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gw = _gw()
    tile = gw.tile_names().index(gw.default_tile_name(prec))
    for (n, nv, nc, r2, seed) in [(12, 8, 64, 10.0, 0), (8, 3, 20, 6.0, 4)]:     # the second call is smaller
        print(f"[case] noalloc {prec} n={n} nv={nv} nc={nc}", flush=True)
        s = gs.make_system(n, nv, nc, r2_psi=r2, seed=seed).as_c64()
        pv = torch.from_numpy(s.psi_v.astype(np.complex64)).to("cuda:0")
        pc = torch.from_numpy(s.psi_c.astype(np.complex64)).to("cuda:0")
        out = torch.full((s.nr, s.nr), float("nan"), dtype=torch.complex64, device="cuda:0")
        gw.polarizability_r_noalloc(pv, pc, s.e_v, s.e_c, out, precision=prec, tile=tile)
        ref = gw.polarizability_r(pv, pc, s.e_v, s.e_c, precision=prec, tile=tile)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"{prec} n={n}: differs from gw_polarizability_r"
        e = orc.rel_f(out.cpu().numpy(), orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c))
        print(f"noalloc {prec} n={n}: rel_F {e:.2e}")
        assert e < tol


@pytest.mark.gpu
def test_noalloc_accumulate_and_limit_on_device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gw = _gw()
    s = gs.make_system(8, 6, 24, r2_psi=6.0, seed=3).as_c64()
    pv = torch.from_numpy(s.psi_v.astype(np.complex64)).to("cuda:0")
    pc = torch.from_numpy(s.psi_c.astype(np.complex64)).to("cuda:0")
    out = torch.empty((s.nr, s.nr), dtype=torch.complex64, device="cuda:0")
    gw.polarizability_r_noalloc(pv[:2].contiguous(), pc, s.e_v[:2], s.e_c, out, prefactor=2.0)
    gw.polarizability_r_noalloc(pv[2:].contiguous(), pc, s.e_v[2:], s.e_c, out, prefactor=2.0, accumulate=True)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c, prefactor=2.0)
    assert orc.rel_f(out.cpu().numpy(), ref) < 1e-5
    # 128 x 16384 pairs: the scale table alone is 8 MiB, so the host check rejects the call before any launch
    big_ev, big_ec = np.linspace(-1.0, -0.5, 128), np.linspace(1.0, 2.0, 16384)
    with pytest.raises(gw.GwError, match="limit"):
        gw.polarizability_r_noalloc(torch.zeros((128, s.nr), dtype=torch.complex64, device="cuda:0"),
                                    torch.zeros((16384, s.nr), dtype=torch.complex64, device="cuda:0"), big_ev,
                                    big_ec, out)
