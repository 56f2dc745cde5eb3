"""Host-side checks of the C ABI that need no GPU: the library loads, exports every symbol the
header declares, and its argument checks (run on a dry-run context) accept and reject what the
header says."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import gwsynth as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gw():
    import paper_1810_07772_amd as gw
    if not os.path.exists(gw.LIB_PATH):
        pytest.fail("libgw.so is not built (run __graft_entry__.build())")
    gw.load()
    return gw


def header_functions():
    text = open(os.path.join(ROOT, "include", "gw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[a-z_0-9]+)\s*\(", text)))


def test_exports_match_header(gw):
    declared = header_functions()
    assert declared, "no declarations parsed"
    lib = C.CDLL(gw.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(gw.EXPORTS) == declared


def test_status_strings_and_version(gw):
    lib = gw.load()
    assert lib.gw_version() >= 10000
    for st in range(6):
        assert lib.gw_status_string(st).decode().startswith("GW_")
    names = gw.tile_names()
    assert len(names) == lib.gw_tile_count() and all(names)


class Dry:
    def __init__(self, gw):
        self.ctx = gw.Context(-1)
        self.lib = self.ctx.lib

    def err(self):
        return self.lib.gw_last_error(self.ctx.handle).decode()


def vp(x=16):
    return C.c_void_p(x)


def f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.c_void_p)


def i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.c_void_p)


def test_dry_run_polarizability_checks(gw):
    d = Dry(gw)
    lib, h = d.lib, d.ctx.handle
    o = gw._lib._opts()
    ev, pev = f64([-0.4, -0.1])
    ec, pec = f64([0.05, 0.2, 0.3])
    q, pq = f64([0, 0, 0])
    n = 6
    m, pm = i32(gs.sphere((n, n, n), r2=4.0))
    grid = gw._lib.Grid(n, n, n, 5.13)
    call = lambda **kw: lib.gw_polarizability(h, kw.get("pv", vp()), kw.get("nv", 2), kw.get("pc", vp()),
                                              kw.get("nc", 3), kw.get("ev", pev), kw.get("ec", pec),
                                              kw.get("grid", grid), kw.get("q", pq), kw.get("m", pm),
                                              kw.get("ng", len(m)), C.byref(kw.get("o", o)), kw.get("prr", vp()),
                                              kw.get("pgg", vp()), None)
    assert call() == 0
    assert call(pv=vp(0)) == 1
    assert call(nv=0) == 1
    assert call(pgg=vp(0)) == 1
    assert call(q=vp(0)) == 1
    bad_e, pbad = f64([0.1, 0.2, 0.3])
    too_high, pth = f64([-0.4, 0.1])
    assert call(ev=pth) == 1 and "E_c - E_v" in d.err()
    nan_e, pnan = f64([np.nan, 0.2, 0.3])
    assert call(ec=pnan) == 1
    dup = m.copy(); dup[3] = dup[2]
    _, pdup = i32(dup)
    assert call(m=pdup) == 1 and "duplicates" in d.err()
    # several repeats: the first index that repeats an earlier G is the one reported
    dup2 = m.copy(); dup2[9] = dup2[1]; dup2[5] = dup2[4]
    _, pdup2 = i32(dup2)
    assert call(m=pdup2) == 1 and "g_miller[5] duplicates" in d.err()
    # a sphere that passed is remembered by content, not by address: the same buffer edited in place
    # into a repeat fails again, and passes once restored
    same = m.copy()
    _, psame = i32(same)
    assert call(m=psame) == 0
    keep = same[6].copy(); same[6] = same[0]
    assert call(m=psame) == 1 and "g_miller[6] duplicates" in d.err()
    same[6] = keep
    assert call(m=psame) == 0
    nyq = m.copy(); nyq[1] = [3, 0, 0]
    _, pnyq = i32(nyq)
    assert call(m=pnyq) == 1 and "|m| < n/2" in d.err()
    assert call(ng=0) == 1
    assert call(ng=n ** 3 + 1) == 1
    o2 = gw._lib._opts(precision=7)
    assert call(o=o2) == 1
    o3 = gw._lib._opts(prefactor=-1.0)
    assert call(o=o3) == 1
    o4 = gw._lib._opts(accumulate=True)
    assert call(o=o4, prr=vp(0)) == 1
    o5 = gw._lib._opts(precision="fp32", tile=2)           # a BF16 tile for the FP32 path
    assert call(o=o5) == 1
    assert call(grid=gw._lib.Grid(7, 7, 7, 6.0), m=i32(gs.sphere((7, 7, 7), r2=2.0))[1], ng=19) == 5
    assert call(grid=gw._lib.Grid(6, 6, 0, 5.13)) == 1
    assert call(grid=gw._lib.Grid(6, 6, 6, -1.0)) == 1


def test_dry_run_other_entry_points(gw):
    d = Dry(gw)
    lib, h = d.lib, d.ctx.handle
    ev, pev = f64([-0.4])
    ec, pec = f64([0.2, 0.3])
    assert lib.gw_pair_products(h, vp(), 1, vp(), 2, 10, pev, pec, 1.0, vp(), None) == 0
    assert lib.gw_pair_products(h, vp(), 1, vp(), 2, 10, pev, pec, 0.0, vp(), None) == 1
    assert lib.gw_pair_products(h, vp(), 1, vp(), 2, 10, pev, pec, 1.0, vp(0), None) == 1
    n = 8
    m, pm = i32(gs.sphere((n, n, n), r2=4.0))
    grid = gw._lib.Grid(n, n, n, 6.84)
    q, pq = f64([0, 0, 0])
    assert lib.gw_sphere_transform(h, vp(), grid, pm, len(m), vp(), None) == 0
    assert lib.gw_sphere_transform(h, vp(0), grid, pm, len(m), vp(), None) == 1
    assert lib.gw_epsilon(h, vp(), len(m), grid, pq, pm, 1.0, vp(), None) == 0
    assert lib.gw_epsilon(h, vp(), len(m), grid, pq, pm, -2.0, vp(), None) == 1
    assert lib.gw_eps_inverse(h, vp(), len(m), grid, pq, pm, float("nan"), vp(), None) == 0
    # a non-finite q is rejected by every entry point that builds the Coulomb factor
    qn, pqn = f64([0.0, np.nan, 0.0])
    assert lib.gw_epsilon(h, vp(), len(m), grid, pqn, pm, 1.0, vp(), None) == 1
    assert lib.gw_eps_inverse(h, vp(), len(m), grid, pqn, pm, 1.0, vp(), None) == 1
    assert lib.gw_eps_inverse(h, vp(), len(m), grid, None, pm, 1.0, vp(), None) == 1
    assert lib.gw_hpd_inverse(h, vp(), 0, vp(), None) == 1
    assert lib.gw_hpd_inverse(h, vp(), 10, vp(), None) == 0
    assert lib.gw_create(None, 0, 0) == 1
    assert lib.gw_destroy(None) == 1
    # plane-wave coefficients to the grid
    assert lib.gw_orbitals_to_grid(h, vp(), 3, len(m), grid, pm, vp(), None) == 0
    assert lib.gw_orbitals_to_grid(h, vp(), 0, len(m), grid, pm, vp(), None) == 1
    assert lib.gw_orbitals_to_grid(h, vp(0), 3, len(m), grid, pm, vp(), None) == 1
    assert lib.gw_orbitals_to_grid(h, vp(), 3, 0, grid, pm, vp(), None) == 1
    dup = m.copy(); dup[1] = dup[0]
    assert lib.gw_orbitals_to_grid(h, vp(), 3, len(m), grid, i32(dup)[1], vp(), None) == 1
    m7, pm7 = i32(gs.sphere((7, 7, 7), r2=2.0))
    assert lib.gw_orbitals_to_grid(h, vp(), 3, len(m7), gw._lib.Grid(7, 7, 7, 6.0), pm7, vp(), None) == 5
    # plasmon-pole model
    its, res = C.c_int(-1), C.c_double(0.0)
    pp = lambda **kw: lib.gw_plasmon_pole(h, vp(), len(m), grid, pq, pm, vp(), kw.get("nv", 4), kw.get("occ", 2.0),
                                          kw.get("nm", 8), kw.get("tol", 1e-10), kw.get("it", 100), vp(), vp(),
                                          kw.get("modes", vp()), C.byref(its), C.byref(res), None)
    assert pp() == 0 and its.value == 0
    assert pp(nm=0) == 1 and pp(nm=25) == 1 and pp(nm=len(m) + 1) == 1
    assert pp(occ=0.0) == 1 and pp(tol=0.0) == 1 and pp(it=0) == 1 and pp(nv=0) == 1 and pp(modes=vp(0)) == 1
    fr, pfr = f64([0.0, 0.5])
    assert lib.gw_pp_eps_inverse(h, vp(), len(m), grid, pq, pm, vp(), vp(), vp(), 4, pfr, 2, vp(), None) == 0
    assert lib.gw_pp_eps_inverse(h, vp(), len(m), grid, pq, pm, vp(), vp(), vp(), 4, pfr, 0, vp(), None) == 1
    frn, pfrn = f64([np.nan])
    assert lib.gw_pp_eps_inverse(h, vp(), len(m), grid, pq, pm, vp(), vp(), vp(), 4, pfrn, 1, vp(), None) == 1
    # static self-energy
    sg = lambda **kw: lib.gw_sigma_static(h, vp(), kw.get("nn", 4), vp(), kw.get("nv", 3), grid, pq, pm, len(m),
                                          kw.get("ei", vp()), kw.get("sx", vp()), kw.get("ss", vp()), None)
    assert sg() == 0 and sg(ei=None, ss=None) == 0 and sg(sx=None) == 0
    assert sg(sx=None, ss=None) == 1 and sg(ei=None) == 1 and sg(nn=0) == 1 and sg(nn=257) == 1 and sg(nv=0) == 1
    assert lib.gw_sigma_sex_modes(h, vp(), 4, vp(), 3, grid, pm, len(m), vp(), vp(), 5, vp(), None) == 0
    assert lib.gw_sigma_sex_modes(h, vp(), 4, vp(), 3, grid, pm, len(m), vp(), vp(), 0, vp(), None) == 1
    # MFMA rate reference
    assert lib.gw_mfma_rate(h, vp(), 10, 256, vp(), None) == 0
    assert lib.gw_mfma_rate(h, vp(0), 10, 256, vp(), None) == 1 and lib.gw_mfma_rate(h, vp(), 10, 256, vp(0), None) == 1
    assert lib.gw_mfma_rate(h, vp(), 0, 256, vp(), None) == 1 and lib.gw_mfma_rate(h, vp(), 10, 0, vp(), None) == 1
    # Newton iteration arguments
    its = C.c_int(-1)
    assert lib.gw_newton_inverse(h, vp(), 10, 1e-11, 50, vp(), C.byref(its), None, None) == 0 and its.value == 0
    assert lib.gw_newton_inverse(h, vp(), 10, 0.0, 50, vp(), C.byref(its), None, None) == 1
    assert lib.gw_newton_inverse(h, vp(), 10, 1e-11, 0, vp(), C.byref(its), None, None) == 1
    assert lib.gw_newton_inverse(h, vp(), 0, 1e-11, 50, vp(), C.byref(its), None, None) == 1
    assert lib.gw_eps_inverse_newton(h, vp(), len(m), grid, pq, pm, 1.0, 1e-11, 50, vp(), C.byref(its), None,
                                     None) == 0
    assert lib.gw_eps_inverse_newton(h, vp(), len(m), grid, pq, pm, 1.0, float("nan"), 50, vp(), C.byref(its), None,
                                     None) == 1
    assert lib.gw_eps_inverse_newton(h, vp(), len(m), grid, pqn, pm, 1.0, 1e-11, 50, vp(), C.byref(its), None,
                                     None) == 1


def test_product_path_has_no_fallback(gw, monkeypatch):
    """Without the built library the package raises instead of computing elsewhere."""
    import paper_1810_07772_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", os.path.join(ROOT, "does-not-exist", "libgw.so"))
    with pytest.raises(RuntimeError):
        L.load()


def test_package_does_not_import_oracle():
    import ast
    pkg = os.path.join(ROOT, "paper_1810_07772_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                tree = ast.parse(open(os.path.join(dirpath, f)).read())
                for node in ast.walk(tree):
                    if isinstance(node, (ast.Import, ast.ImportFrom)):
                        mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                        assert not any(mm.split(".")[0] == "oracle" for mm in mods), f


def test_graph_capture_counter_without_batches(gw):
    lib = gw.load()
    assert lib.gw_graph_captures(None) == 0
    assert gw.Context(-1).graph_captures == 0
