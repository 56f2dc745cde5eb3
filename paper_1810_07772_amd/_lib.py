"""ctypes binding of libgw.so (include/gw.h).  Argument marshalling only: every step of the
computation runs in the library's HIP kernels.  Device arrays are torch tensors on a ROCm
device; small host arrays (energies, q, Miller lists) are numpy arrays."""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgw.so")

GW_OK, GW_E_INVAL, GW_E_NOMEM, GW_E_HIP, GW_E_NOTPD, GW_E_UNSUPPORTED = range(6)
PRECISIONS = {"fp32": 0, "bf16": 1, "split_bf16": 1, "fp16": 2, "split_fp16": 2}

# Every symbol include/gw.h declares.
EXPORTS = ("gw_opts_default", "gw_version", "gw_status_string", "gw_create", "gw_destroy", "gw_last_error",
           "gw_workspace_bytes", "gw_tile_count", "gw_tile_name", "gw_default_tile", "gw_pair_products", "gw_polarizability_r",
           "gw_polarizability_r_noalloc",
           "gw_sphere_transform", "gw_sphere_transform_herm", "gw_polarizability", "gw_epsilon", "gw_eps_inverse", "gw_hpd_inverse",
           "gw_polarizability_batched", "gw_graph_captures", "gw_autotune", "gw_tail_init", "gw_tail_target", "gw_tail_features",
           "gw_tail_forward", "gw_tail_train_step", "gw_tail_train_steps", "gw_tail_graph_count", "gw_tail_fit_norm",
           "gw_tail_residual_parts", "gw_tail_loss", "gw_tail_correct", "gw_newton_inverse",
           "gw_eps_inverse_newton", "gw_orbitals_to_grid",
           "gw_plasmon_pole", "gw_pp_eps_inverse", "gw_sigma_static", "gw_sigma_sex_modes", "gw_mfma_rate")
TAIL_NWEIGHT, TAIL_NBIAS, TAIL_NPARAM = 21120, 289, 21409


class GwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} [status {status}]")
        self.status = status


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("prefactor", C.c_double), ("accumulate", C.c_int), ("tile", C.c_int)]


class Grid(C.Structure):
    _fields_ = [("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int), ("a_bohr", C.c_double)]


class Mlp(C.Structure):
    _fields_ = [("w", C.c_void_p), ("b", C.c_void_p), ("norm", C.c_void_p), ("rank", C.c_int)]


class Adam(C.Structure):
    _fields_ = [("master", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("grad", C.c_void_p),
                ("step", C.c_int), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class QJob(C.Structure):
    _fields_ = [("psi_unocc", C.c_void_p), ("nc", C.c_int), ("e_c", C.c_void_p), ("q", C.c_double * 3),
                ("g_miller", C.c_void_p), ("ng", C.c_int), ("p_gg", C.c_void_p), ("eps_inv", C.c_void_p)]


_lib = None


def load() -> C.CDLL:
    """Load libgw.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1810_07772_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    sig = {
        "gw_opts_default": (None, [C.POINTER(Opts)]),
        "gw_version": (i, []),
        "gw_status_string": (C.c_char_p, [i]),
        "gw_create": (i, [C.POINTER(vp), i, sz]),
        "gw_destroy": (i, [vp]),
        "gw_last_error": (C.c_char_p, [vp]),
        "gw_workspace_bytes": (sz, [vp]),
        "gw_tile_count": (i, []),
        "gw_tile_name": (C.c_char_p, [i]),
        "gw_default_tile": (i, [i, i]),
        "gw_pair_products": (i, [vp, vp, i, vp, i, i, vp, vp, d, vp, vp]),
        "gw_polarizability_r": (i, [vp, vp, i, vp, i, i, vp, vp, C.POINTER(Opts), vp, vp]),
        "gw_polarizability_r_noalloc": (i, [vp, vp, i, vp, i, i, vp, vp, C.POINTER(Opts), vp, vp]),
        "gw_sphere_transform": (i, [vp, vp, Grid, vp, i, vp, vp]),
        "gw_sphere_transform_herm": (i, [vp, vp, Grid, vp, i, vp, vp]),
        "gw_polarizability": (i, [vp, vp, i, vp, i, vp, vp, Grid, vp, vp, i, C.POINTER(Opts), vp, vp, vp]),
        "gw_epsilon": (i, [vp, vp, i, Grid, vp, vp, d, vp, vp]),
        "gw_eps_inverse": (i, [vp, vp, i, Grid, vp, vp, d, vp, vp]),
        "gw_hpd_inverse": (i, [vp, vp, i, vp, vp]),
        "gw_polarizability_batched": (i, [vp, vp, i, vp, Grid, i, C.POINTER(QJob), C.POINTER(Opts), d, vp]),
        "gw_graph_captures": (i, [vp]),
        "gw_autotune": (i, [vp, vp, i, vp, i, i, vp, vp, i, vp, C.POINTER(i), vp, vp]),
        "gw_tail_init": (i, [vp, C.POINTER(Mlp), vp, vp]),
        "gw_tail_target": (i, [vp, vp, vp, i, vp, vp]),
        "gw_tail_features": (i, [vp, vp, i, Grid, vp, vp, i, d, vp, vp]),
        "gw_tail_forward": (i, [vp, C.POINTER(Mlp), vp, i, vp, vp]),
        "gw_tail_train_step": (i, [vp, C.POINTER(Mlp), C.POINTER(Adam), vp, vp, i, vp, vp]),
        "gw_tail_correct": (i, [vp, C.POINTER(Mlp), vp, i, vp, vp, C.POINTER(i), vp]),
        "gw_tail_loss": (i, [vp, C.POINTER(Mlp), vp, vp, i, vp, vp]),
        "gw_tail_train_steps": (i, [vp, C.POINTER(Mlp), C.POINTER(Adam), i, vp, vp, vp, i, vp, vp, vp]),
        "gw_tail_graph_count": (i, [vp]),
        "gw_tail_fit_norm": (i, [vp, i, vp, vp, vp, vp]),
        "gw_tail_residual_parts": (i, [vp, C.POINTER(Mlp), vp, vp, i, vp, vp]),
        "gw_plasmon_pole": (i, [vp, vp, i, Grid, vp, vp, vp, i, d, i, d, i, vp, vp, vp, C.POINTER(i),
                                C.POINTER(d), vp]),
        "gw_pp_eps_inverse": (i, [vp, vp, i, Grid, vp, vp, vp, vp, vp, i, vp, i, vp, vp]),
        "gw_sigma_static": (i, [vp, vp, i, vp, i, Grid, vp, vp, i, vp, vp, vp, vp]),
        "gw_sigma_sex_modes": (i, [vp, vp, i, vp, i, Grid, vp, i, vp, vp, i, vp, vp]),
        "gw_mfma_rate": (i, [vp, vp, i, i, vp, vp]),
        "gw_orbitals_to_grid": (i, [vp, vp, i, i, Grid, vp, vp, vp]),
        "gw_newton_inverse": (i, [vp, vp, i, d, i, vp, C.POINTER(i), vp, vp]),
        "gw_eps_inverse_newton": (i, [vp, vp, i, Grid, vp, vp, d, d, i, vp, C.POINTER(i), vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class Context:
    """One library context (device workspace, last-error text).  device=-1 makes a dry-run
    context that only checks arguments."""

    def __init__(self, device: int = 0, workspace_cap: int = 0):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.gw_create(C.byref(h), int(device), C.c_size_t(workspace_cap))
        if st != GW_OK:
            raise GwError(st, f"gw_create(device={device}) failed: {self.lib.gw_status_string(st).decode()}")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self.lib.gw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int, what: str):
        if st != GW_OK:
            msg = self.lib.gw_last_error(self.handle).decode()
            raise GwError(st, f"{what}: {self.lib.gw_status_string(st).decode()}: {msg}")

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.gw_workspace_bytes(self.handle))

    @property
    def graph_captures(self) -> int:
        """Batched-q graphs captured by this context so far (replays do not count)."""
        return int(self.lib.gw_graph_captures(self.handle))


_contexts: dict = {}


def context(device: Optional[int] = None) -> Context:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


# ---------------------------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------------------------
def _dev(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _shape(t, shape, name):
    """Raise ValueError unless tensor t (on any device) has exactly this shape.  Runs before any
    library or device call, so a mismatched buffer never reaches a kernel."""
    got = tuple(int(x) for x in getattr(t, "shape", ()))
    want = tuple(int(x) for x in shape)
    if got != want:
        raise ValueError(f"{name} has shape {got}, expected {want}")


def _ndim(t, nd, name):
    got = tuple(int(x) for x in getattr(t, "shape", ()))
    if len(got) != nd:
        raise ValueError(f"{name} must have {nd} dimensions, got shape {got}")
    return got


def _len(a, n, name):
    m = int(np.size(a))
    if m != int(n):
        raise ValueError(f"{name} has {m} entries, expected {int(n)}")


def _nr_of(n) -> int:
    nt = tuple(int(x) for x in (n if np.ndim(n) else (n, n, n)))
    if len(nt) != 3:
        raise ValueError(f"grid must have three lengths, got {nt}")
    return nt[0] * nt[1] * nt[2]


def _miller_rows(miller, name="g_miller"):
    m = np.asarray(miller)
    if m.ndim != 2 or m.shape[1] != 3:
        raise ValueError(f"{name} must be [ng][3], got shape {m.shape}")
    return m.shape[0]


def _orbitals(psi_v, psi_c, e_v, e_c, nr=None):
    """(nv, nc, nr) of an occupied/unoccupied pair of orbital arrays, checked against each other,
    against the energies and (if given) against the grid size."""
    nv, nrv = _ndim(psi_v, 2, "psi_v")
    nc, nrc = _ndim(psi_c, 2, "psi_c")
    if nrv != nrc:
        raise ValueError(f"psi_v has {nrv} grid points per band, psi_c {nrc}")
    if nr is not None and nrv != nr:
        raise ValueError(f"orbitals have {nrv} grid points, the grid has {nr}")
    _len(e_v, nv, "e_v")
    _len(e_c, nc, "e_c")
    return nv, nc, nrv


def _host_f64(a, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(C.c_void_p)


def _host_i32(a, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(C.c_void_p)


def _stream(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _opts(precision="fp32", prefactor=1.0, accumulate=False, tile=-1) -> Opts:
    o = Opts()
    load().gw_opts_default(C.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.prefactor = float(prefactor)
    o.accumulate = 1 if accumulate else 0
    o.tile = int(tile)
    return o


def _grid(n: Sequence[int], a_bohr: float) -> Grid:
    return Grid(int(n[0]), int(n[1]), int(n[2]), float(a_bohr))


def tile_names():
    lib = load()
    return [lib.gw_tile_name(i).decode() for i in range(lib.gw_tile_count())]


def mfma_rate(words, n_iter, grid, out=None, ctx: Optional[Context] = None):
    """One launch of the MFMA-only rate kernel (gw_mfma_rate): `words` a device int32 tensor of 4096
    BF16 pairs, `out` grid * 512 floats.  Executed flop: grid * 8 * n_iter * 393216."""
    import torch
    if words.numel() != 4096:
        raise ValueError("words must hold 4096 uint32 words")
    if out is not None:
        _shape(out, (int(grid) * 512,), "out")
    else:
        out = torch.empty(int(grid) * 512, dtype=torch.float32, device=words.device)
    ctx = ctx or context(words.device.index)
    st = ctx.lib.gw_mfma_rate(ctx.handle, _dev(words, torch.int32, "words"), int(n_iter), int(grid),
                              _dev(out, torch.float32, "out"), _stream(words))
    ctx.check(st, "gw_mfma_rate")
    return out


def default_tile_name(precision="fp32", nr=0):
    lib = load()
    t = lib.gw_default_tile(PRECISIONS[precision] if isinstance(precision, str) else int(precision), int(nr))
    return lib.gw_tile_name(t).decode() if t >= 0 else ""


# ---------------------------------------------------------------------------------------------
# entry points (same names as the C ABI without the gw_ prefix)
# ---------------------------------------------------------------------------------------------
def pair_products(psi_v, psi_c, e_v, e_c, prefactor=1.0, out=None, ctx: Optional[Context] = None):
    import torch
    nv, nc, nr = _orbitals(psi_v, psi_c, e_v, e_c)
    if out is not None:
        _shape(out, (nv * nc, nr), "f_out")
    else:
        out = torch.empty((nv * nc, nr), dtype=torch.complex64, device=psi_v.device)
    ctx = ctx or context(psi_v.device.index)
    ev, pev = _host_f64(e_v, "e_v")
    ec, pec = _host_f64(e_c, "e_c")
    st = ctx.lib.gw_pair_products(ctx.handle, _dev(psi_v, torch.complex64, "psi_v"), nv,
                                  _dev(psi_c, torch.complex64, "psi_c"), nc, nr, pev, pec, float(prefactor),
                                  _dev(out, torch.complex64, "f_out"), _stream(psi_v))
    ctx.check(st, "gw_pair_products")
    return out


def polarizability_r(psi_v, psi_c, e_v, e_c, precision="fp32", prefactor=1.0, accumulate=False, tile=-1, out=None,
                     ctx: Optional[Context] = None):
    import torch
    nv, nc, nr = _orbitals(psi_v, psi_c, e_v, e_c)
    if out is not None:
        _shape(out, (nr, nr), "p_rr")
    else:
        out = torch.empty((nr, nr), dtype=torch.complex64, device=psi_v.device)
    ctx = ctx or context(psi_v.device.index)
    ev, pev = _host_f64(e_v, "e_v")
    ec, pec = _host_f64(e_c, "e_c")
    o = _opts(precision, prefactor, accumulate, tile)
    st = ctx.lib.gw_polarizability_r(ctx.handle, _dev(psi_v, torch.complex64, "psi_v"), nv,
                                     _dev(psi_c, torch.complex64, "psi_c"), nc, nr, pev, pec, C.byref(o),
                                     _dev(out, torch.complex64, "p_rr"), _stream(psi_v))
    ctx.check(st, "gw_polarizability_r")
    return out


def polarizability_r_noalloc(psi_v, psi_c, e_v, e_c, out, precision="fp32", prefactor=1.0, accumulate=False, tile=-1,
                             ctx: Optional[Context] = None):
    """gw_polarizability_r_noalloc: the update into the caller's `out` [nr][nr], with the library's fixed
    scratch array instead of any allocation (tile -1: the precision's default tile)."""
    import torch
    nv, nc, nr = _orbitals(psi_v, psi_c, e_v, e_c)
    _shape(out, (nr, nr), "p_rr")
    ctx = ctx or context(psi_v.device.index)
    ev, pev = _host_f64(e_v, "e_v")
    ec, pec = _host_f64(e_c, "e_c")
    o = _opts(precision, prefactor, accumulate, tile)
    st = ctx.lib.gw_polarizability_r_noalloc(ctx.handle, _dev(psi_v, torch.complex64, "psi_v"), nv,
                                             _dev(psi_c, torch.complex64, "psi_c"), nc, nr, pev, pec, C.byref(o),
                                             _dev(out, torch.complex64, "p_rr"), _stream(psi_v))
    ctx.check(st, "gw_polarizability_r_noalloc")
    return out


def sphere_transform(p_rr, n, miller, out=None, hermitian=False, ctx: Optional[Context] = None):
    """P~ on the sphere from P(r,r'); hermitian=True calls gw_sphere_transform_herm, which reads only the
    upper triangle of a Hermitian P."""
    import torch
    nr = _nr_of(n)
    ng = _miller_rows(miller)
    _shape(p_rr, (nr, nr), "p_rr")
    m, pm = _host_i32(miller, "g_miller")
    if out is not None:
        _shape(out, (ng, ng), "p_gg")
    else:
        out = torch.empty((ng, ng), dtype=torch.complex64, device=p_rr.device)
    ctx = ctx or context(p_rr.device.index)
    fn = ctx.lib.gw_sphere_transform_herm if hermitian else ctx.lib.gw_sphere_transform
    st = fn(ctx.handle, _dev(p_rr, torch.complex64, "p_rr"), _grid(n, 1.0), pm, ng, _dev(out, torch.complex64, "p_gg"),
            _stream(p_rr))
    ctx.check(st, "gw_sphere_transform_herm" if hermitian else "gw_sphere_transform")
    return out


def polarizability(psi_v, psi_c, e_v, e_c, n, a_bohr, q, miller, precision="fp32", prefactor=1.0, accumulate=False,
                   tile=-1, p_rr=None, out=None, ctx: Optional[Context] = None):
    import torch
    nr = _nr_of(n)
    nv, nc, _ = _orbitals(psi_v, psi_c, e_v, e_c, nr)
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    if p_rr is not None:
        _shape(p_rr, (nr, nr), "p_rr")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    if out is not None:
        _shape(out, (ng, ng), "p_gg")
    else:
        out = torch.empty((ng, ng), dtype=torch.complex64, device=psi_v.device)
    ctx = ctx or context(psi_v.device.index)
    ev, pev = _host_f64(e_v, "e_v")
    ec, pec = _host_f64(e_c, "e_c")
    o = _opts(precision, prefactor, accumulate, tile)
    prr = C.c_void_p(None) if p_rr is None else _dev(p_rr, torch.complex64, "p_rr")
    st = ctx.lib.gw_polarizability(ctx.handle, _dev(psi_v, torch.complex64, "psi_occ"), nv,
                                   _dev(psi_c, torch.complex64, "psi_unocc"), nc, pev, pec, _grid(n, a_bohr), pq, pm,
                                   ng, C.byref(o), prr, _dev(out, torch.complex64, "p_gg"), _stream(psi_v))
    ctx.check(st, "gw_polarizability")
    return out


def epsilon(p_gg, n, a_bohr, q, miller, head=1.0, out=None, ctx: Optional[Context] = None):
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(p_gg, (ng, ng), "p_gg")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    if out is not None:
        _shape(out, (ng, ng), "eps_out")
    else:
        out = torch.empty((ng, ng), dtype=torch.complex128, device=p_gg.device)
    ctx = ctx or context(p_gg.device.index)
    st = ctx.lib.gw_epsilon(ctx.handle, _dev(p_gg, torch.complex64, "p_gg"), ng, _grid(n, a_bohr), pq, pm,
                            float(head), _dev(out, torch.complex128, "eps_out"), _stream(p_gg))
    ctx.check(st, "gw_epsilon")
    return out


def eps_inverse(p_gg, n, a_bohr, q, miller, head=1.0, out=None, ctx: Optional[Context] = None):
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(p_gg, (ng, ng), "p_gg")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    if out is not None:
        _shape(out, (ng, ng), "eps_inv")
    else:
        out = torch.empty((ng, ng), dtype=torch.complex128, device=p_gg.device)
    ctx = ctx or context(p_gg.device.index)
    st = ctx.lib.gw_eps_inverse(ctx.handle, _dev(p_gg, torch.complex64, "p_gg"), ng, _grid(n, a_bohr), pq, pm,
                                float(head), _dev(out, torch.complex128, "eps_inv"), _stream(p_gg))
    ctx.check(st, "gw_eps_inverse")
    return out


def hpd_inverse(a, out=None, ctx: Optional[Context] = None):
    import torch
    n = _ndim(a, 2, "a")[0]
    _shape(a, (n, n), "a")
    if out is not None:
        _shape(out, (n, n), "out")
    else:
        out = torch.empty_like(a)
    ctx = ctx or context(a.device.index)
    st = ctx.lib.gw_hpd_inverse(ctx.handle, _dev(a, torch.complex128, "a"), n, _dev(out, torch.complex128, "out"),
                                _stream(a))
    ctx.check(st, "gw_hpd_inverse")
    return out


def autotune(psi_v, psi_c, e_v, e_c, precision="bf16", p_scratch=None, ctx: Optional[Context] = None):
    """Times every update tile of `precision` on these inputs; returns (best tile, {name: ms})."""
    import torch
    nv, nc, nr = _orbitals(psi_v, psi_c, e_v, e_c)
    if p_scratch is not None:
        _shape(p_scratch, (nr, nr), "p_scratch")
    ctx = ctx or context(psi_v.device.index)
    if p_scratch is None:
        p_scratch = torch.empty((nr, nr), dtype=torch.complex64, device=psi_v.device)
    ev, pev = _host_f64(e_v, "e_v")
    ec, pec = _host_f64(e_c, "e_c")
    ntile = ctx.lib.gw_tile_count()
    times = (C.c_double * ntile)()
    best = C.c_int(-1)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    st = ctx.lib.gw_autotune(ctx.handle, _dev(psi_v, torch.complex64, "psi_v"), nv,
                             _dev(psi_c, torch.complex64, "psi_c"), nc, nr, pev, pec, prec,
                             _dev(p_scratch, torch.complex64, "p_scratch"), C.byref(best), times, _stream(psi_v))
    ctx.check(st, "gw_autotune")
    names = tile_names()
    return best.value, {names[t]: times[t] for t in range(ntile) if times[t] >= 0}


def orbitals_to_grid(coeff, n, pw_miller, out=None, ctx: Optional[Context] = None):
    """psi [nb][N_r] complex64 on the grid from plane-wave coefficients [nb][npw] on the device."""
    import torch
    nb, npw = _ndim(coeff, 2, "coeff")
    if _miller_rows(pw_miller, "pw_miller") != npw:
        raise ValueError(f"pw_miller has {np.asarray(pw_miller).shape[0]} rows for {npw} coefficients")
    m, pm = _host_i32(pw_miller, "pw_miller")
    nt = tuple(int(x) for x in (n if np.ndim(n) else (n, n, n)))
    nr = _nr_of(nt)
    if out is not None:
        _shape(out, (nb, nr), "psi")
    if out is None:
        out = torch.empty((nb, nr), dtype=torch.complex64, device=coeff.device)
    ctx = ctx or context(coeff.device.index)
    st = ctx.lib.gw_orbitals_to_grid(ctx.handle, _dev(coeff, torch.complex64, "coeff"), nb, npw, _grid(nt, 1.0), pm,
                                     _dev(out, torch.complex64, "psi"), _stream(coeff))
    ctx.check(st, "gw_orbitals_to_grid")
    return out


def plasmon_pole(eps_inv, n, a_bohr, q, miller, psi_v, occupation=1.0, n_modes=8, tol=1e-10, max_iter=1000,
                 ctx: Optional[Context] = None):
    """The n_modes most negative eigenpairs of S = sqrt(V)(eps^-1 - I)sqrt(V) and their sum-rule
    frequencies.  Returns (sigma [n_modes] f64, omega [n_modes] f64, modes [ng][n_modes] c128 on the
    device, iterations, final relative residual)."""
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(eps_inv, (ng, ng), "eps_inv")
    _ndim(psi_v, 2, "psi_v")
    if psi_v.shape[1] != _nr_of(n):
        raise ValueError(f"psi_v has {psi_v.shape[1]} grid points, the grid has {_nr_of(n)}")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    dev = eps_inv.device
    sigma = torch.empty(n_modes, dtype=torch.float64, device=dev)
    omega = torch.empty(n_modes, dtype=torch.float64, device=dev)
    modes = torch.empty((ng, n_modes), dtype=torch.complex128, device=dev)
    ctx = ctx or context(dev.index)
    its, res = C.c_int(0), C.c_double(0.0)
    st = ctx.lib.gw_plasmon_pole(ctx.handle, _dev(eps_inv, torch.complex128, "eps_inv"), ng, _grid(n, a_bohr), pq, pm,
                                 _dev(psi_v, torch.complex64, "psi_v"), psi_v.shape[0], float(occupation), int(n_modes),
                                 float(tol), int(max_iter), _dev(sigma, torch.float64, "sigma"),
                                 _dev(omega, torch.float64, "omega"), _dev(modes, torch.complex128, "modes"),
                                 C.byref(its), C.byref(res), _stream(eps_inv))
    ctx.check(st, "gw_plasmon_pole")
    return sigma, omega, modes, its.value, res.value


def pp_eps_inverse(eps_inv_static, n, a_bohr, q, miller, modes, sigma, omega, freqs, out=None,
                   ctx: Optional[Context] = None):
    """eps^-1(w) of the pole form for each frequency in freqs (Hartree): [nf][ng][ng] complex128."""
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(eps_inv_static, (ng, ng), "eps_inv_static")
    nm = _ndim(modes, 2, "modes")[1]
    _shape(modes, (ng, nm), "modes")
    _shape(sigma, (nm,), "sigma")
    _shape(omega, (nm,), "omega")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    fr, pf = _host_f64(np.atleast_1d(np.asarray(freqs, np.float64)), "freqs")
    if out is not None:
        _shape(out, (len(fr), ng, ng), "out")
    if out is None:
        out = torch.empty((len(fr), ng, ng), dtype=torch.complex128, device=modes.device)
    ctx = ctx or context(modes.device.index)
    st = ctx.lib.gw_pp_eps_inverse(ctx.handle, _dev(eps_inv_static, torch.complex128, "eps_inv_static"), ng,
                                   _grid(n, a_bohr), pq, pm, _dev(modes, torch.complex128, "modes"),
                                   _dev(sigma, torch.float64, "sigma"), _dev(omega, torch.float64, "omega"), nm, pf,
                                   len(fr), _dev(out, torch.complex128, "out"), _stream(modes))
    ctx.check(st, "gw_pp_eps_inverse")
    return out


def sigma_static(psi_n, psi_v, n, a_bohr, q, miller, eps_inv=None, want_x=True,
                 ctx: Optional[Context] = None):
    """(sigma_x, sigma_sex) [nn][nn] complex128 on the device; sigma_sex is None without eps_inv and
    sigma_x is None when want_x is False."""
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    nr = _nr_of(n)
    nn, nrn = _ndim(psi_n, 2, "psi_n")
    nv, nrv = _ndim(psi_v, 2, "psi_v")
    if nrn != nr or nrv != nr:
        raise ValueError(f"psi_n / psi_v have {nrn} / {nrv} grid points, the grid has {nr}")
    if eps_inv is not None:
        _shape(eps_inv, (ng, ng), "eps_inv")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    dev = psi_n.device
    sx = torch.empty((nn, nn), dtype=torch.complex128, device=dev) if want_x else None
    ss = torch.empty((nn, nn), dtype=torch.complex128, device=dev) if eps_inv is not None else None
    ctx = ctx or context(dev.index)
    st = ctx.lib.gw_sigma_static(ctx.handle, _dev(psi_n, torch.complex64, "psi_n"), nn,
                                 _dev(psi_v, torch.complex64, "psi_v"), nv, _grid(n, a_bohr), pq, pm, ng,
                                 _dev(eps_inv, torch.complex128, "eps_inv") if eps_inv is not None else None,
                                 _dev(sx, torch.complex128, "sigma_x") if sx is not None else None,
                                 _dev(ss, torch.complex128, "sigma_sex") if ss is not None else None, _stream(psi_n))
    ctx.check(st, "gw_sigma_static")
    return sx, ss


def sigma_sex_modes(psi_n, psi_v, n, miller, modes, sigma, ctx: Optional[Context] = None):
    """Screened exchange [nn][nn] complex128 from the plasmon-pole modes (eigen form)."""
    import torch
    ng = _miller_rows(miller)
    nr = _nr_of(n)
    nn, nrn = _ndim(psi_n, 2, "psi_n")
    nv, nrv = _ndim(psi_v, 2, "psi_v")
    if nrn != nr or nrv != nr:
        raise ValueError(f"psi_n / psi_v have {nrn} / {nrv} grid points, the grid has {nr}")
    nm = _ndim(modes, 2, "modes")[1]
    _shape(modes, (ng, nm), "modes")
    _shape(sigma, (nm,), "sigma")
    m, pm = _host_i32(miller, "g_miller")
    out = torch.empty((nn, nn), dtype=torch.complex128, device=psi_n.device)
    ctx = ctx or context(psi_n.device.index)
    st = ctx.lib.gw_sigma_sex_modes(ctx.handle, _dev(psi_n, torch.complex64, "psi_n"), nn,
                                    _dev(psi_v, torch.complex64, "psi_v"), nv, _grid(n, 1.0), pm, ng,
                                    _dev(modes, torch.complex128, "modes"), _dev(sigma, torch.float64, "sigma"),
                                    modes.shape[1], _dev(out, torch.complex128, "sigma_sex"), _stream(psi_n))
    ctx.check(st, "gw_sigma_sex_modes")
    return out


def newton_inverse(a, tol=1e-11, max_iter=100, out=None, ctx: Optional[Context] = None):
    """Inverse by the Newton iteration; returns (inverse, iterations, max-change history)."""
    import torch
    n = _ndim(a, 2, "a")[0]
    _shape(a, (n, n), "a")
    if out is not None:
        _shape(out, (n, n), "out")
    else:
        out = torch.empty_like(a)
    ctx = ctx or context(a.device.index)
    its = C.c_int(0)
    hist = (C.c_double * max_iter)()
    st = ctx.lib.gw_newton_inverse(ctx.handle, _dev(a, torch.complex128, "a"), n, float(tol), int(max_iter),
                                   _dev(out, torch.complex128, "out"), C.byref(its), hist, _stream(a))
    ctx.check(st, "gw_newton_inverse")
    return out, its.value, [hist[i] for i in range(its.value)]


def eps_inverse_newton(p_gg, n, a_bohr, q, miller, head=1.0, tol=1e-11, max_iter=100, out=None,
                       ctx: Optional[Context] = None):
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(p_gg, (ng, ng), "p_gg")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    if out is not None:
        _shape(out, (ng, ng), "eps_inv")
    else:
        out = torch.empty((ng, ng), dtype=torch.complex128, device=p_gg.device)
    ctx = ctx or context(p_gg.device.index)
    its = C.c_int(0)
    hist = (C.c_double * max_iter)()
    st = ctx.lib.gw_eps_inverse_newton(ctx.handle, _dev(p_gg, torch.complex64, "p_gg"), ng, _grid(n, a_bohr), pq, pm,
                                       float(head), float(tol), int(max_iter), _dev(out, torch.complex128, "eps_inv"),
                                       C.byref(its), hist, _stream(p_gg))
    ctx.check(st, "gw_eps_inverse_newton")
    return out, its.value, [hist[i] for i in range(its.value)]


def polarizability_batched(psi_v, e_v, n, a_bohr, jobs, precision="fp32", prefactor=1.0, tile=-1, head=1.0,
                           ctx: Optional[Context] = None):
    """jobs: list of dicts with psi_c (device), e_c, q, miller (host), p_gg and optional eps_inv (device)."""
    import torch
    nr = _nr_of(n)
    nv, nrv = _ndim(psi_v, 2, "psi_occ")
    if nrv != nr:
        raise ValueError(f"psi_occ has {nrv} grid points, the grid has {nr}")
    _len(e_v, nv, "e_v")
    for j, job in enumerate(jobs):
        nc, nrc = _ndim(job["psi_c"], 2, f"jobs[{j}].psi_c")
        if nrc != nr:
            raise ValueError(f"jobs[{j}].psi_c has {nrc} grid points, the grid has {nr}")
        _len(job["e_c"], nc, f"jobs[{j}].e_c")
        _len(job["q"], 3, f"jobs[{j}].q")
        ng = _miller_rows(job["miller"], f"jobs[{j}].miller")
        _shape(job["p_gg"], (ng, ng), f"jobs[{j}].p_gg")
        if job.get("eps_inv") is not None:
            _shape(job["eps_inv"], (ng, ng), f"jobs[{j}].eps_inv")
    ctx = ctx or context(psi_v.device.index)
    ev, pev = _host_f64(e_v, "e_v")
    keep = []
    arr = (QJob * len(jobs))()
    for j, job in enumerate(jobs):
        ec, pec = _host_f64(job["e_c"], "e_c")
        m, pm = _host_i32(job["miller"], "g_miller")
        keep += [ec, m]
        arr[j].psi_unocc = _dev(job["psi_c"], torch.complex64, "psi_unocc").value
        arr[j].nc = job["psi_c"].shape[0]
        arr[j].e_c = pec.value
        for d in range(3):
            arr[j].q[d] = float(job["q"][d])
        arr[j].g_miller = pm.value
        arr[j].ng = m.shape[0]
        arr[j].p_gg = _dev(job["p_gg"], torch.complex64, "p_gg").value
        ei = job.get("eps_inv")
        arr[j].eps_inv = None if ei is None else _dev(ei, torch.complex128, "eps_inv").value
    o = _opts(precision, prefactor, False, tile)
    st = ctx.lib.gw_polarizability_batched(ctx.handle, _dev(psi_v, torch.complex64, "psi_occ"), nv, pev,
                                           _grid(n, a_bohr), len(jobs), arr, C.byref(o), float(head),
                                           _stream(psi_v))
    ctx.check(st, "gw_polarizability_batched")
    return jobs


# ---------------------------------------------------------------------------------------------
# learned band tail
# ---------------------------------------------------------------------------------------------
class TailModel:
    """Device state of the band-tail MLP: BF16 weights, FP32 biases, feature normalisation and
    training box, and the Adam state on an FP32 master copy."""

    def __init__(self, master, norm, device="cuda:0", lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, rank=16,
                 ctx: Optional[Context] = None):
        import torch
        dev = torch.device(device)
        self.ctx = ctx or context(dev.index if dev.index is not None else 0)
        self.w = torch.empty(TAIL_NWEIGHT, dtype=torch.bfloat16, device=dev)
        self.b = torch.empty(TAIL_NBIAS, dtype=torch.float32, device=dev)
        if isinstance(norm, torch.Tensor):
            _shape(norm, (16,), "norm")
            self.norm = norm.to(device=dev, dtype=torch.float32).contiguous()
        else:
            self.norm = torch.as_tensor(np.asarray(norm, np.float32)).to(dev).contiguous()
        self.master = torch.as_tensor(np.asarray(master, np.float32)).to(dev).contiguous()
        self.m = torch.zeros(TAIL_NPARAM, dtype=torch.float32, device=dev)
        self.v = torch.zeros(TAIL_NPARAM, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(TAIL_NPARAM, dtype=torch.float32, device=dev)
        self.adam = Adam(C.c_void_p(self.master.data_ptr()), C.c_void_p(self.m.data_ptr()),
                         C.c_void_p(self.v.data_ptr()), C.c_void_p(self.grad.data_ptr()), 0, lr, beta1, beta2, eps)
        self.mlp = Mlp(C.c_void_p(self.w.data_ptr()), C.c_void_p(self.b.data_ptr()),
                       C.c_void_p(self.norm.data_ptr()), int(rank))
        st = self.ctx.lib.gw_tail_init(self.ctx.handle, C.byref(self.mlp), C.c_void_p(self.master.data_ptr()),
                                       _stream(self.master))
        self.ctx.check(st, "gw_tail_init")

    @property
    def step(self):
        return self.adam.step

    @property
    def rank(self):
        return self.mlp.rank

    @rank.setter
    def rank(self, r):
        if not 0 <= int(r) <= 16:
            raise ValueError("rank must be in [0, 16]")
        self.mlp.rank = int(r)

    def train_steps(self, feats, targets, order, losses):
        """gw_tail_train_steps: one graph-replayed step per entry of `order` (indices into feats/targets);
        losses (device float32 [len(feats)]) receives each step's loss at its system's index."""
        import torch
        nsys = len(feats)
        if len(targets) != nsys:
            raise ValueError("feats and targets differ in length")
        _shape(losses, (nsys,), "losses")
        ngs = np.zeros(nsys, np.int32)
        for j in range(nsys):
            ng = _ndim(feats[j], 2, f"feats[{j}]")[0]
            _shape(feats[j], (ng, 4), f"feats[{j}]")
            _shape(targets[j], (ng, ng), f"targets[{j}]")
            ngs[j] = ng
        order = np.ascontiguousarray(np.asarray(order, np.int64).astype(np.int32))
        if order.size and (order.min() < 0 or order.max() >= nsys):
            raise ValueError("order entries must index the systems")
        fp = (C.c_void_p * nsys)(*[_dev(f, torch.float32, "feat").value for f in feats])
        tp = (C.c_void_p * nsys)(*[_dev(t, torch.complex64, "target").value for t in targets])
        st = self.ctx.lib.gw_tail_train_steps(self.ctx.handle, C.byref(self.mlp), C.byref(self.adam), nsys, fp, tp,
                                              ngs.ctypes.data_as(C.c_void_p), int(order.size),
                                              order.ctypes.data_as(C.c_void_p),
                                              _dev(losses, torch.float32, "losses"), _stream(losses))
        self.ctx.check(st, "gw_tail_train_steps")
        return losses

    def residual_parts(self, feat, target, out=None):
        """(||offdiag(dP~ - T)||^2, ||offdiag T||^2, ||diag(dP~ - T)||^2, ||diag T||^2) as a device float32 [4]."""
        import torch
        ng = _ndim(feat, 2, "feat")[0]
        _shape(feat, (ng, 4), "feat")
        _shape(target, (ng, ng), "target")
        if out is not None:
            _shape(out, (4,), "parts")
        else:
            out = torch.empty(4, dtype=torch.float32, device=feat.device)
        st = self.ctx.lib.gw_tail_residual_parts(self.ctx.handle, C.byref(self.mlp), _dev(feat, torch.float32, "feat"),
                                                 _dev(target, torch.complex64, "target"), ng,
                                                 _dev(out, torch.float32, "parts"), _stream(feat))
        self.ctx.check(st, "gw_tail_residual_parts")
        return out

    def forward(self, feat, out=None):
        import torch
        ng = _ndim(feat, 2, "feat")[0]
        _shape(feat, (ng, 4), "feat")
        if out is not None:
            _shape(out, (ng, 33), "out")
        else:
            out = torch.empty((ng, 33), dtype=torch.float32, device=feat.device)
        st = self.ctx.lib.gw_tail_forward(self.ctx.handle, C.byref(self.mlp), _dev(feat, torch.float32, "feat"), ng,
                                          _dev(out, torch.float32, "out"), _stream(feat))
        self.ctx.check(st, "gw_tail_forward")
        return out

    def train_step(self, feat, target, loss_out=None):
        import torch
        ng = _ndim(feat, 2, "feat")[0]
        _shape(feat, (ng, 4), "feat")
        _shape(target, (ng, ng), "target")
        if loss_out is not None:
            _shape(loss_out, (1,), "loss_out")
        else:
            loss_out = torch.empty(1, dtype=torch.float32, device=feat.device)
        st = self.ctx.lib.gw_tail_train_step(self.ctx.handle, C.byref(self.mlp), C.byref(self.adam),
                                             _dev(feat, torch.float32, "feat"), _dev(target, torch.complex64, "target"),
                                             ng, _dev(loss_out, torch.float32, "loss_out"), _stream(feat))
        self.ctx.check(st, "gw_tail_train_step")
        return loss_out

    def loss(self, feat, target, loss_out=None):
        import torch
        ng = _ndim(feat, 2, "feat")[0]
        _shape(feat, (ng, 4), "feat")
        _shape(target, (ng, ng), "target")
        if loss_out is not None:
            _shape(loss_out, (1,), "loss_out")
        else:
            loss_out = torch.empty(1, dtype=torch.float32, device=feat.device)
        st = self.ctx.lib.gw_tail_loss(self.ctx.handle, C.byref(self.mlp), _dev(feat, torch.float32, "feat"),
                                       _dev(target, torch.complex64, "target"), ng,
                                       _dev(loss_out, torch.float32, "loss_out"), _stream(feat))
        self.ctx.check(st, "gw_tail_loss")
        return loss_out

    def correct(self, p_trunc, feat, out=None):
        """Returns (p_corr, used_fallback); with the fallback p_corr is None."""
        import torch
        ng = _ndim(p_trunc, 2, "p_trunc")[0]
        _shape(p_trunc, (ng, ng), "p_trunc")
        _shape(feat, (ng, 4), "feat")
        if out is not None:
            _shape(out, (ng, ng), "p_corr")
        else:
            out = torch.empty_like(p_trunc)
        fb = C.c_int(0)
        st = self.ctx.lib.gw_tail_correct(self.ctx.handle, C.byref(self.mlp), _dev(p_trunc, torch.complex64, "p_trunc"),
                                          ng, _dev(feat, torch.float32, "feat"), _dev(out, torch.complex64, "p_corr"),
                                          C.byref(fb), _stream(p_trunc))
        self.ctx.check(st, "gw_tail_correct")
        return (None, True) if fb.value else (out, False)


def tail_fit_norm(feats, out=None, ctx: Optional[Context] = None):
    """gw_tail_fit_norm: mean, std, min and max of the raw features over all rows of `feats` (device
    float32 [ng_i][4] each), as a device float32 [16]."""
    import torch
    nsys = len(feats)
    if nsys == 0:
        raise ValueError("no feature arrays")
    ngs = np.zeros(nsys, np.int32)
    for j, f in enumerate(feats):
        ng = _ndim(f, 2, f"feats[{j}]")[0]
        _shape(f, (ng, 4), f"feats[{j}]")
        ngs[j] = ng
    if out is not None:
        _shape(out, (16,), "norm")
    else:
        out = torch.empty(16, dtype=torch.float32, device=feats[0].device)
    ctx = ctx or context(feats[0].device.index)
    fp = (C.c_void_p * nsys)(*[_dev(f, torch.float32, "feat").value for f in feats])
    st = ctx.lib.gw_tail_fit_norm(ctx.handle, nsys, fp, ngs.ctypes.data_as(C.c_void_p),
                                  _dev(out, torch.float32, "norm"), _stream(feats[0]))
    ctx.check(st, "gw_tail_fit_norm")
    return out


def tail_target(p_full, p_trunc, out=None, ctx: Optional[Context] = None):
    import torch
    ng = _ndim(p_full, 2, "p_full")[0]
    _shape(p_full, (ng, ng), "p_full")
    _shape(p_trunc, (ng, ng), "p_trunc")
    if out is not None:
        _shape(out, (ng, ng), "target")
    else:
        out = torch.empty_like(p_full)
    ctx = ctx or context(p_full.device.index)
    st = ctx.lib.gw_tail_target(ctx.handle, _dev(p_full, torch.complex64, "p_full"),
                                _dev(p_trunc, torch.complex64, "p_trunc"), ng, _dev(out, torch.complex64, "target"),
                                _stream(p_full))
    ctx.check(st, "gw_tail_target")
    return out


def tail_features(p_gg, n, a_bohr, q, miller, nc, e_max, out=None, ctx: Optional[Context] = None):
    import torch
    ng = _miller_rows(miller)
    _len(q, 3, "q")
    _shape(p_gg, (ng, ng), "p_gg")
    m, pm = _host_i32(miller, "g_miller")
    qa, pq = _host_f64(q, "q")
    if out is not None:
        _shape(out, (ng, 4), "feat")
    else:
        out = torch.empty((ng, 4), dtype=torch.float32, device=p_gg.device)
    ctx = ctx or context(p_gg.device.index)
    st = ctx.lib.gw_tail_features(ctx.handle, _dev(p_gg, torch.complex64, "p_gg"), ng, _grid(n, a_bohr), pq, pm,
                                  int(nc), float(e_max), _dev(out, torch.float32, "feat"), _stream(p_gg))
    ctx.check(st, "gw_tail_features")
    return out
