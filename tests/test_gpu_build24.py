"""Parity of the whole build on the 24^3 grid of the learned tail's evaluation (N_r = 13824, Nv = 32,
Nc = 256, K = 8192, N_g = 3071, the transform length 24 = 4 x 6 on every axis), in the FP32 and the
default split-BF16 precision: sampled rows of P(r,r') over the full K (including both sides of a
128-point tile boundary and the last, partial tile), the whole P~ on the sphere against the
Adler-Wiser route of Eq.(gpsaceP), and the whole eps^-1 against LU of the oracle's own eps."""
import time

import numpy as np
import pytest

import gwsynth as gs
import oracle as orc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROWS = np.array([0, 1, 127, 128, 5000, 13695, 13696, 13823])


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_07772_amd as gw
    gw.load()
    t0 = time.time()
    s = gs.truncate(gs.tail_eval_system(2000), 256).as_c64()
    print(f"[case] 24^3 system nv={s.nv} nc={s.nc} ng={s.ng} ({time.time() - t0:.1f} s)", flush=True)
    rows_ref = orc.polarizability_r(s.psi_v, s.psi_c, s.e_v, s.e_c, rows=ROWS)
    pt_ref = orc.adler_wiser(s.psi_v, s.psi_c, s.e_v, s.e_c, s.n, s.miller)
    ei_ref = orc.eps_inverse(orc.epsilon(pt_ref, orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)))
    print(f"[case] 24^3 oracle done at {time.time() - t0:.1f} s", flush=True)
    dev = torch.device("cuda:0")
    return dict(gw=gw, s=s, pv=torch.from_numpy(s.psi_v.astype(np.complex64)).to(dev),
                pc=torch.from_numpy(s.psi_c.astype(np.complex64)).to(dev), rows_ref=rows_ref, pt_ref=pt_ref,
                ei_ref=ei_ref)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-4)])
def test_build_24(setup, prec, tol):
    gw, s = setup["gw"], setup["s"]
    print(f"[case] 24^3 build, {prec}", flush=True)
    prr = torch.empty((s.nr, s.nr), dtype=torch.complex64, device="cuda:0")
    pgg = gw.polarizability(setup["pv"], setup["pc"], s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller, precision=prec,
                            p_rr=prr)
    einv = gw.eps_inverse(pgg, s.n, s.a_bohr, s.q, s.miller)
    torch.cuda.synchronize()
    rows = prr[torch.from_numpy(ROWS).to(prr.device)].cpu().numpy()
    e_rows = orc.rel_f(rows, setup["rows_ref"])
    e_pt = orc.rel_f(pgg.cpu().numpy(), setup["pt_ref"])
    ei = einv.cpu().numpy()
    e_ei = orc.rel_f(ei, setup["ei_ref"])
    eye = np.eye(s.ng)
    e_eim = orc.rel_f(ei - eye, setup["ei_ref"] - eye)
    print(f"24^3 {prec}: P rows {e_rows:.2e}, P~ {e_pt:.2e}, eps^-1 {e_ei:.2e}, eps^-1 - I {e_eim:.2e}")
    assert e_rows < tol and e_pt < tol and e_ei < tol and e_eim < 10 * tol
