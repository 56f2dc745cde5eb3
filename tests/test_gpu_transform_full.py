"""The two sphere transforms at the 32^3 and 36^3 grids of the q batch and of the production build,
alone: a dense P(r,r') = sum_k a_k(r) conj(b_k(r')) of rank 4 (seeded complex factors, formed in
complex64 on the device), transformed to the whole sphere by the library, against the oracle's
direct grid sums of the factors on sampled rows and columns, including the first and last sphere
vectors."""
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


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,r2,q", [(32, 81.0, (1 / 16, 1 / 32, 1 / 64)), (36, 98.0, (0.0, 0.0, 0.0))])
def test_sphere_transform_sampled(gw, n, r2, q):
    grid = (n, n, n)
    nr = n ** 3
    rng = np.random.default_rng(n)
    a = (rng.standard_normal((4, nr)) + 1j * rng.standard_normal((4, nr))).astype(np.complex64)
    b = (rng.standard_normal((4, nr)) + 1j * rng.standard_normal((4, nr))).astype(np.complex64)
    mill = gs.sphere(grid, r2=r2, q=q)
    ng = len(mill)
    print(f"[case] {n}^3 ng={ng} q={q}", flush=True)
    dev = torch.device("cuda:0")
    at = torch.from_numpy(a).to(dev)
    bt = torch.from_numpy(b).to(dev)
    p = torch.matmul(at.transpose(0, 1).contiguous(), bt.conj().resolve_conj().contiguous())   # [nr][nr]
    torch.cuda.synchronize()
    out = gw.sphere_transform(p, grid, mill)
    torch.cuda.synchronize()
    del p
    rows = np.unique(np.concatenate([[0, 1, ng // 2, ng - 1], rng.choice(ng, 28, replace=False)]))
    cols = np.unique(np.concatenate([[0, 2, ng // 3, ng - 1], rng.choice(ng, 28, replace=False)]))
    got = out[torch.from_numpy(rows).to(dev)][:, torch.from_numpy(cols).to(dev)].cpu().numpy()
    ref = orc.to_sphere_factored(a.astype(np.complex128), b.astype(np.complex128), grid, mill[rows], mill[cols])
    e = orc.rel_f(got, ref)
    print(f"{n}^3: sampled {len(rows)} x {len(cols)} entries rel_F {e:.2e}")
    assert e < 5e-6
