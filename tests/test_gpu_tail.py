"""GPU tests of the learned band-tail correction: kernels against the FP64 MLP oracle, the
training-box fallback, and the gain of the trained network on the 24^3 evaluation systems."""
import numpy as np
import pytest

import gwsynth as gs
import oracle as orc
from oracle import mlp_oracle as mo

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_07772_amd as gw
    gw.load()
    return gw


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def c64(x):
    return dev(np.asarray(x).astype(np.complex64))


def random_case(n=257, seed=0):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(0.3, 2.7, n), rng.uniform(-13, -7, n), np.full(n, 0.1), np.full(n, 0.31)],
                 axis=1).astype(np.float32)
    mean, std = x.mean(axis=0), x.std(axis=0)
    std[std == 0] = 1.0
    norm = np.concatenate([mean, std, x.min(axis=0), x.max(axis=0)]).astype(np.float32)
    a = rng.standard_normal((n, 24)) + 1j * rng.standard_normal((n, 24))
    t = (-(a @ a.conj().T) * 1e-6).astype(np.complex64)                    # Hermitian NSD target
    t = 0.5 * (t + t.conj().T)
    return x, norm, t


def oracle_params(master):
    p = mo.unflatten(np.asarray(master, np.float64))
    for k in ("w1", "w2", "w3"):
        p[k] = mo.bf16_round(p[k])
    return p


def test_forward_matches_oracle(gw):
    x, norm, _ = random_case()
    master = gs.mlp_init(0)
    model = gw.TailModel(master, norm)
    o = model.forward(dev(x)).cpu().numpy()
    ref, _ = mo.forward(x.astype(np.float64), oracle_params(master), norm[:4].astype(np.float64),
                        norm[4:8].astype(np.float64))
    e = orc.rel_f(o, ref)
    print(f"forward rel_F = {e:.2e}")
    assert e < 1e-5


def test_loss_gradient_and_adam_match_oracle(gw):
    x, norm, t = random_case(seed=3)
    master = gs.mlp_init(1)
    lr = 1e-3
    model = gw.TailModel(master, norm, lr=lr)
    fx, ft = dev(x), dev(t)
    l0 = float(model.loss(fx, ft).cpu().numpy()[0])
    lt = float(model.train_step(fx, ft).cpu().numpy()[0])
    torch.cuda.synchronize()
    params = oracle_params(master)
    mean, std = norm[:4].astype(np.float64), norm[4:8].astype(np.float64)
    o, cache = mo.forward(x.astype(np.float64), params, mean, std)
    s = np.exp(x[:, 1].astype(np.float64))
    ref_loss = mo.loss(o, s, t.astype(np.complex128))
    print(f"loss gpu {l0:.7f} / {lt:.7f} oracle {ref_loss:.7f}")
    assert abs(l0 - ref_loss) < 1e-5 * abs(ref_loss) and abs(lt - ref_loss) < 1e-5 * abs(ref_loss)
    g_ref = mo.flatten(mo.backward(mo.loss_grad_o(o, s, t.astype(np.complex128)), params, cache))
    g = model.grad.cpu().numpy().astype(np.float64)
    e = orc.rel_f(g, g_ref)
    print(f"gradient rel_F = {e:.2e}")
    assert e < 1e-4
    # one Adam step from zero moments, on the GPU's own gradient (the update is then exact to FP32)
    new, _, _, p = mo.adam(master.astype(np.float64), np.zeros(g.size), np.zeros(g.size), g, 1, lr)
    got = model.master.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - new)) <= 1e-6 * np.max(np.abs(new))
    w = model.w.float().cpu().numpy().astype(np.float64)
    w_ref = np.concatenate([p["w1"].ravel(), p["w2"].ravel(), p["w3"].ravel()])
    assert np.mean(w != w_ref) < 1e-3           # BF16 ties may round apart when the FP32 masters differ by an ulp
    assert model.step == 1


def test_features_target_and_correction(gw):
    s = gs.make_system(8, 4, 48, r2_psi=6.0, seed=9).as_c64()
    pv, pc = c64(s.psi_v), c64(s.psi_c)
    p12 = gw.polarizability(pv, pc[:12].contiguous(), s.e_v, s.e_c[:12], s.n, s.a_bohr, s.q, s.miller)
    p48 = gw.polarizability(pv, pc, s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)
    feat = gw.tail_features(p12, s.n, s.a_bohr, s.q, s.miller, 12, float(s.e_c[11]))
    t = gw.tail_target(p48, p12)
    torch.cuda.synchronize()
    a, b = p12.cpu().numpy().astype(np.complex128), p48.cpu().numpy().astype(np.complex128)
    f_ref = mo.features(a, s.q, s.miller, s.a_bohr, 12, float(s.e_c[11]))
    assert np.max(np.abs(feat.cpu().numpy() - f_ref) / np.maximum(1.0, np.abs(f_ref))) < 1e-6
    t_ref = 0.5 * (b + b.conj().T) - 0.5 * (a + a.conj().T)
    assert orc.rel_f(t.cpu().numpy(), t_ref) < 1e-6
    fv = feat.cpu().numpy()
    norm = np.concatenate([fv.mean(0), np.where(fv.std(0) > 0, fv.std(0), 1.0), fv.min(0), fv.max(0)]).astype(np.float32)
    master = gs.mlp_init(2)
    model = gw.TailModel(master, norm)
    corr, fb = model.correct(p12, feat)
    assert not fb
    o, _ = mo.forward(fv.astype(np.float64), oracle_params(master), norm[:4].astype(np.float64),
                      norm[4:8].astype(np.float64))
    ref = a + mo.correction(o, np.exp(fv[:, 1].astype(np.float64)))
    e = orc.rel_f(corr.cpu().numpy(), ref)
    print(f"corrected build rel_F = {e:.2e}")
    assert e < 1e-5
    # out of the training box (E_max far beyond the trained range): the caller must run the plain sum
    far = gw.tail_features(p12, s.n, s.a_bohr, s.q, s.miller, 12, 10.0)
    corr2, fb2 = model.correct(p12, far)
    assert fb2 and corr2 is None


def test_reduced_rank_correction_gradient_and_parts(gw):
    """rank 5: the correction, the gradient and the residual parts against the oracle at the same rank."""
    x, norm, t = random_case(n=301, seed=5)
    master = gs.mlp_init(3)
    model = gw.TailModel(master, norm, rank=5)
    fx, ft = dev(x), dev(t)
    params = oracle_params(master)
    mean, std = norm[:4].astype(np.float64), norm[4:8].astype(np.float64)
    o, cache = mo.forward(x.astype(np.float64), params, mean, std)
    s = np.exp(x[:, 1].astype(np.float64))
    p0 = np.zeros((301, 301), np.complex64)
    corr, fb = model.correct(dev(p0), fx)
    assert not fb
    ref = mo.correction(o, s, rank=5)
    e = orc.rel_f(corr.cpu().numpy(), ref)
    assert e < 1e-5, e
    parts = model.residual_parts(fx, ft).cpu().numpy().astype(np.float64)
    parts_ref = np.array(mo.residual_parts(o, s, t.astype(np.complex128), rank=5))
    print(f"rank 5: correction rel_F {e:.2e}, parts {parts} vs {parts_ref}")
    assert np.max(np.abs(parts - parts_ref) / parts_ref) < 1e-4
    model.train_step(fx, ft)
    torch.cuda.synchronize()
    g_ref = mo.flatten(mo.backward(mo.loss_grad_o(o, s, t.astype(np.complex128), rank=5), params, cache))
    g = model.grad.cpu().numpy().astype(np.float64)
    assert orc.rel_f(g, g_ref) < 1e-4
    # outputs of unused columns get exactly zero gradient: the W3 columns 6..16 and 22..32
    w3 = g[640 + 16384 + 128:640 + 16384 + 128 + 128 * 33].reshape(128, 33)
    assert np.all(w3[:, 6:17] == 0) and np.all(w3[:, 22:] == 0)


def test_fit_norm_matches_oracle(gw):
    rng = np.random.default_rng(12)
    feats = [np.stack([rng.uniform(0.2, 3.0, n), rng.uniform(-14, -6, n), np.full(n, 0.05 * (i + 1)),
                       np.full(n, 0.3)], axis=1).astype(np.float32) for i, n in enumerate((925, 700, 1))]
    got = gw.tail_fit_norm([dev(f) for f in feats]).cpu().numpy()
    ref = mo.fit_norm(feats)
    print("fit_norm", got, ref)
    np.testing.assert_allclose(got, ref, rtol=1e-6)
    assert got[7] == 1.0                       # E_max is constant over the set


def test_graph_training_equals_eager_steps(gw):
    """gw_tail_train_steps (graph replays) performs exactly the eager steps: same losses, same master
    weights and moments, bit for bit; a second epoch in another order captures no new graph."""
    cases = [random_case(n=n, seed=20 + i) for i, n in enumerate((150, 97, 150))]
    norm = cases[0][1]
    feats = [dev(c[0]) for c in cases]
    targets = [dev(c[2]) for c in cases]
    eager = gw.TailModel(gs.mlp_init(4), norm, lr=1e-3)
    graph = gw.TailModel(gs.mlp_init(4), norm, lr=1e-3)
    orders = [[2, 0, 1], [1, 2, 0, 0]]
    le = torch.zeros(3, dtype=torch.float32, device="cuda:0")
    lg = torch.zeros(3, dtype=torch.float32, device="cuda:0")
    ctx = graph.ctx
    for ep, order in enumerate(orders):
        for j in order:
            eager.train_step(feats[j], targets[j], loss_out=le[j:j + 1])
        graph.train_steps(feats, targets, order, lg)
        torch.cuda.synchronize()
        assert torch.equal(le, lg), (le, lg)
        if ep == 0:
            n_graphs = gw.load().gw_tail_graph_count(ctx.handle)
            assert n_graphs >= 3
    assert gw.load().gw_tail_graph_count(ctx.handle) == n_graphs
    assert eager.step == graph.step == 7
    for a, b in ((eager.master, graph.master), (eager.m, graph.m), (eager.v, graph.v), (eager.w, graph.w)):
        assert torch.equal(a, b)


@pytest.mark.timeout(900)
def test_training_and_gain_on_larger_systems(gw):
    """Train on 200 seeded 16^3 systems (Nc in {64, 96, 128}, each against 4 Nc; 180 train, 20 validation),
    then correct the 24^3 systems (Nv 32) truncated at Nc = 256 and compare them with the plain Nc = 1024 sum."""
    from paper_1810_07772_amd import tail
    entries = []
    for k in range(200):
        s = gs.tail_train_system(1000 + k)
        nc = (64, 96, 128)[k % 3]
        feat, target, _, _ = tail.pair_builds(c64(s.psi_v), c64(s.psi_c), s.e_v, s.e_c, s.n, s.a_bohr, s.q,
                                              s.miller, nc)
        entries.append(dict(feat=feat, target=target))
        if k % 50 == 0:
            print(f"[case] training system {k}", flush=True)
    train_e, val_e = entries[:180], entries[180:]
    norm = tail.fit_norm([e["feat"] for e in train_e])
    # the rank of the U U^H term is chosen on the validation systems among 16 and 0
    model, hist, report = tail.train_select_rank(gs.mlp_init(0), norm, train_e, val_e, 60, lr=3e-4,
                                                 log=lambda m: print(m, flush=True) if ("0/" in m or "rank" in m) else None)
    print(f"selected rank {model.rank}; validation parts {report}")
    assert hist[-1][1] < 0.5 * hist[0][1], hist
    gains = []
    for k in range(8):
        s = gs.tail_eval_system(2000 + k)
        pv, pc = c64(s.psi_v), c64(s.psi_c)
        p256 = gw.polarizability(pv, pc[:256], s.e_v, s.e_c[:256], s.n, s.a_bohr, s.q, s.miller)
        p1024 = gw.polarizability(pv, pc, s.e_v, s.e_c, s.n, s.a_bohr, s.q, s.miller)
        feat = gw.tail_features(p256, s.n, s.a_bohr, s.q, s.miller, 256, float(s.e_c[255]))
        pcorr, fb = model.correct(p256, feat)
        assert not fb, "evaluation features left the training box"
        a, b, c = (x.cpu().numpy().astype(np.complex128) for x in (p256, p1024, pcorr))
        D = lambda x: np.diag(np.diag(x))
        sv = orc.coulomb_sqrt(s.n, s.a_bohr, s.q, s.miller)
        inv = lambda x: orc.eps_inverse(orc.epsilon(0.5 * (x + x.conj().T), sv)) - np.eye(len(sv))
        ib = inv(b)
        row = dict(full=(orc.rel_f(a, b), orc.rel_f(c, b)), diag=(orc.rel_f(D(a), D(b)), orc.rel_f(D(c), D(b))),
                   offdiag=(orc.rel_f(a - D(a), b - D(b)), orc.rel_f(c - D(c), b - D(b))),
                   eps_inv=(orc.rel_f(inv(a), ib), orc.rel_f(inv(c), ib)))
        gains.append(row)
        print(f"eval {k}: " + "  ".join(f"{kk} {v[0]:.3f}->{v[1]:.3f}" for kk, v in row.items()), flush=True)
    for row in gains:
        assert row["full"][1] < row["full"][0]
        assert row["diag"][1] < 0.5 * row["diag"][0]
        assert row["offdiag"][1] <= row["offdiag"][0]
        assert row["eps_inv"][1] < 0.5 * row["eps_inv"][0]
