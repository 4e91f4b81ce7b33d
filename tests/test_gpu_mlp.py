"""The BF16 MLP kernels (MFMA GEMMs, reductions, Adam) against the CPU reference."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import mlp as m
    return m


def _data(seed, nf=34, npnt=3, B=1000, n_traj=5):
    import torch
    rng = np.random.default_rng(seed)
    feat = (0.5 * rng.normal(size=(n_traj, nf))).astype(np.float32)
    traj = rng.integers(0, n_traj, B).astype(np.int32)
    x = rng.normal(size=(B, npnt)).astype(np.float32)
    target = rng.normal(size=B).astype(np.float32)
    dev = [torch.from_numpy(a).cuda() for a in (feat, traj, x, target)]
    return (feat, traj, x, target), dev


def _blocks(n_in):
    lay, _ = ref.layout(n_in)
    return [(k, o, int(np.prod(s))) for k, (o, s) in lay.items()]


def test_gradients_match_cpu_reference(M):
    net = M.MLP(34, 3, seed=1)
    (feat, traj, x, target), dev = _data(2)
    g, ls = net.grad(*dev)
    g = g.cpu().numpy().astype(np.float64)
    theta = net.get_params().astype(np.float64)
    loss, gr = ref.loss_and_grad(theta, feat, traj, x, target, bf=True)
    assert abs(ls.item() / len(x) - loss) <= 1e-4 * loss
    for name, o, n in _blocks(37):
        a, b = g[o:o + n], gr[o:o + n]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("grad %s: rel err %.2e" % (name, err), flush=True)
        assert err < 5e-3, name


def test_forward_folded_matches_cpu_reference(M):
    net = M.MLP(34, 3, seed=4)
    (feat, traj, x, target), dev = _data(5, B=777)
    y = net.forward(dev[0], dev[1], dev[2]).cpu().numpy().astype(np.float64)
    yr, _ = ref.forward(net.get_params().astype(np.float64), feat, traj, x, bf=True)
    err = np.max(np.abs(y - yr)) / np.max(np.abs(yr))
    print("forward rel err %.2e" % err, flush=True)
    assert err < 5e-3


@pytest.mark.parametrize("nf,npnt,B,n_traj", [(34, 3, 1, 1), (34, 3, 31, 2), (34, 3, 4099, 7), (1, 8, 200, 1),
                                             (34, 9, 333, 3)])
def test_forward_paths_match_cpu_reference(M, nf, npnt, B, n_traj):
    """Inference at ragged sizes: n_point <= 8 runs the fused kernel (activations never
    leave the registers), n_point = 9 the layer-by-layer path; both against the CPU
    reference with BF16 rounding."""
    net = M.MLP(nf, npnt, seed=5 + npnt)
    (feat, traj, x, target), dev = _data(6 + B, nf=nf, npnt=npnt, B=B, n_traj=n_traj)
    y = net.forward(dev[0], dev[1], dev[2]).cpu().numpy().astype(np.float64)
    yr, _ = ref.forward(net.get_params().astype(np.float64), feat, traj, x, bf=True)
    err = np.max(np.abs(y - yr)) / max(np.max(np.abs(yr)), 1e-30)
    print("forward nf %d np %d B %d: rel err %.2e" % (nf, npnt, B, err), flush=True)
    assert err < 5e-3


def test_forward_grid_equals_forward(M):
    """The grid form (every trajectory at every point of one table) gives exactly what the
    per-point form gives on the materialised inputs."""
    import torch
    net = M.MLP(38, 3, seed=17)
    rng = np.random.default_rng(18)
    feat = torch.from_numpy((0.5 * rng.normal(size=(5, 38))).astype(np.float32)).cuda()
    table = torch.from_numpy(rng.normal(size=(1000, 3)).astype(np.float32)).cuda()
    yg = net.forward_grid(feat, table)
    traj = torch.arange(5, dtype=torch.int32, device="cuda").repeat_interleave(1000)
    yp = net.forward(feat, traj, table.repeat(5, 1).contiguous()).view(5, 1000)
    assert torch.equal(yg, yp)


def test_adam_step_matches_cpu_reference(M):
    import torch
    net = M.MLP(34, 3, seed=7)
    theta0 = net.get_params().astype(np.float64)
    rng = np.random.default_rng(8)
    g = (1e-3 * rng.normal(size=theta0.size)).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    net.adam(gd, lr=1e-3)
    net.adam(gd, lr=1e-3)
    t1, m1, m2 = ref.adam(theta0, np.zeros_like(theta0), np.zeros_like(theta0), g.astype(np.float64), 1, 1e-3)
    t2, m1, m2 = ref.adam(t1, m1, m2, g.astype(np.float64), 2, 1e-3)
    got = net.get_params().astype(np.float64)
    assert np.max(np.abs(got - t2)) < 1e-6
    a1, a2, step = net.get_adam()
    assert step == 2 and np.allclose(a1, m1, rtol=1e-5, atol=1e-12)


def test_training_reduces_loss(M):
    import torch
    net = M.MLP(4, 3, seed=11)
    rng = np.random.default_rng(12)
    n_traj, B = 8, 4096
    feat = rng.normal(size=(n_traj, 4)).astype(np.float32)
    fd = torch.from_numpy(feat).cuda()
    losses = []
    for it in range(300):
        traj = rng.integers(0, n_traj, B).astype(np.int32)
        x = rng.uniform(-2, 2, size=(B, 3)).astype(np.float32)
        t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] + 0.3 * feat[traj, 0]).astype(np.float32)
        l = net.train_step(fd, torch.from_numpy(traj).cuda(), torch.from_numpy(x).cuda(),
                           torch.from_numpy(t).cuda(), lr=2e-3)
        losses.append(l.item())
    print("loss %.4f -> %.4f" % (np.mean(losses[:10]), np.mean(losses[-10:])), flush=True)
    assert np.mean(losses[-10:]) < 0.1 * np.mean(losses[:10])


def test_checkpoint_resume_is_bitwise(M, tmp_path):
    import torch
    (feat, traj, x, target), dev = _data(13, nf=6, B=512)
    a = M.MLP(6, 3, seed=21)
    for _ in range(3):
        a.train_step(*dev, lr=1e-3)
    a.save(tmp_path / "ck.npz")
    for _ in range(4):
        a.train_step(*dev, lr=1e-3)
    b = M.MLP(6, 3, seed=99)
    b.load(tmp_path / "ck.npz")
    for _ in range(4):
        b.train_step(*dev, lr=1e-3)
    assert np.array_equal(a.get_params(), b.get_params())
    assert a.get_adam()[2] == b.get_adam()[2] == 7


@pytest.mark.parametrize("B,n_traj", [(300, 3), (1000, 5), (65536, 64)])
def test_gradients_at_training_sizes_are_reproducible(M, B, n_traj):
    """The gradient at the training batch (65 536 points: 64 split-K slices of the weight
    gradients placed by XCD, the final reductions over 1024 output-layer and 1024 bias
    partial rows) and at ragged batches that pad to 384 rows (one slice) and 1024 rows
    (8 slices): against the CPU reference with BF16 rounding, and bit for bit the same
    on a second call (every reduction has a fixed order)."""
    import torch
    net = M.MLP(38, 3, seed=11)
    (feat, traj, x, target), dev = _data(17 + B, nf=38, npnt=3, B=B, n_traj=n_traj)
    g1, l1 = net.grad(*dev)
    g2, l2 = net.grad(*dev)
    assert torch.equal(g1, g2) and torch.equal(l1, l2), "gradient not reproducible"
    g = g1.cpu().numpy().astype(np.float64)
    theta = net.get_params().astype(np.float64)
    loss, gr = ref.loss_and_grad(theta, feat, traj, x, target, bf=True)
    assert abs(l1.item() / B - loss) <= 1e-4 * loss
    for name, o, n in _blocks(41):
        a, b = g[o:o + n], gr[o:o + n]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("B %d grad %s: rel err %.2e" % (B, name, err), flush=True)
        assert err < 5e-3, (B, name)
