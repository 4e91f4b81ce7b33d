"""The CPU reference MLP against finite differences, the BF16 definition and Adam's formula."""
import numpy as np

from oracle import mlp


def _case(seed=0, nf=5, npnt=3, B=24, n_traj=3):
    rng = np.random.default_rng(seed)
    n_in = nf + npnt
    _, total = mlp.layout(n_in)
    theta = rng.normal(0, 0.08, total)
    feat = rng.normal(0, 1, (n_traj, nf))
    traj = rng.integers(0, n_traj, B)
    x = rng.normal(0, 1, (B, npnt))
    target = rng.normal(0, 1, B)
    return theta, feat, traj, x, target


def test_gradient_matches_finite_differences():
    theta, feat, traj, x, target = _case()
    loss, g = mlp.loss_and_grad(theta, feat, traj, x, target)
    lay, _ = mlp.layout(8)
    rng = np.random.default_rng(1)
    idx = []
    for name, (o, shape) in lay.items():          # a few entries of every block
        n = int(np.prod(shape))
        idx += list(o + rng.choice(n, size=min(n, 6), replace=False))
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, feat, traj, x, target)[0] -
              mlp.loss_and_grad(tm, feat, traj, x, target)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_silu_derivative():
    z = np.linspace(-8, 8, 41)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.dsilu(z), fd, rtol=1e-7, atol=1e-10)
    assert mlp.silu(0.0) == 0.0 and abs(mlp.silu(50.0) - 50.0) < 1e-12


def test_bf16_rounding():
    # exact values, halfway cases round to even
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -2.5, 3.1415926])
    r = mlp.bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2.0 ** -7 or r[1] == 1.0          # representable? 1 + 2^-8 is a tie
    assert r[1] == 1.0                                       # tie -> even mantissa (1.0)
    assert r[2] == 1.0 + 2.0 ** -6                           # tie -> even (...10)
    assert r[3] == 1.0                                       # below half an ulp
    assert r[4] == -2.5
    assert abs(r[5] - 3.140625) < 1e-12


def test_adam_first_step_is_sign_step():
    g = np.array([0.3, -2.0, 1e-3])
    t, m1, m2 = mlp.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=1e-12)
    assert np.allclose(t, -0.01 * np.sign(g), rtol=1e-9)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_bf16_mode_close_to_fp64():
    theta, feat, traj, x, target = _case(seed=3)
    l64, g64 = mlp.loss_and_grad(theta, feat, traj, x, target)
    lbf, gbf = mlp.loss_and_grad(theta, feat, traj, x, target, bf=True)
    assert abs(lbf - l64) / l64 < 2e-2
    assert np.linalg.norm(gbf - g64) / np.linalg.norm(g64) < 5e-2
