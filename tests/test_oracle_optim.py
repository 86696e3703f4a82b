"""Pins of the training-step oracle (L1 loss, activation chain, Adam) against closed forms and
finite differences."""
import numpy as np

from oracle import optim as OP


def _params(n, rng):
    return dict(means=rng.standard_normal((3, n)), scales=rng.uniform(-5, -1, (3, n)),
                quats=rng.standard_normal((4, n)), opacities=rng.standard_normal(n),
                sh=rng.standard_normal((48, n)))


def test_l1_worked_example_and_gradient():
    rgb = np.array([0.5, 0.25, 1.0, 0.0])
    tgt = np.array([0.25, 0.25, 0.0, 0.5])
    loss, g = OP.l1_loss(rgb, tgt)
    assert loss == (0.25 + 0.0 + 1.0 + 0.5) / 4
    np.testing.assert_array_equal(g, [0.25, 0.0, 0.25, -0.25])
    # central differences away from the kinks
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(50), rng.standard_normal(50)
    _, g = OP.l1_loss(a, b)
    for i in range(0, 50, 7):
        h = 1e-7
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = (OP.l1_loss(ap, b)[0] - OP.l1_loss(am, b)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7


def test_activation_chain_by_finite_differences():
    """d/draw of a linear functional of the activated parameters equals the chained gradient."""
    rng = np.random.default_rng(2)
    raw = _params(20, rng)
    w = {k: rng.standard_normal(a.shape) for k, a in OP.activate(raw).items()}
    f = lambda r: sum(float((OP.activate(r)[k] * w[k]).sum()) for k in w)
    g = OP.raw_gradients(raw, w)
    for name in ("scales", "opacities"):
        for idx in [(0, 3), (2, 7)] if name == "scales" else [(3,), (11,)]:
            h = 1e-6
            rp = {k: a.copy() for k, a in raw.items()}
            rm = {k: a.copy() for k, a in raw.items()}
            rp[name][idx] += h
            rm[name][idx] -= h
            fd = (f(rp) - f(rm)) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_moves_by_lr_times_sign():
    """With zero moments, the bias-corrected first step is lr * g / (|g| + eps): -lr sign(g)."""
    rng = np.random.default_rng(3)
    raw = _params(10, rng)
    grads = {k: rng.standard_normal(a.shape) for k, a in OP.activate(raw).items()}
    zeros = {k: np.zeros_like(a) for k, a in raw.items()}
    lr = [1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 6e-3]
    p, m, v = OP.adam_step(raw, grads, zeros, zeros, 0, lr)
    g = OP.raw_gradients(raw, grads)
    np.testing.assert_allclose(p["means"] - raw["means"], -lr[0] * np.sign(g["means"]), rtol=1e-9)
    np.testing.assert_allclose(p["opacities"] - raw["opacities"], -lr[3] * np.sign(g["opacities"]), rtol=1e-9)
    np.testing.assert_allclose(p["sh"][:3] - raw["sh"][:3], -lr[4] * np.sign(g["sh"][:3]), rtol=1e-9)
    np.testing.assert_allclose(p["sh"][3:] - raw["sh"][3:], -lr[5] * np.sign(g["sh"][3:]), rtol=1e-9)


def test_adam_constant_gradient_keeps_unit_steps():
    """A constant gradient keeps the bias-corrected moments at g and g^2, so every step moves
    every parameter by the same -lr sign(g) (t = 1..20)."""
    rng = np.random.default_rng(4)
    raw = dict(means=rng.standard_normal((3, 5)), scales=np.zeros((3, 5)), quats=rng.standard_normal((4, 5)),
               opacities=np.zeros(5), sh=rng.standard_normal((3, 5)))
    gm = rng.standard_normal((3, 5))
    grads = dict(means=gm, scales=np.zeros((3, 5)), quats=np.zeros((4, 5)), opacities=np.zeros(5),
                 sh=np.zeros((3, 5)))
    m = {k: np.zeros_like(a) for k, a in raw.items()}
    v = {k: np.zeros_like(a) for k, a in raw.items()}
    p = raw
    lr = [1e-2, 0, 0, 0, 0, 0]
    for t in range(20):
        p, m, v = OP.adam_step(p, grads, m, v, t, lr)
    np.testing.assert_allclose(p["means"] - raw["means"], -20 * lr[0] * np.sign(gm), rtol=1e-9)
