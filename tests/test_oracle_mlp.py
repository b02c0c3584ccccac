"""Pins of the FP64 surrogate oracle against mathematics outside it.

The backward pass is pinned by central finite differences of the loss, the
forward pass by hand evaluations (math.exp) for special weights, Adam by its
closed-form first step, and the peak refinement by exact parabolas.
"""

import math

import numpy as np
import pytest

import oracle.mlp as m
from paper_2609_20536_amd import workloads as W


def _theta(seed=1):
    rng = np.random.default_rng(seed)
    th = np.array(W.mlp_init_params(), dtype=np.float64)
    return th + 0.05 * rng.standard_normal(th.size)


def _data(n=7, seed=2):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 2)), rng.standard_normal((n, 4))


def test_silu_closed_forms():
    assert m.silu(np.array(0.0)) == 0.0
    assert abs(m.silu(np.array(1.0)) - 1.0 / (1.0 + math.exp(-1.0))) < 1e-16
    assert abs(m.silu(np.array(-2.0)) - (-2.0 / (1.0 + math.exp(2.0)))) < 1e-16
    assert abs(m.dsilu(np.array(0.0)) - 0.5) < 1e-16
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (m.silu(z + h) - m.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - m.dsilu(z))) < 1e-9


def test_parameter_count_and_layout():
    assert m.NPARAM == W.MLP_NPARAM == 17412
    th = np.arange(m.NPARAM, dtype=float)
    W1, b1, W2, b2, W3, b3 = m.unpack(th)
    assert W1.shape == (128, 2) and W1[0, 1] == 1.0 and b1[0] == 256.0
    assert W2[0, 0] == 384.0 and b2[0] == 384.0 + 16384
    assert W3.shape == (4, 128) and b3[-1] == m.NPARAM - 1


def test_forward_hand_evaluation():
    """Only two hidden units carry signal; y_c = (c+1) s(s(1)) - s(s(-2)) + c."""
    W1 = np.zeros((128, 2)); W1[0, 0] = 1.0; W1[1, 1] = 1.0
    W2 = np.zeros((128, 128)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    W3 = np.zeros((4, 128))
    for c in range(4):
        W3[c, 0] = c + 1.0
        W3[c, 1] = -1.0
    th = m.pack([W1, np.zeros(128), W2, np.zeros(128), W3, np.arange(4.0)])
    s = lambda x: x / (1.0 + math.exp(-x))  # noqa: E731
    y, _ = m.forward(th, np.array([[1.0, -2.0]]))
    for c in range(4):
        assert abs(y[0, c] - ((c + 1) * s(s(1.0)) - s(s(-2.0)) + c)) < 1e-15


def test_forward_constant_when_first_layers_vanish():
    th = _theta()
    W1, b1, W2, b2, W3, b3 = [p.copy() for p in m.unpack(th)]
    W1[:] = 0.0
    W2[:] = 0.0
    th0 = m.pack([W1, b1, W2, b2, W3, b3])
    X, _ = _data(5)
    y, _ = m.forward(th0, X)
    expect = W3 @ (b2 / (1.0 + np.exp(-b2))) + b3
    assert np.max(np.abs(y - expect[None, :])) < 1e-14


def _fd_check(grad_fn, seed=3, nsub=300):
    th = _theta(seed)
    X, T = _data(9, seed)
    _, g = grad_fn(th, X, T)
    rng = np.random.default_rng(seed)
    idx = np.concatenate([rng.choice(m.NPARAM, nsub, replace=False),
                          np.arange(m.NPARAM - 516, m.NPARAM)])   # all of W3, b3
    h = 1e-6
    fd = np.empty(idx.size)
    for a, i in enumerate(idx):
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd[a] = (m.loss(tp, X, T) - m.loss(tm, X, T)) / (2 * h)
    return np.linalg.norm(fd - g[idx]) / np.linalg.norm(fd)


def test_backward_matches_central_differences():
    assert _fd_check(m.grad) < 1e-7


def test_backward_mutations_fail_the_difference_check(monkeypatch):
    orig = m.dsilu
    monkeypatch.setattr(m, "dsilu", lambda z: m.sigmoid(z))   # dropped term
    assert _fd_check(m.grad) > 1e-3
    monkeypatch.setattr(m, "dsilu", orig)

    def grad_w2_transposed(th, X, T):
        lval, g = m.grad(th, X, T)
        parts = [p.copy() for p in m.unpack(g)]
        parts[2] = parts[2].T.copy()                           # transposed operand
        return lval, m.pack(parts)
    assert _fd_check(grad_w2_transposed) > 1e-3


def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    opt = m.Adam(50, lr=1e-3)
    th1 = opt.step(th, g)
    expect = th - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(th1 - expect)) < 1e-18 + 1e-15 * np.max(np.abs(th))
    # |step| = lr |g| / (|g| + eps): lr up to the relative eps / |g|
    assert np.all(np.abs(np.abs(th1 - th) - 1e-3) <= 1e-3 * 1e-8 / np.abs(g) + 1e-15)


def test_adam_minimises_a_quadratic():
    a = np.array([1.0, 10.0, 0.1])
    th = np.array([1.0, -1.0, 2.0])
    opt = m.Adam(3, lr=1e-2)
    for _ in range(4000):
        th = opt.step(th, a * th)
    assert np.max(np.abs(th)) < 1e-2


def test_training_decreases_loss_and_reports_initial_loss():
    th0 = np.array(W.mlp_init_params(), dtype=np.float64)
    rng = np.random.default_rng(5)
    X = rng.uniform(-1.5, 1.5, (40, 2))
    T = np.stack([np.sin(X[:, 0]), X[:, 1] ** 2, X[:, 0] * X[:, 1], np.cos(X[:, 1])], axis=1)
    th, losses = m.train(th0, X, T, 300, lr=3e-3)
    assert losses[0] == m.loss(th0, X, T)
    assert losses[-1] < 0.2 * losses[0]


def test_standardisation_round_trip():
    rng = np.random.default_rng(6)
    X = rng.uniform([0.5, 0.0], [1.5, 1.0], (30, 2))
    Y = np.stack([-rng.uniform(1, 2, 30), rng.uniform(0.1, 2, 30),
                  np.exp(rng.standard_normal(30)), np.exp(rng.standard_normal(30))], axis=1)
    Yt = m.transform_targets(Y, 0b1100)
    assert np.allclose(np.exp(Yt[:, 2:]), Y[:, 2:], rtol=1e-15)
    xm, xs, ym, ys = m.scaling(X, Yt)
    assert np.allclose(((X - xm) / xs).mean(axis=0), 0.0, atol=1e-15)
    assert np.allclose(((Yt - ym) / ys).std(axis=0), 1.0, atol=1e-14)
    # a network whose output is zero predicts the target means (log columns: exp)
    th = np.zeros(m.NPARAM)
    y = m.predict(th, X, (xm, xs, ym, ys), 0b1100)
    assert np.allclose(y[:, :2], ym[None, :2], rtol=1e-15)
    assert np.allclose(y[:, 2:], np.exp(ym[None, 2:]), rtol=1e-15)


@pytest.mark.parametrize("c", [10.0, 10.25, 9.6, 0.0, 31.0])
def test_column_peak_recovers_parabola_vertex(c):
    i = np.arange(32, dtype=float)
    idx, off = m.column_peak(-(i - c) ** 2 + 3.0)
    assert idx == int(np.clip(np.round(c), 0, 31))
    if 0 < idx < 31:
        assert abs(idx + off - c) < 1e-13
    else:
        assert off == 0.0


def test_lattice_corners():
    L = m.lattice(5, 3, 0.5, 1.5, 0.0, 1.0)
    assert L.shape == (3, 5, 2)
    assert L[0, 0, 0] == 0.5 and L[0, -1, 0] == 1.5
    assert L[0, 0, 1] == 0.0 and L[-1, 0, 1] == 1.0


def test_init_is_xavier_uniform_and_seeded():
    p = np.array(W.mlp_init_params())
    W1, b1, W2, b2, W3, b3 = m.unpack(p)
    for Wl, (fo, fi) in zip((W1, W2, W3), W.MLP_LAYERS):
        a = math.sqrt(6.0 / (fo + fi))
        assert np.max(np.abs(Wl)) <= a and np.max(np.abs(Wl)) > 0.9 * a
    assert abs(W2.mean()) < 0.01 and abs(W2.std() - math.sqrt(6 / 256) / math.sqrt(3)) < 0.01
    assert not np.any(b1) and not np.any(b2) and not np.any(b3)
    assert np.array_equal(p, np.array(W.mlp_init_params()))
    assert not np.array_equal(p, np.array(W.mlp_init_params(seed=1)))
