"""Surrogate MLP on the GPU (C ABI) against the FP64 oracle (oracle/mlp.py).

Bars: gradients per parameter tensor within 1e-4 relative (l2) of the oracle
at the same FP32 parameters and data; short training runs follow the
oracle's loss curve to 1e-4 relative; FP32 inference within 1e-5 relative;
BF16 inference within the bound implied by bfloat16 rounding of the
128 x 128 layer's operands (2^-8 relative each, propagated with the
oracle's own intermediates); proposals valid against the oracle's
predictions (a maximum, up to the BF16 bound).
"""

import math

import numpy as np
import pytest

import oracle.mlp as om
from paper_2609_20536_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


@pytest.fixture()
def net(ctx):
    from paper_2609_20536_amd import hotrg as H
    s = H.Surrogate(ctx, seed=W.MLP_SEED)
    yield s
    s.close()


def _targets(X):
    """Smooth synthetic stand-ins for (f, C_v, chi, chi_n) over (beta, Delta)."""
    b, d = X[:, 0], X[:, 1]
    f = -np.log(2.0 + b * (1.0 + d)) / b
    cv = 1.0 + np.exp(-((b - (0.8 + 0.4 * d)) / 0.1) ** 2)
    chi = np.exp(2.0 * np.tanh(4.0 * (b - 0.9 - 0.3 * d)))
    chin = np.exp(1.0 + np.sin(3.0 * b) * d)
    return np.stack([f, cv, chi, chin], axis=1)


def _grid(n, seed=7):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.5, 1.5, n), rng.uniform(0.0, 1.0, n)], axis=1)


def _rel_by_tensor(a, b):
    out = []
    at = 0
    for shp in om.SHAPES:
        k = int(np.prod(shp))
        x, y = a[at:at + k], b[at:at + k]
        out.append(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))
        at += k
    return out


def test_init_matches_seeded_xavier(net):
    p = net.get_params()
    ref = np.array(W.mlp_init_params(W.MLP_SEED), dtype=np.float64).astype(np.float32)
    assert np.array_equal(p, ref)


@pytest.mark.parametrize("n", [1, 37, 300])
def test_gradient_matches_oracle(net, n):
    rng = np.random.default_rng(n)
    th = (np.array(W.mlp_init_params()) + 0.05 * rng.standard_normal(om.NPARAM)).astype(np.float32)
    net.set_params(th)
    X = rng.standard_normal((n, 2)).astype(np.float32)
    T = rng.standard_normal((n, 4)).astype(np.float32)
    loss, g = net.grad(X, T)
    lref, gref = om.grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(_rel_by_tensor(g.astype(np.float64), gref)) <= 1e-4


def test_training_follows_oracle(net):
    X = _grid(230)
    Y = _targets(X)
    th0 = net.get_params().astype(np.float64)
    hist = net.train(X, Y, epochs=60, lr=1e-3, log_targets=0b1100)
    Yt = om.transform_targets(Y, 0b1100)
    xm, xs, ym, ys = om.scaling(X, Yt)
    th_ref, lref = om.train(th0, (X - xm) / xs, (Yt - ym) / ys, 60, lr=1e-3)
    assert np.max(np.abs(hist - lref) / lref) <= 1e-4
    rel = _rel_by_tensor(net.get_params().astype(np.float64), th_ref)
    assert max(rel) <= 1e-3, rel
    gx, gxs, gy, gys, mask = net.scaling()
    assert mask == 0b1100
    assert np.allclose(gx, xm, rtol=1e-14) and np.allclose(gxs, xs, rtol=1e-14)
    assert np.allclose(gy, ym, rtol=1e-13) and np.allclose(gys, ys, rtol=1e-13)


def test_training_is_bitwise_reproducible(ctx):
    from paper_2609_20536_amd import hotrg as H
    X = _grid(100, seed=3)
    Y = _targets(X)
    outs = []
    for _ in range(2):
        s = H.Surrogate(ctx, seed=11)
        h = s.train(X, Y, epochs=40)
        outs.append((h, s.get_params()))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def _trained(net, epochs=400):
    X = _grid(230)
    Y = _targets(X)
    net.train(X, Y, epochs=epochs, lr=1e-3, log_targets=0b1100)
    th = net.get_params().astype(np.float64)
    gx, gxs, gy, gys, mask = net.scaling()
    return th, (gx, gxs, gy, gys), mask


def test_predict_fp32_and_bf16_against_oracle(net):
    th, sc, mask = _trained(net)
    Xq = _grid(1000, seed=9)          # 1000 = 15 full workgroups of 64 and a ragged tail
    ref = om.predict(th, Xq, sc, mask)
    y32 = net.predict(Xq, bf16=False)
    assert np.max(np.abs(y32 - ref) / (np.abs(ref) + 1e-3)) <= 1e-5
    y16 = net.predict(Xq, bf16=True)
    # bound: bfloat16 rounding (2^-8 relative) of a1 and W2 in the second layer
    W1, b1, W2, b2, W3, b3 = om.unpack(th)
    xm, xs, ym, ys = sc
    _, (X0, h1, a1, h2, a2) = om.forward(th, (Xq - xm) / xs)
    dh2 = 2.0 ** -7 * (np.abs(a1) @ np.abs(W2).T) + 1e-6
    dy = (dh2 * 1.1) @ np.abs(W3).T * ys[None, :]
    for c in range(4):
        err = np.abs(y16[:, c] - ref[:, c])
        lim = dy[:, c] * (np.abs(ref[:, c]) * 1.01 if (mask >> c) & 1 else 1.0)
        assert np.all(err <= lim + 1e-12), (c, float(np.max(err / (lim + 1e-12))))
    assert np.max(np.abs(y16 - y32)) > 0.0


def test_proposals_are_maxima_of_the_predictions(net):
    th, sc, mask = _trained(net)
    nb, nd = 64, 16
    out = net.propose(nbeta=nb, ndelta=nd, jitter=0.0, cv_col=1, chi_col=2)
    assert out.shape == (2 * nd, 2)
    L = om.lattice(nb, nd, 0.5, 1.5, 0.0, 1.0)
    pred = om.predict(th, L.reshape(-1, 2), sc, mask).reshape(nd, nb, 4)
    h = 1.0 / (nb - 1)
    for j in range(nd):
        for kind, col in ((0, 1), (1, 2)):
            b, d = out[2 * j + kind]
            assert d == L[j, 0, 1]
            assert 0.5 <= b <= 1.5
            i = int(round((b - 0.5) / h))
            colv = pred[j, :, col]
            span = colv.max() - colv.min()
            # the proposed point sits at a maximum of the oracle's curve, up to
            # the BF16 inference error and half a spacing of refinement
            near = colv[max(0, i - 1):i + 2].max()
            assert near >= colv.max() - 0.02 * span - 1e-12
            io, off = om.column_peak(colv)
            if abs(colv[io] - np.sort(colv)[-2]) > 0.05 * span:
                assert abs(b - (0.5 + h * (io + off))) <= 1.01 * h


def test_proposal_jitter_is_seeded_and_bounded(net):
    _trained(net, epochs=50)
    a = net.propose(nbeta=32, ndelta=8, jitter=0.0)
    b = net.propose(nbeta=32, ndelta=8, jitter=1.0, seed=5)
    c = net.propose(nbeta=32, ndelta=8, jitter=1.0, seed=5)
    assert np.array_equal(b, c)
    h = 1.0 / 31
    assert np.all(np.abs(b[:, 0] - a[:, 0]) <= 0.5 * h + 1e-12)
    assert np.any(b[:, 0] != a[:, 0])


def test_invalid_arguments(ctx, net):
    from paper_2609_20536_amd import hotrg as H
    with pytest.raises(H.GxyError):
        net.propose(nbeta=2)
    with pytest.raises(H.GxyError):
        net.propose(jitter=2.0)
    with pytest.raises(H.GxyError):
        net.train(np.zeros((0, 2)), np.zeros((0, 4)))
