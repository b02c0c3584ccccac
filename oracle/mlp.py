"""FP64 CPU reference of the learned surrogate (test infrastructure only).

Only tests/, the package smoke check and the benchmark's CPU baseline may
import this module; the product path never does.

The surrogate maps a parameter point (beta, Delta) to four thermodynamic
quantities (f, C_v, chi, chi_n) of the gXY model, the observables of
Ch. 3 (free energy, specific heat and the two susceptibilities). It is a
multilayer perceptron 2 -> 128 -> 128 -> 4 with SiLU after both hidden
layers and a linear output, trained by Adam on the mean squared error over
standardised inputs and standardised targets (chi and chi_n enter through
their logarithms). The thesis fixes none of this (it only motivates cheaper
scans of the phase diagram); the choices are stated here and followed by
the GPU path.

Parameter vector (17 412 entries): W1[128][2], b1[128], W2[128][128],
b2[128], W3[4][128], b3[4], row-major; layer l maps a -> W_l a + b_l.

Every function is written from its definition, in FP64, with no blocking or
fusion:
* silu(z) = z sigma(z), sigma(z) = 1 / (1 + e^-z);
  silu'(z) = sigma(z) (1 + z (1 - sigma(z)));
* loss(theta) = (1 / 4n) sum_s sum_c (y_sc - t_sc)^2;
* backward: the chain rule through the three affine maps and two SiLUs;
* Adam (Kingma and Ba, 2015): with g the gradient at step t = 1, 2, ...,
  m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
against the backward pass; closed-form SiLU values; reductions of the
network for special weights; the first Adam step moving every parameter by
lr sign(g); a quadratic minimised by Adam; standardisation round trips.
"""

from __future__ import annotations

import numpy as np

SHAPES = ((128, 2), (128,), (128, 128), (128,), (4, 128), (4,))
NPARAM = 17412


def unpack(theta):
    """Views W1, b1, W2, b2, W3, b3 of the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, at = [], 0
    for shp in SHAPES:
        size = int(np.prod(shp))
        out.append(theta[at:at + size].reshape(shp))
        at += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """Network output y (n, 4) and the intermediates of the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = X @ W1.T + b1
    a1 = silu(h1)
    h2 = a1 @ W2.T + b2
    a2 = silu(h2)
    y = a2 @ W3.T + b3
    return y, (X, h1, a1, h2, a2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(theta, X, T):
    """Gradient of loss(theta) by the chain rule; returns (loss, g)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, h1, a1, h2, a2) = forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    dy = 2.0 * (y - T) / (4.0 * n)
    gW3 = dy.T @ a2
    gb3 = dy.sum(axis=0)
    dh2 = (dy @ W3) * dsilu(h2)
    gW2 = dh2.T @ a1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * dsilu(h1)
    gW1 = dh1.T @ X
    gb1 = dh1.sum(axis=0)
    return float(np.mean((y - T) ** 2)), pack([gW1, gb1, gW2, gb2, gW3, gb3])


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def train(theta, X, T, epochs, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Full-batch Adam; returns the final parameters and the loss before
    each update (losses[e] is the loss at the parameters of epoch e)."""
    theta = np.array(theta, dtype=np.float64)
    opt = Adam(theta.size, lr, b1, b2, eps)
    losses = np.empty(epochs)
    for e in range(epochs):
        losses[e], g = grad(theta, X, T)
        theta = opt.step(theta, g)
    return theta, losses


# ---------------------------------------------------------------------------
# Standardisation of inputs and targets
# ---------------------------------------------------------------------------

def transform_targets(Y, log_mask):
    """Targets in network units before standardisation: columns whose bit is
    set in log_mask enter through their natural logarithm."""
    Y = np.array(Y, dtype=np.float64)
    for c in range(Y.shape[1]):
        if (log_mask >> c) & 1:
            Y[:, c] = np.log(Y[:, c])
    return Y


def scaling(X, Yt):
    """Mean and (population) standard deviation per column."""
    X = np.asarray(X, dtype=np.float64)
    Yt = np.asarray(Yt, dtype=np.float64)
    return X.mean(axis=0), X.std(axis=0), Yt.mean(axis=0), Yt.std(axis=0)


def predict(theta, X, sc, log_mask):
    """Predictions in physical units from raw (beta, Delta)."""
    xm, xs, ym, ys = sc
    y, _ = forward(theta, (np.asarray(X, dtype=np.float64) - xm) / xs)
    y = y * ys + ym
    for c in range(y.shape[1]):
        if (log_mask >> c) & 1:
            y[:, c] = np.exp(y[:, c])
    return y


# ---------------------------------------------------------------------------
# Proposals: one point at the predicted C_v maximum and one at the predicted
# chi maximum along beta, for every Delta of a lattice.
# ---------------------------------------------------------------------------

def lattice(nbeta, ndelta, beta_lo, beta_hi, delta_lo, delta_hi):
    """Candidate lattice: beta_i = lo + i (hi - lo)/(nbeta - 1), likewise Delta;
    row j of the returned (ndelta, nbeta, 2) array holds Delta_j."""
    b = beta_lo + (beta_hi - beta_lo) * np.arange(nbeta) / (nbeta - 1)
    d = delta_lo + (delta_hi - delta_lo) * np.arange(ndelta) / (ndelta - 1)
    out = np.empty((ndelta, nbeta, 2))
    out[:, :, 0] = b[None, :]
    out[:, :, 1] = d[:, None]
    return out


def column_peak(values):
    """Index of the largest value of a column (first one on ties) and the
    vertex offset in [-1/2, 1/2] of the parabola through it and its two
    neighbours (0 at the ends or when the three points are collinear)."""
    i = int(np.argmax(values))
    if i == 0 or i == len(values) - 1:
        return i, 0.0
    ym, y0, yp = values[i - 1], values[i], values[i + 1]
    den = ym - 2.0 * y0 + yp
    if den >= 0.0:
        return i, 0.0
    off = 0.5 * (ym - yp) / den
    return i, float(min(0.5, max(-0.5, off)))
