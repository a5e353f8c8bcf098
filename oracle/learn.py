"""POD basis and the warm-start network (oracle, FP64).

Not in the paper: the learned warm start is a production form beside the plain
solve.  Definitions written out plainly:

  * POD by the method of snapshots: the leading K left singular vectors of the
    snapshot matrix A = [x_1 ... x_S] (numpy SVD); Eckart-Young: the best rank-K
    approximation error is sqrt(sum_{i>K} sigma_i^2).
  * Network: y = W3 tanh(W2 tanh(W1 f + b1) + b2) + b3 with f = (d_x, d_y, d_z, s);
    loss = mean over batch and outputs of (y - t)^2; gradients by backpropagation
    (chain rule, d tanh = 1 - tanh^2).
  * Glorot-uniform initial weights: w = (2u - 1) sqrt(6/(fan_in + fan_out)) with u
    the SplitMix64 stream mapped to [0, 1) by (z >> 11) 2^-53, drawn for W1, W2,
    W3 in order, row-major (out, in); biases 0.
  * Per-epoch Fisher-Yates shuffle with SplitMix64(seed + 1 + epoch), uniform
    index on [0, i] as the high 64 bits of z (i + 1).
  * Adam (Kingma & Ba 2015) with beta = (0.9, 0.999), eps = 1e-8 and a cosine
    learning rate from lr_max to lr_min over all steps.
  * Linear-in-polarisation model (pol_model 1): a solution is linear in the
    polarisation vector e, so the network takes f = (d_x, d_y, d_z, 0) and gives
    three coefficient sets f_x, f_y, f_z (6K outputs); the coefficients for e
    are y = e_x f_x + e_y f_y + e_z f_z and the loss is the mean squared error of
    y against the 2K targets.
"""
from __future__ import annotations

import math

import numpy as np

from .sampling import SplitMix64


def pod(X: np.ndarray, K: int):
    """X: S x N snapshots (rows).  Returns U (K x N, orthonormal rows) and all singular values."""
    U, s, _ = np.linalg.svd(X.T, full_matrices=False)
    return U[:, :K].T.copy(), s


def layout(K: int, H: int, pol_model: int = 0):
    O = (6 if pol_model == 1 else 2) * K
    sizes = [H * 4, H, H * H, H, O * H, O]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return offs, O


def unpack(p: np.ndarray, K: int, H: int, pol_model: int = 0):
    offs, O = layout(K, H, pol_model)
    W1 = p[offs[0]:offs[1]].reshape(H, 4); b1 = p[offs[1]:offs[2]]
    W2 = p[offs[2]:offs[3]].reshape(H, H); b2 = p[offs[3]:offs[4]]
    W3 = p[offs[4]:offs[5]].reshape(O, H); b3 = p[offs[5]:offs[6]]
    return W1, b1, W2, b2, W3, b3


def glorot(K: int, H: int, seed: int, pol_model: int = 0) -> np.ndarray:
    offs, O = layout(K, H, pol_model)
    p = np.zeros(offs[-1])
    g = SplitMix64(seed)

    def fill(off, fan_out, fan_in):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        for i in range(fan_out * fan_in):
            u = (g.next() >> 11) * (1.0 / 9007199254740992.0)
            p[off + i] = (2.0 * u - 1.0) * lim
    fill(offs[0], H, 4)
    fill(offs[2], H, H)
    fill(offs[4], O, H)
    return p


def forward(p, K, H, F, pol_model: int = 0):
    W1, b1, W2, b2, W3, b3 = unpack(p, K, H, pol_model)
    a1 = np.tanh(F @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    return a2 @ W3.T + b3, (a1, a2)


def _backprop(p, K, H, F, dy, a1, a2, pol_model=0):
    """Gradient of the loss with respect to p from dL/d(outputs) = dy."""
    W1, b1, W2, b2, W3, b3 = unpack(p, K, H, pol_model)
    gW3 = dy.T @ a2; gb3 = dy.sum(0)
    da2 = (dy @ W3) * (1.0 - a2 * a2)
    gW2 = da2.T @ a1; gb2 = da2.sum(0)
    da1 = (da2 @ W2) * (1.0 - a1 * a1)
    gW1 = da1.T @ F; gb1 = da1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def loss_grad(p, K, H, F, T):
    """Mean squared error and its gradient (same layout as p)."""
    y, (a1, a2) = forward(p, K, H, F)
    B, O = y.shape
    d = y - T
    loss = float(np.mean(d * d))
    return loss, _backprop(p, K, H, F, 2.0 * d / (B * O), a1, a2)


def combine(raw, E, K):
    """Coefficients of the linear-in-polarisation model: sum_c E[:, c] f_c."""
    return sum(E[:, c:c + 1] * raw[:, 2 * K * c:2 * K * (c + 1)] for c in range(3))


def loss_grad_pol(p, K, H, D, E, T):
    """Linear-in-polarisation model: inputs D (directions, B x 3), polarisations E
    (B x 3), targets T (B x 2K); mean squared error of the combination and its
    gradient."""
    F = np.concatenate([D, np.zeros((D.shape[0], 1))], axis=1)
    raw, (a1, a2) = forward(p, K, H, F, 1)
    y = combine(raw, E, K)
    B = y.shape[0]
    d = y - T
    loss = float(np.mean(d * d))
    dyc = 2.0 * d / (B * 2 * K)
    draw = np.concatenate([E[:, c:c + 1] * dyc for c in range(3)], axis=1)
    return loss, _backprop(p, K, H, F, draw, a1, a2, 1)


def shuffle(S: int, seed: int, epoch: int) -> np.ndarray:
    perm = list(range(S))
    g = SplitMix64(seed + 1 + epoch)
    for i in range(S - 1, 0, -1):
        j = (g.next() * (i + 1)) >> 64
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(perm)


def cosine_lr(step: int, total: int, lr_max: float, lr_min: float) -> float:
    """Learning rate of step 1..total: lr_max at the first step, lr_min at the last,
    following half a cosine period in between."""
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * (step - 1) / max(1, total - 1)))


def adam_update(p, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1): moment estimates, their bias
    correction by 1 - beta^step, and the update.  Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def train(p0, K, H, F, T, epochs, batch, lr_max, lr_min, seed, D=None, E=None):
    """Adam on mini-batches in the shuffled order; returns the final parameters.
    With D and E (directions and polarisations) the linear-in-polarisation model
    is trained (loss_grad_pol; F is then unused), else the base model on F."""
    p = p0.astype(np.float64).copy()
    m = np.zeros_like(p); v = np.zeros_like(p)
    S = (F if D is None else D).shape[0]
    nb = (S + batch - 1) // batch
    total = epochs * nb
    step = 0
    for ep in range(epochs):
        perm = shuffle(S, seed, ep)
        for bi in range(nb):
            idx = perm[bi * batch:(bi + 1) * batch]
            if D is None:
                _, g = loss_grad(p, K, H, F[idx], T[idx])
            else:
                _, g = loss_grad_pol(p, K, H, D[idx], E[idx], T[idx])
            step += 1
            p, m, v = adam_update(p, m, v, g, step, cosine_lr(step, total, lr_max, lr_min))
    return p
