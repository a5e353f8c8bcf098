"""Pins of the oracle's POD and warm-start network (FP64)."""
import math

import numpy as np

from oracle import learn


def test_gradient_matches_central_differences():
    K, H = 3, 5
    rng = np.random.default_rng(0)
    p = learn.glorot(K, H, 7) + 0.05 * rng.standard_normal(learn.layout(K, H)[0][-1])
    F = rng.standard_normal((6, 4))
    T = rng.standard_normal((6, 2 * K))
    _, g = learn.loss_grad(p, K, H, F, T)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p); e[i] = h
        fd[i] = (learn.loss_grad(p + e, K, H, F, T)[0] - learn.loss_grad(p - e, K, H, F, T)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * np.max(np.abs(g)) + 1e-10


def test_pod_eckart_young_and_orthonormality():
    rng = np.random.default_rng(1)
    S, N, K = 40, 90, 7
    A = (rng.standard_normal((S, 10)) + 1j * rng.standard_normal((S, 10))) @ \
        (rng.standard_normal((10, N)) + 1j * rng.standard_normal((10, N)))
    A += 1e-3 * (rng.standard_normal((S, N)) + 1j * rng.standard_normal((S, N)))
    U, s = learn.pod(A, K)
    assert np.max(np.abs(U @ U.conj().T - np.eye(K))) < 1e-12
    P = A - (A @ U.conj().T) @ U          # rows projected out of span(U)
    assert abs(np.linalg.norm(P) - math.sqrt(np.sum(s[K:] ** 2))) < 1e-10 * np.linalg.norm(A)


def test_glorot_bounds_and_determinism():
    K, H = 8, 32
    p = learn.glorot(K, H, 555)
    offs, O = learn.layout(K, H)
    W1 = p[offs[0]:offs[1]]
    lim = math.sqrt(6.0 / (4 + H))
    assert np.all(np.abs(W1) <= lim) and np.max(np.abs(W1)) > 0.9 * lim
    assert np.all(p[offs[1]:offs[2]] == 0)
    assert np.array_equal(p, learn.glorot(K, H, 555))
    assert not np.array_equal(p, learn.glorot(K, H, 556))


def test_shuffle_is_a_permutation():
    for S in (1, 7, 256, 1000):
        perm = learn.shuffle(S, 555, 3)
        assert sorted(perm) == list(range(S))
    assert not np.array_equal(learn.shuffle(100, 555, 0), learn.shuffle(100, 555, 1))


def test_training_fits_a_smooth_map():
    rng = np.random.default_rng(2)
    K, H = 2, 16
    d = rng.standard_normal((64, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    F = np.concatenate([d, np.where(rng.random((64, 1)) < 0.5, 1.0, -1.0)], axis=1)
    T = np.stack([d[:, 0] * F[:, 3], d[:, 1], np.sin(d[:, 2]), d[:, 0] * d[:, 1]], axis=1)
    p0 = learn.glorot(K, H, 5)
    l0 = learn.loss_grad(p0, K, H, F, T)[0]
    p = learn.train(p0, K, H, F, T, epochs=150, batch=16, lr_max=1e-2, lr_min=1e-4, seed=5)
    assert learn.loss_grad(p, K, H, F, T)[0] < 0.05 * l0


def test_linear_polarisation_gradient_and_combination():
    """Linear-in-polarisation model: the gradient equals central differences, and
    the combination is linear in e (a theta/phi pair at one direction reproduces
    any other real polarisation in their span)."""
    K, H = 3, 6
    rng = np.random.default_rng(7)
    p = learn.glorot(K, H, 123, pol_model=1) + 0.05 * rng.standard_normal(learn.layout(K, H, 1)[0][-1])
    D = rng.standard_normal((5, 3)); D /= np.linalg.norm(D, axis=1, keepdims=True)
    E = rng.standard_normal((5, 3)); E -= (E * D).sum(1, keepdims=True) * D; E /= np.linalg.norm(E, axis=1, keepdims=True)
    T = rng.standard_normal((5, 2 * K))
    loss, g = learn.loss_grad_pol(p, K, H, D, E, T)
    h = 1e-6
    idx = rng.choice(len(p), 40, replace=False)
    for i in idx:
        q = p.copy(); q[i] += h; lp, _ = learn.loss_grad_pol(q, K, H, D, E, T)
        q[i] -= 2 * h; lm, _ = learn.loss_grad_pol(q, K, H, D, E, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    # linearity in e: y(a e1 + b e2) = a y(e1) + b y(e2)
    F = np.concatenate([D, np.zeros((5, 1))], axis=1)
    raw, _ = learn.forward(p, K, H, F, 1)
    e1, e2 = E, np.cross(D, E)
    a, b = 0.6, -0.8
    assert np.allclose(learn.combine(raw, a * e1 + b * e2, K), a * learn.combine(raw, e1, K) + b * learn.combine(raw, e2, K),
                       atol=1e-14)
    # the output layer has 6K rows; the first layers are those of the base model
    assert learn.layout(K, H, 1)[1] == 6 * K
    assert np.array_equal(learn.glorot(K, H, 9, 1)[:learn.layout(K, H)[0][4]], learn.glorot(K, H, 9)[:learn.layout(K, H)[0][4]])
