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


def test_cosine_schedule_values():
    """lr_max at the first step, lr_min at the last, their mean half-way (the
    cosine's zero), and lr_max for a single step."""
    assert learn.cosine_lr(1, 5, 1e-3, 1e-5) == 1e-3
    assert abs(learn.cosine_lr(5, 5, 1e-3, 1e-5) - 1e-5) < 1e-20
    assert abs(learn.cosine_lr(3, 5, 1e-3, 1e-5) - 5.05e-4) < 1e-18
    assert learn.cosine_lr(1, 1, 2e-3, 1e-5) == 2e-3
    lrs = [learn.cosine_lr(s, 50, 1e-3, 1e-5) for s in range(1, 51)]
    assert all(a > b for a, b in zip(lrs, lrs[1:]))


def test_adam_steps_worked_by_hand():
    """Two Adam steps with bias correction, values worked out by hand.

    Step 1: m = 0.1 g, v = 0.001 g^2, and the corrections 1 - 0.9 and 1 - 0.999
    give m^ = g, v^ = g^2, so every coordinate moves by lr against the sign of its
    gradient, whatever the gradient's size (up to eps / |g|).
    Step 2 with the gradient reversed: m = 0.09 g - 0.1 g = -0.01 g and
    m^ = -0.01 g / 0.19 = -g / 19; v = 0.000999 g^2 + 0.001 g^2 and v^ = g^2: the
    move is lr / 19 back.  With the same gradient again: m^ = 0.19 g / 0.19 = g, a
    full lr move.  A dropped bias correction (step 1 would move sqrt(1000)/10 lr)
    or swapped betas (step 2 would move 5e-4 lr back) fails these."""
    p0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([2.0, -3.0, 1e-3, -40.0])
    m = np.zeros(4); v = np.zeros(4)
    lr1, lr2 = 0.01, 0.02
    p1, m1, v1 = learn.adam_update(p0, m, v, g, 1, lr1)
    assert np.all(np.abs(p1 - (p0 - lr1 * np.sign(g))) <= lr1 * 1e-8 / np.abs(g) * 1.001)
    p2, _, _ = learn.adam_update(p1, m1, v1, -g, 2, lr2)
    assert np.all(np.abs(p2 - (p1 + lr2 * np.sign(g) / 19.0)) <= lr2 * 1e-8 / np.abs(g))
    p2s, _, _ = learn.adam_update(p1, m1, v1, g, 2, lr2)
    assert np.all(np.abs(p2s - (p1 - lr2 * np.sign(g))) <= lr2 * 1e-8 / np.abs(g) * 1.001)


def test_train_first_steps():
    """train() wiring: its first step is the sign step of Adam (above) at lr_max on
    the first mini-batch of epoch 0's shuffle; over 2 steps with lr_min = 0 the second
    step does not move (the schedule ends at lr_min), so training for 2 steps equals
    training for 1; and the linear-in-polarisation branch does the same with its own
    gradient."""
    K, H = 2, 5
    rng = np.random.default_rng(11)
    p0 = learn.glorot(K, H, 3)
    S, batch = 6, 3
    F = rng.standard_normal((S, 4))
    T = rng.standard_normal((S, 2 * K))
    perm = learn.shuffle(S, 9, 0)
    _, g = learn.loss_grad(p0, K, H, F[perm[:batch]], T[perm[:batch]])
    lr = 1e-3
    p1 = learn.train(p0, K, H, F, T, epochs=1, batch=S, lr_max=lr, lr_min=lr, seed=9)
    _, gall = learn.loss_grad(p0, K, H, F, T)      # one mini-batch of all S: order does not matter
    nz = np.abs(gall) > 1e-6
    assert np.all(np.abs(p1 - (p0 - lr * np.sign(gall)))[nz] <= lr * 1e-8 / np.abs(gall[nz]) * 1.01)
    # two mini-batches in one epoch, lr_min = 0: the first step (on perm[:3]) is the
    # only one that moves
    p2 = learn.train(p0, K, H, F, T, epochs=1, batch=batch, lr_max=lr, lr_min=0.0, seed=9)
    nzg = np.abs(g) > 1e-6
    assert np.all(np.abs(p2 - (p0 - lr * np.sign(g)))[nzg] <= lr * 1e-8 / np.abs(g[nzg]) * 1.01)
    assert np.array_equal(learn.train(p0, K, H, F, T, epochs=2, batch=S, lr_max=lr, lr_min=0.0, seed=9), p1)
    # linear-in-polarisation model
    D = rng.standard_normal((S, 3)); D /= np.linalg.norm(D, axis=1, keepdims=True)
    E = np.cross(D, [0.0, 0.0, 1.0]); E /= np.linalg.norm(E, axis=1, keepdims=True)
    pp = learn.glorot(K, H, 4, pol_model=1)
    _, gp = learn.loss_grad_pol(pp, K, H, D[perm], E[perm], T[perm])
    pp1 = learn.train(pp, K, H, None, T, epochs=1, batch=S, lr_max=lr, lr_min=lr, seed=9, D=D, E=E)
    nzp = np.abs(gp) > 1e-6
    assert np.all(np.abs(pp1 - (pp - lr * np.sign(gp)))[nzp] <= lr * 1e-8 / np.abs(gp[nzp]) * 1.01)
