"""Pins of the flow oracle: exact gradients, invertibility, unit mean weight,
unbiasedness on a closed form, and that training lowers the variance."""
import math

import numpy as np
import pytest
import torch

from oracle import flow, points


def random_params(n, seed, scale=0.5):
    P = flow.init_params(n, seed, 0)
    g = torch.Generator().manual_seed(seed)
    for d in P:
        for k in d:
            d[k] = d[k] + scale * torch.randn(d[k].shape, generator=g, dtype=torch.float64) / math.sqrt(d[k].numel() ** 0.5)
    return P


def lattice(n, m, seed=3):
    z = points.cbc_vector(m, n)
    sh = points.shift_table(seed, 0, 1, n, m)[0]
    return points.lattice_u(z, m, sh, 0, 1 << m)


def test_initial_flow_is_identity():
    P = flow.init_params(3, 7, 0)
    u = lattice(3, 8)
    x, lq = flow.sample(P, u)
    assert np.allclose(x, u, atol=1e-15) and np.allclose(lq, 0.0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_inverse_then_forward_is_identity(n):
    P = random_params(n, 11)
    u = lattice(n, 9)
    x, lq = flow.sample(P, u)
    y, lq2 = flow.forward(P, torch.tensor(x))
    assert np.allclose(y.numpy(), u, atol=1e-12)
    assert np.allclose(lq2.numpy(), lq, atol=1e-11)
    assert np.all((x >= 0) & (x <= 1))


def test_mean_weight_is_one_and_unbiased():
    P = random_params(2, 5)
    R, m = 8, 12
    z = points.cbc_vector(m, 2)
    est_w, est_f = [], []
    for r in range(R):
        u = points.lattice_u(z, m, points.shift_table(9, 0, R, 2, m)[r], 0, 1 << m)
        x, lq = flow.sample(P, u)
        w = np.exp(-lq)
        est_w.append(w.mean())
        est_f.append(np.mean(w * np.exp(x[:, 0]) * x[:, 1] ** 2))
    assert abs(np.mean(est_w) - 1.0) < 5 * np.std(est_w) / math.sqrt(R) + 1e-12
    exact = (math.e - 1) / 3
    assert abs(np.mean(est_f) - exact) < 5 * np.std(est_f) / math.sqrt(R) + 1e-12


def test_gradient_matches_finite_differences():
    flow.EMULATE_BF16 = False
    try:
        P = random_params(3, 21)
        rng = np.random.default_rng(4)
        x = rng.uniform(0.02, 0.98, size=(64, 3))
        c = rng.uniform(0.1, 1.0, size=64)
        _, G = flow.loss_and_grad(P, x, c)
        h = 1e-6
        checked = 0
        for l in range(flow.L_LAYERS):
            for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
                flat = P[l][name].view(-1)
                for i in rng.choice(flat.numel(), size=3, replace=False):
                    old = float(flat[i])
                    flat[i] = old + h
                    lp, _ = flow.loss_and_grad(P, x, c)
                    flat[i] = old - h
                    lm, _ = flow.loss_and_grad(P, x, c)
                    flat[i] = old
                    fd = (lp - lm) / (2 * h)
                    g = float(G[l][name].view(-1)[i])
                    assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (l, name, i, fd, g)
                    checked += 1
        assert checked == flow.L_LAYERS * 6 * 3
    finally:
        flow.EMULATE_BF16 = True


def test_training_lowers_variance():
    """A peaked 2-D integrand: the trained map's variance of f/q falls well below the identity's."""
    def f(x):
        return np.exp(-((x[:, 0] - 0.2) ** 2 + (x[:, 1] - 0.7) ** 2) / 0.01)
    P = flow.init_params(2, 3, 0)
    st = flow.adam_init(P)
    rng_seed = 0
    m = 10
    z = points.cbc_vector(m, 2)

    def var_of(P):
        u = points.lattice_u(z, m, points.shift_table(99, 0, 1, 2, m)[0], 0, 1 << m)
        x, lq = flow.sample(P, u)
        v = f(x) * np.exp(-lq)
        return v.var()
    v0 = var_of(P)
    for step in range(60):
        u = points.lattice_u(z, m, points.shift_table(rng_seed, 0, step + 1, 2, m)[step], 0, 1 << m)
        x, lq = flow.sample(P, u)
        c = flow.importance_weights(f(x)[None, :], lq)
        _, G = flow.loss_and_grad(P, x, c)
        flow.adam_step(P, G, st, lr=3e-3)
    v1 = var_of(P)
    assert v1 < 0.3 * v0, (v0, v1)


def test_bin_probabilities_stay_positive():
    """Extreme weights push logits hundreds apart; the logit range bound keeps every
    bin probability positive (>= e^-60 / 32) and the map invertible."""
    n = 3
    P = random_params(n, 5, scale=200.0)
    u = lattice(n, 9)
    h = torch.tensor(u, dtype=torch.float64)
    A, B = flow.masks(n)[0]
    Q = flow._probs(P[0], h[:, A], len(B))
    assert float(Q.min()) >= math.exp(-60.0) / flow.NBINS * 0.999
    logits_gap = (torch.amax(Q, dim=2) / torch.amin(Q, dim=2)).max()
    assert float(logits_gap) > 1e20          # the bound is active here
    x, lq = flow.sample(P, u)
    y, lq2 = flow.forward(P, torch.tensor(x))
    assert np.all(np.isfinite(lq))
    ok = np.abs(y.numpy() - u).max(axis=1) < 1e-6
    assert ok.mean() > 0.99
