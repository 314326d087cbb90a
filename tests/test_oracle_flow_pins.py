"""Pins of the flow oracle's optimiser and training objective against routes
that share none of its code: torch's own Adam, and the variance-optimal density
q = |f| / int |f| that the chi^2 objective must reach."""
import math

import numpy as np
import pytest
import torch

from oracle import flow, points


def test_adam_step_matches_torch_adam():
    """Five steps on gradients whose magnitudes span 1e-9 .. 1 (the small ones
    separate eps outside the square root from eps inside, the first step
    separates bias-corrected moments from raw ones) agree with torch.optim.Adam
    in fp64 up to the fp32 storage of the oracle's state."""
    gen = torch.Generator().manual_seed(0)
    P = flow.init_params(2, 5, 0)
    ref = [{k: v.clone().requires_grad_(True) for k, v in d.items()} for d in P]
    opt = torch.optim.Adam([t for d in ref for t in d.values()], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    st = flow.adam_init(P)
    for step in range(5):
        grads = []
        for d in P:
            g = {}
            for k, v in d.items():
                mag = 10.0 ** (-9 + 9 * torch.rand(v.shape, generator=gen, dtype=torch.float64))
                g[k] = mag * torch.sign(torch.randn(v.shape, generator=gen, dtype=torch.float64))
            grads.append(g)
        flow.adam_step(P, grads, st, lr=1e-2)
        opt.zero_grad()
        for d, g in zip(ref, grads):
            for k in d:
                d[k].grad = g[k].clone()
        opt.step()
        for d, r in zip(P, ref):
            for k in d:
                a, b = d[k], r[k].detach()
                # fp32 storage of parameters and moments: a few ulp of fp32 per step
                tol = 4 * (step + 1) * 2.0 ** -24 * (b.abs() + 1e-2)
                assert torch.all((a - b).abs() <= tol), (step, k, float((a - b).abs().max()))


def density_on_grid(P, xs):
    return np.exp(flow.log_q(P, torch.tensor(xs[:, None])).detach().numpy())


@pytest.mark.parametrize("kind", ["x2", "step"])
def test_training_reaches_the_chi2_optimal_density(kind):
    """One variable: minimising the variance of f/q over q makes q = |f| / int |f|
    (the chi^2-optimal density; a weight of |f|^2/q instead of |f|^2/q^2 would
    drive q to f^2 / int f^2, a weight of |f|^2 to a point mass).  Trained on
    the flow's own samples with the oracle's loss weights and gradient, the
    learned density approaches |f| / int |f| in L1 and in coarse-bin masses."""
    if kind == "x2":
        f = lambda x: x ** 2
        cdf = lambda x: x ** 3
    else:
        f = lambda x: np.where(x < 0.3, 4.0, 1.0)
        cdf = lambda x: np.where(x < 0.3, 4.0 * x, 1.2 + (x - 0.3)) / 1.9
    m = 9
    z = points.cbc_vector(m, 1)
    P = flow.init_params(1, 3, 0)
    st = flow.adam_init(P)
    for step in range(150):
        u = points.lattice_u(z, m, points.shift_table(17, 0, step + 1, 1, m)[step], 0, 1 << m)
        x, lq = flow.sample(P, u)
        c = flow.importance_weights(f(x[:, 0])[None, :], lq)
        _, G = flow.loss_and_grad(P, x, c)
        flow.adam_step(P, G, st, lr=2e-2)
    xs = (np.arange(4096) + 0.5) / 4096
    q = density_on_grid(P, xs)
    target = np.abs(f(xs)) / np.mean(np.abs(f(xs)))
    l1 = np.mean(np.abs(q - target))
    assert l1 < 0.1, l1
    # masses of 8 coarse bins
    e = np.linspace(0, 1, 9)
    mass_q = np.array([np.mean(q[(xs >= a) & (xs < b)]) * (b - a) for a, b in zip(e, e[1:])])
    mass_t = np.diff(cdf(e))
    assert np.max(np.abs(mass_q - mass_t)) < 0.02, (mass_q, mass_t)
    # and the alternative optimum f^2 / int f^2 is clearly further away
    alt = f(xs) ** 2 / np.mean(f(xs) ** 2)
    assert np.mean(np.abs(q - alt)) > 3 * l1


def test_importance_weights_order_handling():
    """Orders are normalised to their batch totals, weighted by the caller's
    order weights, and an all-zero order contributes nothing."""
    rng = np.random.default_rng(1)
    f = rng.normal(size=(3, 50)) + 1j * rng.normal(size=(3, 50))
    f[2] = 0.0
    lq = rng.normal(size=50) * 0.1
    c = flow.importance_weights(f, lq)
    q2 = np.exp(2 * lq)
    parts = [np.abs(f[k]) ** 2 / q2 / np.sum(np.abs(f[k]) ** 2 / q2) for k in range(2)]
    assert np.allclose(c, parts[0] + parts[1], rtol=1e-13)
    c1 = flow.importance_weights(f, lq, order_weights=[0.0, 2.0, 5.0])
    assert np.allclose(c1, 2 * parts[1], rtol=1e-13)
    assert math.isclose(float(np.sum(c)), 2.0, rel_tol=1e-12)
