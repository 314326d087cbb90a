"""Oracle: learned importance-sampling map (piecewise-linear coupling flow).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's integrator adapts its sampling density with Vegas (section 4.4);
this is the learned replacement: a normalising flow of piecewise-linear
coupling layers (Mueller, McWilliams, Rousselle, Gross, Novak, "Neural
Importance Sampling", ACM TOG 2019) whose map and Jacobian are applied in fp64,
so that the estimator E_u[f(x(u)) / q(x(u))] stays exactly unbiased whatever
the network's precision.  Only the network runs in reduced precision: its
weights and the activations entering each matrix product are bfloat16, products
accumulate in fp32 (here fp64; the difference is the accumulation order only).

Definition (one flow per sector, n variables):
* L = 4 layers; layer l transforms the variables B_l = {j : j = l mod 2} and
  conditions on A_l = the others (for n = 1, B_l = {0} and A_l is empty);
* MLP_l: a0 = bf16(2 h_A - 1); a1 = bf16(relu(W1 a0 + b1)); a2 = bf16(relu(W2 a1 + b2));
  logits = W3 a2 + b3 with bf16 weights, H = 64 hidden units, NB = 32 logits per
  transformed variable; every bf16 rounding (weights, input, activations) is
  straight-through in the gradient;
* Q_{j,k} = softmax_k(max(logits_j, max_k logits_j - 60)): bin probabilities of
  variable j, each logit raised to at most 60 below the largest (a constant of
  the map, no gradient through it), so that every bin keeps a positive
  probability in fp32 and the map's density is positive on the whole cube, which
  an unbiased importance-sampling estimator needs;
* forward (data h -> latent y), per j in B_l: b = min(floor(h_j NB), NB - 1),
  y_j = sum_{k<b} Q_k + (h_j NB - b) Q_b, log J += log(NB Q_b);
* inverse (latent -> data): b = the last bin whose running sum cum_b <= y_j,
  h_j = (b + (y_j - cum_b) / Q_b) / NB with the fraction clamped to [0, 1];
* sampling: y = u (uniform), layers applied inverse from L-1 down to 0;
  q(x) = prod over layers of prod_{j in B_l} NB Q_{b_j}, weight 1/q(x).
* initial parameters: W1, W2 uniform in (-1/sqrt(fan_in), 1/sqrt(fan_in)) from
  Philox4x32-10 (key = seed, counter = (parameter index, layer, sector,
  0x464c4f57)), biases and the output layer zero, so the initial map is the
  identity;
* training: for samples x_i drawn from q and weights c_i (held fixed), minimise
  -sum_i c_i log q(x_i) with Adam (beta1 0.9, beta2 0.999, eps 1e-8); with
  c_i proportional to rho(x_i)/q(x_i)^2 this is the score-function gradient of
  the variance (chi^2 divergence) of rho^(1/2)/q.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from .points import philox4x32_10

L_LAYERS = 4
HIDDEN = 64
NBINS = 32
INIT_TAG = 0x464C4F57
LOGIT_RANGE = 60.0


def masks(n: int):
    out = []
    for l in range(L_LAYERS):
        if n == 1:
            B, A = [0], []
        else:
            B = [j for j in range(n) if j % 2 == l % 2]
            A = [j for j in range(n) if j % 2 != l % 2]
        out.append((A, B))
    return out


def layer_shapes(n: int):
    """[(name, shape)] of every parameter, layer by layer, in storage order."""
    shapes = []
    for (A, B) in masks(n):
        na, nb = len(A), len(B)
        shapes.append([("W1", (HIDDEN, max(na, 1))), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
                       ("b2", (HIDDEN,)), ("W3", (nb * NBINS, HIDDEN)), ("b3", (nb * NBINS,))])
    return shapes


EMULATE_BF16 = True


def bf16(t: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (nearest even) and back, in the tensor's dtype."""
    if not EMULATE_BF16:
        return t
    return t.to(torch.float32).to(torch.bfloat16).to(t.dtype)


def ste_bf16(t: torch.Tensor) -> torch.Tensor:
    """bf16 value in the forward pass, identity in the backward pass."""
    return t + (bf16(t) - t).detach()


def init_params(n: int, seed: int, sector: int) -> List[dict]:
    """fp32 master parameters of one sector's flow (as float64 tensors holding fp32 values)."""
    params = []
    for l, shp in enumerate(layer_shapes(n)):
        d = {}
        idx = 0
        for name, shape in shp:
            size = int(np.prod(shape))
            if name in ("W1", "W2"):
                fan_in = shape[1]
                s = 1.0 / math.sqrt(fan_in)
                vals = np.empty(size)
                for i in range(size):
                    o = philox4x32_10((idx + i, l, sector, INIT_TAG), (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
                    u = (o[0] >> 8) * 2.0 ** -24
                    vals[i] = np.float32(s * (2.0 * u - 1.0))
                if name == "W1" and len(masks(n)[l][0]) == 0:
                    vals[:] = 0.0
                t = torch.tensor(vals.reshape(shape), dtype=torch.float64)
            else:
                t = torch.zeros(shape, dtype=torch.float64)
            d[name] = t
            idx += size
        params.append(d)
    return params


def _probs(p: dict, hA: torch.Tensor, nb: int) -> torch.Tensor:
    """Bin probabilities (npts, nb, NBINS) from the MLP of one layer."""
    npts = hA.shape[0]
    if hA.shape[1] == 0:
        a0 = torch.zeros((npts, 1), dtype=torch.float64)
    else:
        a0 = ste_bf16(2.0 * hA - 1.0)
    a1 = ste_bf16(torch.relu(a0 @ ste_bf16(p["W1"]).T + p["b1"]))
    a2 = ste_bf16(torch.relu(a1 @ ste_bf16(p["W2"]).T + p["b2"]))
    logits = (a2 @ ste_bf16(p["W3"]).T + p["b3"]).reshape(npts, nb, NBINS)
    floor = torch.amax(logits, dim=2, keepdim=True).detach() - LOGIT_RANGE
    return torch.softmax(torch.maximum(logits, floor), dim=2)


def log_q(params: List[dict], x: torch.Tensor) -> torch.Tensor:
    """log q(x) by the forward direction (data -> latent); differentiable in the params."""
    return forward(params, x)[1]


def forward(params: List[dict], x: torch.Tensor):
    """Latent point and log q(x) of data points x (the forward direction)."""
    n = x.shape[1]
    h = x.clone()
    lq = torch.zeros(x.shape[0], dtype=torch.float64)
    for l, (A, B) in enumerate(masks(n)):
        Q = _probs(params[l], h[:, A], len(B))
        hB = h[:, B]
        b = torch.clamp(torch.floor(hB.detach() * NBINS), max=NBINS - 1).long()
        alpha = hB * NBINS - b
        cum = torch.cumsum(Q, dim=2) - Q
        qb = torch.gather(Q, 2, b[..., None])[..., 0]
        cb = torch.gather(cum, 2, b[..., None])[..., 0]
        y = cb + alpha * qb
        lq = lq + torch.sum(torch.log(NBINS * qb), dim=1)
        h = h.clone()
        h[:, B] = y
    return h, lq


@torch.no_grad()
def sample(params: List[dict], u: np.ndarray):
    """x and log q(x) for latent points u (npts, n) by the inverse layers."""
    n = u.shape[1]
    h = torch.tensor(u, dtype=torch.float64)
    lq = torch.zeros(u.shape[0], dtype=torch.float64)
    for l in reversed(range(L_LAYERS)):
        A, B = masks(n)[l]
        Q = _probs(params[l], h[:, A], len(B)).numpy()
        hB = h[:, B].numpy()
        out = np.empty_like(hB)
        for i in range(hB.shape[0]):
            for jj in range(hB.shape[1]):
                q = Q[i, jj]
                y = hB[i, jj]
                cum, b, cb = 0.0, 0, 0.0
                for k in range(NBINS):           # last bin whose running sum is <= y
                    if cum <= y:
                        b, cb = k, cum
                    cum += q[k]
                frac = min(max((y - cb) / q[b], 0.0), 1.0)
                out[i, jj] = (b + frac) / NBINS
                lq[i] += math.log(NBINS * q[b])
        h[:, B] = torch.tensor(out)
    return h.numpy(), lq.numpy()


def loss_and_grad(params: List[dict], x: np.ndarray, c: np.ndarray):
    """L = -sum_i c_i log q(x_i) and dL/dparams (straight-through for the bf16 roundings)."""
    P = [{k: v.clone().requires_grad_(True) for k, v in d.items()} for d in params]
    xt = torch.tensor(x, dtype=torch.float64)
    L = -(torch.tensor(c, dtype=torch.float64) * log_q(P, xt)).sum()
    L.backward()
    return float(L.detach()), [{k: v.grad.clone() for k, v in d.items()} for d in P]


@dataclass
class AdamState:
    m: List[dict]
    v: List[dict]
    t: int = 0


def adam_init(params) -> AdamState:
    return AdamState([{k: torch.zeros_like(v) for k, v in d.items()} for d in params],
                     [{k: torch.zeros_like(v) for k, v in d.items()} for d in params])


def adam_step(params, grads, st: AdamState, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the fp32 master parameters (values kept representable in fp32)."""
    st.t += 1
    for d, g, m, v in zip(params, grads, st.m, st.v):
        for k in d:
            m[k] = (b1 * m[k] + (1 - b1) * g[k]).float().double()
            v[k] = (b2 * v[k] + (1 - b2) * g[k] * g[k]).float().double()
            mh = m[k] / (1 - b1 ** st.t)
            vh = v[k] / (1 - b2 ** st.t)
            d[k] = (d[k] - lr * mh / (torch.sqrt(vh) + eps)).float().double()
    return params


def importance_weights(f: np.ndarray, logq: np.ndarray, order_weights=None) -> np.ndarray:
    """c_i = sum_k w_k (|f_k(x_i)|^2 / q_i^2) / S_k, S_k the batch total of that order
    (zero orders skipped), w_k the caller's order weights (default 1)."""
    w2 = np.exp(-2.0 * logq)
    a = np.abs(f) ** 2 * w2[None, :]
    c = np.zeros(f.shape[1])
    for k in range(f.shape[0]):
        tot = a[k].sum()
        wk = 1.0 if order_weights is None else float(order_weights[k])
        if tot > 0.0 and np.isfinite(tot) and wk != 0.0:
            c += wk * a[k] / tot
    return c
