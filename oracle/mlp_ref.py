"""FP64 reference of the surrogate network (plain numpy).

TEST INFRASTRUCTURE ONLY (see oracle.py).  The surrogate is not part of the
paper: it is a multilayer perceptron that emulates the moment maps of the
evaluation (Sec. 2.2.5) from the parameter row, used to screen candidates of
the nested sampler (Sec. 2.3.2).  This module states what the GPU network
computes, in the plainest form:

  inputs  x = encode(p): every free slot s except PA mapped linearly from its
          prior box to [-1, 1]; PA as (cos PA, sin PA); fixed slots give 0;
          padded with zeros to a multiple of 32
  hidden  h_l = gelu(h_{l-1} W_l^T + b_l), gelu(z) = z Phi(z) (exact, erf form)
  output  y = h_L W_o^T + b_o: the velocity map / 300 then the dispersion
          map / 100 (km/s), row-major
  loss    sum mask (y - t)^2 / sum mask  (mask: truth flux >= 1% of its peak,
          the same mask on both maps)
  Adam    m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
          w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SLOT_ORDER = (0, 1, 2, 3, 4, 5, 6, 7, 8, 9)  # x0 y0 PA i Vsys Vt rt sigma r0 I0
PA = 2


def n_inputs() -> int:
    return 11


def encode(p: np.ndarray, lo: np.ndarray, hi: np.ndarray, pad_to: int = 32) -> np.ndarray:
    """[B][12] parameter rows -> [B][pad_to] inputs."""
    p = np.atleast_2d(np.asarray(p, dtype=np.float64))
    x = np.zeros((p.shape[0], pad_to))
    col = 0
    for s in SLOT_ORDER:
        if s == PA:
            a = np.radians(p[:, s])
            x[:, col], x[:, col + 1] = np.cos(a), np.sin(a)
            col += 2
        else:
            w = hi[s] - lo[s]
            x[:, col] = 2.0 * (p[:, s] - lo[s]) / w - 1.0 if w > 0 else 0.0
            col += 1
    return x


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(x, Ws, bs):
    """Returns the output and the list of (pre-activation, activation) pairs."""
    h, cache = x, []
    for W, b in zip(Ws[:-1], bs[:-1]):
        z = h @ W.T + b
        cache.append((z, h))
        h = gelu(z)
    y = h @ Ws[-1].T + bs[-1]
    cache.append((None, h))
    return y, cache


def loss_and_grads(x, t, mask, Ws, bs, with_terms=False):
    """Masked MSE and its gradients with respect to every weight and bias.
    mask [B][n_out] (1/0).  with_terms: also returns, per layer, the output
    gradient d_l and the layer input h_{l-1} whose product gives the weight
    gradient (for error bounds of lower-precision implementations)."""
    y, cache = forward(x, Ws, bs)
    cnt = max(float(mask.sum()), 1.0)
    r = (y - t) * mask
    loss = float(np.sum(r * r) / cnt)
    dy = 2.0 * r / cnt
    gW, gb = [None] * len(Ws), [None] * len(bs)
    terms = [None] * len(Ws)
    _, h = cache[-1]
    gW[-1], gb[-1] = dy.T @ h, dy.sum(axis=0)
    terms[-1] = (dy, h)
    dh = dy @ Ws[-1]
    for l in range(len(Ws) - 2, -1, -1):
        z, hin = cache[l]
        dz = dh * gelu_grad(z)
        gW[l], gb[l] = dz.T @ hin, dz.sum(axis=0)
        terms[l] = (dz, hin)
        dh = dz @ Ws[l]
    if with_terms:
        return loss, gW, gb, terms
    return loss, gW, gb


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return w, m, v
