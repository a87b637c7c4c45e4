"""numpy forward/backward of the learned proposal -- TEST INFRASTRUCTURE ONLY.

Network (weights as in the library: W1 [H][Kp], b1 [H], W2 [H][H], b2 [H],
W3 [Mp][H], b3 [Mp]; padding columns/rows zero):
    f  = log1p(X) (N inputs, zero-padded to Kp)
    h1 = relu(W1 f + b1),  h2 = relu(W2 h1 + b2),  z = W3 h2 + b3
    q  = softmax of z over the reactions with alpha_j > 0 (0 elsewhere)
    loss = mean over rows of -sum_j p_j log q_j,  p = alpha / sum(alpha)
Backward: dz = (q - p) / B, dW3 = dz^T h2, db3 = sum dz, dh2 = dz W3 . [h2 > 0],
dW2 = dh2^T h1, db2 = sum dh2, dh1 = dh2 W2 . [h1 > 0], dW1 = dh1^T f, db1 = sum dh1.

With mirror_bf16 the weights, f, h1, h2 and the propagated gradients are
rounded to bfloat16 (nearest even) where the GPU stores them in that format;
all arithmetic is float64.  Without it the computation is plain float64
(used for the finite-difference pin).

Optimizer: Adam (Kingma & Ba, "Adam: a method for stochastic optimization",
ICLR 2015, Algorithm 1) on float32 master weights, every operation rounded to
float32 in the order of that algorithm's update rules (adam_step).

Pins (tests/test_oracle_mlp.py): a network small enough to evaluate by hand
(forward values, loss), central finite differences of the backward pass,
and closed forms of two Adam steps on scalars.
"""
from __future__ import annotations

import math

import numpy as np


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def _r(x, on):
    return bf16_round(np.asarray(x, np.float32)).astype(np.float64) if on else np.asarray(x, np.float64)


def features(X, N, Kp, mirror_bf16=True):
    f = np.zeros((X.shape[0], Kp), dtype=np.float64)
    f[:, :N] = np.log1p(np.maximum(np.asarray(X, np.float64), 0.0)).astype(np.float32)
    return _r(f, mirror_bf16)


def forward(params, X, alpha, N, M, mirror_bf16=True):
    W1, b1, W2, b2, W3, b3 = params
    Kp = W1.shape[1]
    f = features(X, N, Kp, mirror_bf16)
    W1r, W2r, W3r = (_r(w, mirror_bf16) for w in (W1, W2, W3))
    pre1 = f @ W1r.T + b1
    h1 = _r(np.maximum(pre1, 0.0), mirror_bf16)
    pre2 = h1 @ W2r.T + b2
    h2 = _r(np.maximum(pre2, 0.0), mirror_bf16)
    z = h2 @ W3r.T + b3
    a = np.asarray(alpha, np.float64)
    sup = a > 0
    zm = np.where(sup, z[:, :M], -np.inf)
    zmax = zm.max(axis=1, keepdims=True)
    e = np.where(sup, np.exp(zm - zmax), 0.0)
    q = e / e.sum(axis=1, keepdims=True)
    return dict(f=f, h1=h1, h2=h2, z=z, q=q, sup=sup, W=(W1r, W2r, W3r))


def loss_and_grads(params, X, alpha, N, M, mirror_bf16=True):
    W1, b1, W2, b2, W3, b3 = params
    B = X.shape[0]
    fw = forward(params, X, alpha, N, M, mirror_bf16)
    q, sup = fw["q"], fw["sup"]
    a = np.asarray(alpha, np.float64)
    p = np.where(sup, a / a.sum(axis=1, keepdims=True), 0.0)
    logq = np.where(sup, np.log(np.where(sup, q, 1.0)), 0.0)
    loss = float(-(p * logq).sum() / B)
    dz = np.zeros((B, W3.shape[0]))
    dz[:, :M] = (q - p) / B
    dzr = _r(dz, mirror_bf16)
    W1r, W2r, W3r = fw["W"]
    g = [None] * 6
    g[4] = dzr.T @ fw["h2"]
    g[5] = dz.sum(axis=0)
    dh2 = (dzr @ W3r) * (fw["h2"] > 0)
    dh2r = _r(dh2, mirror_bf16)
    g[2] = dh2r.T @ fw["h1"]
    g[3] = dh2.sum(axis=0)
    dh1 = (dh2r @ W2r) * (fw["h1"] > 0)
    dh1r = _r(dh1, mirror_bf16)
    g[0] = dh1r.T @ fw["f"]
    g[1] = dh1.sum(axis=0)
    return loss, g, fw


def quantise(q, sup, M):
    """Q_j = max(1, floor(q_j 2^(31-L))) on the support, 0 elsewhere."""
    L = 0
    while (1 << L) < M:
        L += 1
    Q = np.floor(np.asarray(q, np.float64) * 2.0 ** (31 - L))
    Q = np.where(sup, np.maximum(Q, 1.0), 0.0)
    return Q.astype(np.uint64).astype(np.uint32)


def adam_step(w, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update at step t >= 1 (Kingma & Ba 2015, Algorithm 1), in
    float32 with each operation rounded as written:

        m_t   = beta1 * m_{t-1} + (1 - beta1) * g
        v_t   = beta2 * v_{t-1} + (1 - beta2) * (g * g)
        m_hat = m_t / c1,   c1 = 1 - beta1^t
        v_hat = v_t / c2,   c2 = 1 - beta2^t
        w_t   = w_{t-1} - (lr * m_hat) / (sqrt(v_hat) + eps)

    The bias corrections c1, c2 are computed in binary64 from the float32
    betas and rounded once to float32.  Returns (w_t, m_t, v_t) as new
    float32 arrays; the bfloat16 copy the GPU keeps is bf16_round(w_t)."""
    f = np.float32
    w, m, v, g = (np.asarray(x, dtype=np.float32) for x in (w, m, v, g))
    b1, b2, e, a = f(beta1), f(beta2), f(eps), f(lr)
    c1 = f(1.0 - math.pow(float(b1), float(t)))
    c2 = f(1.0 - math.pow(float(b2), float(t)))
    m_t = b1 * m + (f(1.0) - b1) * g
    v_t = b2 * v + (f(1.0) - b2) * (g * g)
    m_hat = m_t / c1
    v_hat = v_t / c2
    w_t = w - (a * m_hat) / (np.sqrt(v_hat) + e)
    return w_t.astype(np.float32), m_t.astype(np.float32), v_t.astype(np.float32)
