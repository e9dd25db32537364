"""FP64 reference of the learned warm-start network and its training step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU
leg, never by the library.

The network is not part of the paper (its only warm start is the previous
step's impulses, Sec. 4.1); it maps a world's state features to the dual
impulses of the coming step.  Definition followed here:

* input standardisation  x^ = (x - mu_in) * s_in   (padded features are 0)
* z1 = W1 x^ + b1,  h1 = gelu(z1),  z2 = W2 h1 + b2,  h2 = gelu(z2),
  y^ = W3 h2 + b3,  y = mu_out + sigma_out * y^
* gelu(z) = z Phi(z) with Phi the standard normal CDF (erf form)
* loss = mean over the batch and the n_out active outputs of (y^ - t^)^2,
  t^ = (t - mu_out) / sigma_out
* Adam (Kingma and Ba 2015): beta1 0.9, beta2 0.999, eps 1e-8, bias
  corrected, on FP32 master weights.

With ``bf16=True`` every GEMM operand is rounded to bfloat16 (round to
nearest even of the FP32 value) at the points where the device kernels round
them: the normalised input, the weights, the hidden activations h1 and h2,
and in the backward pass the output gradient and the pre-activation
gradients.  Products and sums are FP64, so a comparison with the device
isolates the FP32 accumulation order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8
_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def bf16_round(a):
    """Round to bfloat16 (nearest, ties to even) after rounding to FP32, and
    return the value as FP64.  NaN stays NaN."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z * _SQRT1_2))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z * _SQRT1_2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


@dataclass
class MLP:
    """Weights in the device's packed order: W1 [H, n_in_pad], b1 [H],
    W2 [H, H], b2 [H], W3 [n_out_pad, H], b3 [n_out_pad]."""
    n_in: int
    n_hidden: int
    n_out: int
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray
    mu_in: np.ndarray
    s_in: np.ndarray
    mu_out: np.ndarray
    sigma_out: np.ndarray
    m: list = field(default_factory=list)
    v: list = field(default_factory=list)
    t: int = 0

    @property
    def n_in_pad(self):
        return self.W1.shape[1]

    @property
    def n_out_pad(self):
        return self.W3.shape[0]

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def packed(self):
        return np.concatenate([p.ravel() for p in self.params()])

    @staticmethod
    def from_packed(n_in, n_hidden, n_out, vec, mu_in=None, s_in=None, mu_out=None, sigma_out=None):
        fp = pad64(n_in)
        op = pad64(n_out)
        shapes = [(n_hidden, fp), (n_hidden,), (n_hidden, n_hidden), (n_hidden,), (op, n_hidden), (op,)]
        out, k = [], 0
        vec = np.asarray(vec, dtype=np.float64)
        for s in shapes:
            n = int(np.prod(s))
            out.append(vec[k:k + n].reshape(s).copy())
            k += n
        assert k == vec.size
        mu_in = np.zeros(fp) if mu_in is None else np.asarray(mu_in, np.float64)
        s_in = np.ones(fp) if s_in is None else np.asarray(s_in, np.float64)
        mu_out = np.zeros(op) if mu_out is None else np.asarray(mu_out, np.float64)
        sigma_out = np.ones(op) if sigma_out is None else np.asarray(sigma_out, np.float64)
        return MLP(n_in, n_hidden, n_out, *out, mu_in=mu_in, s_in=s_in, mu_out=mu_out, sigma_out=sigma_out)


def pad64(n):
    return (int(n) + 63) // 64 * 64


def _r(a, bf16):
    return bf16_round(a) if bf16 else a


def normalise_input(net, x):
    """x [B, n_in] -> x^ [B, n_in_pad] with zero padding."""
    B = x.shape[0]
    xh = np.zeros((B, net.n_in_pad))
    xh[:, :net.n_in] = (x - net.mu_in[:net.n_in]) * net.s_in[:net.n_in]
    return xh


def forward(net, x, bf16=True):
    """Returns (y [B, n_out] physical, cache)."""
    xh = _r(normalise_input(net, np.asarray(x, np.float64)), bf16)
    W1, W2, W3 = (_r(w, bf16) for w in (net.W1, net.W2, net.W3))
    z1 = xh @ W1.T + net.b1
    h1 = _r(gelu(z1), bf16)
    z2 = h1 @ W2.T + net.b2
    h2 = _r(gelu(z2), bf16)
    yn = h2 @ W3.T + net.b3
    y = net.mu_out + net.sigma_out * yn
    cache = dict(xh=xh, z1=z1, h1=h1, z2=z2, h2=h2, yn=yn, W1=W1, W2=W2, W3=W3)
    return y[:, :net.n_out], cache


def loss_and_grads(net, x, t, bf16=True):
    """Loss and gradients with respect to (W1, b1, W2, b2, W3, b3)."""
    x = np.asarray(x, np.float64)
    t = np.asarray(t, np.float64)
    B = x.shape[0]
    _, c = forward(net, x, bf16)
    tn = np.zeros((B, net.n_out_pad))
    tn[:, :net.n_out] = (t - net.mu_out[:net.n_out]) / net.sigma_out[:net.n_out]
    err = c["yn"] - tn
    err[:, net.n_out:] = 0.0
    loss = float((err ** 2).sum() / (B * net.n_out))
    dyn = 2.0 * err / (B * net.n_out)
    dy_r = _r(dyn, bf16)
    gW3 = dy_r.T @ c["h2"]
    gb3 = dyn.sum(axis=0)
    dz2 = (dy_r @ c["W3"]) * gelu_grad(c["z2"])
    dz2_r = _r(dz2, bf16)
    gW2 = dz2_r.T @ c["h1"]
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2_r @ c["W2"]) * gelu_grad(c["z1"])
    dz1_r = _r(dz1, bf16)
    gW1 = dz1_r.T @ c["xh"]
    gb1 = dz1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(net, grads, lr):
    """One bias-corrected Adam update of the FP64 weights (in place)."""
    if not net.m:
        net.m = [np.zeros_like(p) for p in net.params()]
        net.v = [np.zeros_like(p) for p in net.params()]
    net.t += 1
    c1 = 1.0 - BETA1 ** net.t
    c2 = 1.0 - BETA2 ** net.t
    for p, g, m, v in zip(net.params(), grads, net.m, net.v):
        m *= BETA1
        m += (1.0 - BETA1) * g
        v *= BETA2
        v += (1.0 - BETA2) * g * g
        p -= lr * (m / c1) / (np.sqrt(v / c2) + ADAM_EPS)
