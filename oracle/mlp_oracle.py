"""FP64 CPU oracle of the inter-pulse surrogate perceptron -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and bench.py's CPU-baseline leg may import this
module; the HIP engine never imports, links or calls it and shares no code with
it.  Plain numpy in float64, written from the definitions:

  * network: x -> [W_l a + b_l, GELU after the hidden layers] for layers
    296-256-256-256-256-7; GELU(z) = z * Phi(z) with Phi the standard normal
    CDF (erf form); loss = mean of the squared output errors;
  * BF16 emulation (optional): the operands the device rounds to BF16 (the
    input, the weights, the hidden activations, and in the backward pass the
    output-side gradients) are rounded to nearest even on 8 significant bits,
    then every sum is taken in float64;
  * backward pass by the chain rule; Adam (Kingma & Ba, bias-corrected).

Flat parameter layout (as the C ABI): per layer W[n_out][n_in] row-major, then
b[n_out].
"""
from __future__ import annotations

import math

import numpy as np

SIZES = [296, 256, 256, 256, 256, 7]


def param_count() -> int:
    return sum(SIZES[l] * SIZES[l + 1] + SIZES[l + 1] for l in range(len(SIZES) - 1))


def unflatten(w: np.ndarray):
    out, off = [], 0
    for l in range(len(SIZES) - 1):
        k, n = SIZES[l], SIZES[l + 1]
        W = np.asarray(w[off:off + n * k], dtype=np.float64).reshape(n, k)
        off += n * k
        b = np.asarray(w[off:off + n], dtype=np.float64)
        off += n
        out.append((W, b))
    assert off == len(w)
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64.
    The value is first rounded to float32 (the device holds FP32 values)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(w, x, emulate_bf16=True):
    """Output y[B][7] and the activations entering each layer (acts[0] = the
    possibly rounded input) and the hidden pre-activations."""
    layers = unflatten(w)
    r = bf16 if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    acts, pre = [a], []
    for l, (W, b) in enumerate(layers):
        z = a @ r(W).T + b
        if l + 1 < len(layers):
            pre.append(z)
            a = r(gelu(z))
            acts.append(a)
        else:
            return z, acts, pre
    raise AssertionError


def loss_and_grads(w, x, t, emulate_bf16=True):
    """Mean squared error and its gradient in the flat layout."""
    layers = unflatten(w)
    r = bf16 if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    y, acts, pre = forward(w, x, emulate_bf16)
    B, n_out = y.shape
    diff = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / (B * n_out)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dzr = r(dz)
        grads[l] = (dzr.T @ acts[l], dz.sum(axis=0))
        if l == 0:
            break
        da = dzr @ r(W)
        dz = da * gelu_grad(pre[l - 1])
    return loss, flatten(grads)


def adam_step(w, m1, m2, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (w, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2


def init_params(seed: int, scale: float = 1.0) -> np.ndarray:
    """He-uniform weights (limit sqrt(6 / n_in)), zero biases; seeded."""
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(len(SIZES) - 1):
        k, n = SIZES[l], SIZES[l + 1]
        lim = scale * math.sqrt(6.0 / k)
        layers.append((rng.uniform(-lim, lim, size=(n, k)), np.zeros(n)))
    return flatten(layers)
