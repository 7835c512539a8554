"""Pins of the surrogate perceptron's FP64 oracle (CPU only).

  * BF16 rounding equals torch's CPU float32 -> bfloat16 conversion (a library
    routine) on random, tie and special values;
  * GELU: closed-form values (0, Phi(1), Phi(-1), large |z|) and its
    derivative against central differences;
  * gradients of the FP64 network (no rounding) against central finite
    differences of the loss, on parameters of every layer;
  * one Adam step against its closed form (the first bias-corrected step
    moves each parameter by lr * g / (|g| + eps));
  * with zero weights the network outputs its last bias.
"""
import math
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import mlp_oracle as M  # noqa: E402


def test_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 1000), rng.normal(0, 1e4, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 1.0078125, 3.4e38, -3.4e38, 1e-40]])
    x = x.astype(np.float32)
    # exact ties: mantissa halfway between two bf16 values, both parities
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32) + np.float32(0)
    x = np.concatenate([x, ties, (0x3F800000 | np.arange(0, 2000, 7, dtype=np.uint32)).view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = M.bf16(x)
    assert np.array_equal(got, ref)


def test_gelu_closed_forms():
    phi1 = 0.5 * (1.0 + math.erf(1.0 / math.sqrt(2.0)))
    assert M.gelu(0.0) == 0.0
    assert abs(float(M.gelu(1.0)) - 0.8413447460685429) < 1e-15 and abs(phi1 - 0.8413447460685429) < 1e-15
    assert abs(float(M.gelu(-1.0)) + (1.0 - 0.8413447460685429)) < 1e-15
    assert abs(float(M.gelu(12.0)) - 12.0) < 1e-12 and abs(float(M.gelu(-12.0))) < 1e-30
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(z))) < 1e-8


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    w = M.init_params(5, scale=0.5)
    B = 6
    x = rng.normal(0, 1, size=(B, 296))
    t = rng.normal(0, 1, size=(B, 7))
    loss, g = M.loss_and_grads(w, x, t, emulate_bf16=False)
    # a few coordinates of every weight matrix and bias
    offs, off = [], 0
    for l in range(5):
        k, n = M.SIZES[l], M.SIZES[l + 1]
        offs += [off + int(i) for i in rng.integers(0, n * k, 4)] + [off + n * k + int(i) for i in rng.integers(0, n, 2)]
        off += n * k + n
    h = 1e-6
    for i in offs:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.loss_and_grads(wp, x, t, False)[0] - M.loss_and_grads(wm, x, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-3, 1e-8
    w1, m1, m2 = M.adam_step(w, np.zeros(50), np.zeros(50), g, 1, lr, 0.9, 0.999, eps)
    assert np.allclose(w - w1, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_zero_weights_give_last_bias():
    w = np.zeros(M.param_count())
    b = np.arange(7, dtype=np.float64)
    w[-7:] = b
    y, _, _ = M.forward(w, np.random.default_rng(0).normal(size=(3, 296)), emulate_bf16=True)
    assert np.array_equal(y, np.tile(b, (3, 1)))
    assert M.param_count() == 275207


# ------------------------------------------------------ feature oracle pins ---
def test_feature_pair_counts_ideal_gas_and_hand_cases():
    """g(r) of uniform points is 1 within Poisson error; a pair at a known
    separation lands in the shell floor(32 ln(r/R) / ln(r_m/R)); the
    concentration of one molecule in 1 um^3 is 1/(N_A 1e-15 L)."""
    from oracle import surrogate_oracle as S
    rng = np.random.default_rng(0)
    L = 400.0
    n = 6000
    xyz = rng.uniform(-L / 2, L / 2, size=(n, 3)).astype(np.float32)
    sp = np.zeros(n, dtype=np.int64)
    uid = np.arange(n, dtype=np.uint64)
    _, e2, vol = S.shells(1.0, L, 150.0)
    hist, nref = S.pair_counts(xyz, sp, uid, 0, 0, L, e2, 300)
    assert 280 <= nref <= 320
    expect = nref * ((n - 1) / L ** 3) * vol
    z = (hist - expect) / np.sqrt(expect)
    assert np.all(np.abs(z[expect > 50]) < 5) and abs(hist.sum() / expect.sum() - 1) < 0.02
    # two molecules at a known separation
    R, rm = 0.5, 100.0
    e, e2, _ = S.shells(R, 1000.0, rm)
    for r in (0.3, 0.7, 3.0, 42.0, 99.0):
        xyz2 = np.array([[0, 0, 0], [r, 0, 0]], dtype=np.float32)
        h2, _ = S.pair_counts(xyz2, np.array([0, 1]), np.array([0, 1], dtype=np.uint64), 0, 1, 1000.0, e2, 10)
        k = max(0, int(math.floor(32 * math.log(r / R) / math.log(rm / R)))) if r >= R else 0
        assert h2[k] == 1 and h2.sum() == 1, (r, k, np.nonzero(h2))
    f = S.features(np.zeros((1, 3), dtype=np.float32), np.array([1]), np.array([0], dtype=np.uint64), 1000.0,
                   [1.0] * 7, [], 10.0, c_floor=1e-30)
    assert abs(10 ** f[1] - 1.0 / (6.02214076e23 * 1e-15)) < 1e-12 * 10 ** f[1] and abs(f[-1] - 1.0) < 1e-15
