"""Parity of the surrogate perceptron's HIP kernels (BF16 matrix cores, FP32
accumulation) with the FP64 oracle, through the C ABI.

Tolerances: each layer is checked from the device's own input activations so
that only the FP32 accumulation order differs from the oracle's FP64 sums:
hidden outputs (BF16) agree exactly or by one BF16 step where the FP32 sum
sits at a rounding boundary (at most 1% of the entries); the FP32 outputs
agree to 1e-5 of the sum of |terms|.  Gradients (BF16 operands of the
products, FP32 sums) against the oracle with the same rounding: relative L2
error below 2e-2 per layer.  Adam: the device step equals the FP64 formula
applied to the device's gradients to 1e-5 relative.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import mlp_oracle as M  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the device"
    from paper_2509_03313_amd import gsbs
    return gsbs, torch


def layers_of(w):
    return M.unflatten(w.astype(np.float64))


def test_forward_layers(env):
    g, torch = env
    B = 37  # ragged: not a multiple of 16
    rng = np.random.default_rng(11)
    w = M.init_params(2, scale=0.7).astype(np.float32)
    w[-7:] = rng.normal(size=7)
    x = rng.normal(0, 1.5, size=(B, 296)).astype(np.float32)
    say("mlp forward", B)
    net = g.Mlp(64)
    net.set_weights(w)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    layers = layers_of(w)
    acts = [net.activation(l, B).astype(np.float64) for l in range(5)]
    assert np.array_equal(acts[0], M.bf16(x))
    for l in range(4):
        W, b = layers[l]
        Wr = M.bf16(W)
        z = acts[l] @ Wr.T + b
        ref = M.bf16(M.gelu(z))
        # the FP32 sum may differ from the FP64 one by a few ulp of the sum of |terms|,
        # and the FP32 GELU (erff) by a few ulp of its value; BF16 rounding is monotone
        dz = 2e-6 * (np.abs(acts[l]) @ np.abs(Wr).T + np.abs(b))
        gv = np.stack([M.gelu(z), M.gelu(z - dz), M.gelu(z + dz)])
        slack = 1e-6 * np.abs(gv).max(axis=0) + 1e-30
        lo, hi = M.bf16(gv.min(axis=0) - slack), M.bf16(gv.max(axis=0) + slack)
        got = acts[l + 1]
        frac = np.mean(got != ref)
        bad = ~((got >= lo) & (got <= hi))
        say("layer", l, "entries off the FP64 rounding", frac, "outside the bound", int(bad.sum()))
        if bad.any():
            i = np.argwhere(bad)[0]
            say("first", i, got[tuple(i)], ref[tuple(i)], z[tuple(i)], dz[tuple(i)])
        assert not bad.any(), l
        assert frac <= 0.01
    W, b = layers[4]
    ref = acts[4] @ M.bf16(W).T + b
    scale = np.abs(acts[4]) @ np.abs(M.bf16(W)).T + np.abs(b)
    assert np.all(np.abs(y - ref) <= 1e-5 * scale + 1e-6)
    net.close()


def test_backward_matches_oracle(env):
    g, torch = env
    B = 50
    rng = np.random.default_rng(12)
    w = M.init_params(4, scale=0.7).astype(np.float32)
    x = rng.normal(0, 1.0, size=(B, 296)).astype(np.float32)
    t = rng.normal(0, 1.0, size=(B, 7)).astype(np.float32)
    say("mlp backward", B)
    net = g.Mlp(64)
    net.set_weights(w)
    loss = net.backward(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    gg = net.get_grads().astype(np.float64)
    lo, go = M.loss_and_grads(w.astype(np.float64), x, t, emulate_bf16=True)
    assert abs(loss - lo) <= 1e-3 * lo
    off = 0
    for l in range(5):
        k, n = M.SIZES[l], M.SIZES[l + 1]
        for sl in (slice(off, off + n * k), slice(off + n * k, off + n * k + n)):
            a, b = gg[sl], go[sl]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            say("layer", l, "grad rel err", rel)
            assert rel < 2e-2
        off += n * k + n
    net.close()


def test_adam_and_training(env):
    g, torch = env
    B = 256
    rng = np.random.default_rng(13)
    w = M.init_params(6, scale=0.5).astype(np.float32)
    x = rng.normal(0, 1.0, size=(B, 296)).astype(np.float32)
    # a smooth target of the inputs
    A = rng.normal(0, 0.1, size=(296, 7))
    t = np.tanh(x @ A).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    net = g.Mlp(B)
    net.set_weights(w)
    # one Adam step equals the FP64 formula applied to the device's gradients
    net.backward(xd, td)
    gr = net.get_grads().astype(np.float64)
    net.adam(1e-3)
    w1 = net.get_weights().astype(np.float64)
    ref, _, _ = M.adam_step(w.astype(np.float64), 0.0, 0.0, gr, 1, 1e-3)
    assert np.allclose(w1, ref, rtol=1e-5, atol=1e-7)
    say("mlp training")
    first = None
    for it in range(300):
        loss = net.train_step(xd, td, 1e-3)
        first = loss if first is None else first
    say("loss", first, "->", loss)
    assert loss < 0.1 * first
    net.close()
