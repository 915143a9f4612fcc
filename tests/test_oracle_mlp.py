"""Pins of the FP64 surrogate-MLP oracle: bfloat16 rounding against brute
force, SiLU and the whole backward pass against central differences, a
single-path network against its closed form, and Adam's first two steps
against their closed forms."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2002_03120_amd import workloads as W

NORM = np.array([0.2, 4.0, 2.75e-3, -4.6, 0.12, 1.15, 1.3e-3, 1.33])


def test_param_count():
    assert W.mlp_param_count() == 8705
    assert W.mlp_init(0).size == 8705


def test_bf16_rounding_brute_force():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        np.float32([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0])])
    r = M.bf16_round(x)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
    bits = x.view(np.uint32)
    lo = (bits & 0xFFFF0000).view(np.float32).astype(np.float64)
    hi = ((bits & 0xFFFF0000) + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    xd = x.astype(np.float64)
    dl, dh = np.abs(xd - lo), np.abs(hi - xd)
    even_lo = ((bits >> 16) & 1) == 0
    expect = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(even_lo, lo, hi)))
    assert np.array_equal(r.astype(np.float64), expect)
    # the tie 1 + 2^-8 goes to the even neighbour 1.0; 1 + 3 2^-8 goes up
    assert r[-5] == 1.0 and r[-4] == 1.0 and r[-3] == np.float32(1.0 + 2.0 ** -6)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    e = 1e-5  # central differences: truncation ~e^2, rounding ~1e-16/e
    fd = (M.silu(z + e) - M.silu(z - e)) / (2 * e)
    assert np.allclose(M.silu_grad(z), fd, rtol=0, atol=1e-9)


def test_single_path_network_closed_form():
    p = np.zeros(8705, np.float32)
    Ws = M.split(p)
    Ws[0][0, 0] = 1.0
    Ws[2][0, 0] = 1.0
    Ws[4][0, 0] = 1.0
    Ws[6][0, 0] = 1.0
    Ws[7][0] = 0.5
    x = np.array([[0.3, 2.0, 1e-3, -3.0], [0.05, 5.0, 4e-3, -1.0]])
    xn = (x[:, 0] - NORM[0]) / NORM[4]
    s = lambda z: z / (1.0 + np.exp(-z))
    assert np.allclose(M.forward(p, x, NORM), s(s(s(xn))) + 0.5, rtol=1e-15, atol=0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    p = M.bf16_round(W.mlp_init(3)).astype(np.float64)
    p[M.split(np.arange(8705))[1]] = rng.normal(scale=0.1, size=64)  # nonzero biases
    x = W.mlp_queries(24, seed=2)
    t = rng.normal(size=24)
    loss, g = M.loss_and_grad(p, x, t, NORM, quantise=False)
    idx = rng.choice(8705, size=200, replace=False)
    idx = np.concatenate([idx, [8704, 8640, 0, 300, 4420]])
    for k in idx:
        e = 1e-6 * max(1.0, abs(p[k]))
        a, b = p.copy(), p.copy()
        a[k] += e
        b[k] -= e
        la = M.loss_and_grad(a, x, t, NORM, quantise=False)[0]
        lb = M.loss_and_grad(b, x, t, NORM, quantise=False)[0]
        fd = (la - lb) / (2 * e)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_adam_first_steps_closed_form():
    p0 = np.array([1.0, -2.0, 0.5], np.float32)
    opt = M.Adam(p0, lr=1e-2)
    g1 = np.array([0.3, -4.0, 1e-3])
    p1 = opt.step(g1)
    # first step: m^ = g, v^ = g^2, so the step is lr g / (|g| + eps)
    exp1 = p0.astype(np.float64) - 1e-2 * g1 / (np.abs(g1) + 1e-8)
    assert np.allclose(p1, exp1.astype(np.float32), rtol=0, atol=0)
    g2 = np.array([-0.3, 2.0, 3e-3])
    p2 = opt.step(g2)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    exp2 = p1.astype(np.float64) - 1e-2 * mh / (np.sqrt(vh) + 1e-8)
    assert np.allclose(p2, exp2.astype(np.float32), rtol=0, atol=0)


def test_training_reduces_loss():
    x = W.mlp_queries(256, seed=5)
    t = np.sin(3 * x[:, 0]) + 0.1 * x[:, 1] - 0.2 * x[:, 3]
    opt = M.Adam(W.mlp_init(7), lr=3e-3)
    l0 = None
    for _ in range(200):
        loss, g = M.loss_and_grad(opt.p, x, t, NORM)
        l0 = loss if l0 is None else l0
        opt.step(g)
    assert loss < 0.1 * l0
