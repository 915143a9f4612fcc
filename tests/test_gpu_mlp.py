"""The surrogate MLP's HIP kernels against the FP64 oracle (oracle/mlp_oracle.py).

The oracle takes the same bfloat16-rounded parameters and differs from the
GPU only by float32 arithmetic and summation order, so: outputs within
1e-5 (1 + |y|); gradients within 1e-4 of the largest component per element
and 1e-5 in the 2-norm; Adam steps identical where the gradient is not
within 1e-5 of zero relative to the largest component (there the FP32 sign
of m/sqrt(v) may differ).  Every call goes through the C ABI.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu

NORM = np.array([0.2, 4.0, 2.75e-3, -4.6, 0.12, 1.15, 1.3e-3, 1.33], np.float32)


@pytest.fixture(scope="module")
def mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import mlp
    mlp.lib()
    return mlp


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 17, 64, 1000, 10007])
def test_predict_matches_oracle(mlp, n):
    p0 = W.mlp_init(0)
    net = mlp.Mlp(p0, NORM)
    x = W.mlp_queries(n, seed=n)
    y = net.predict(_dev(x)).cpu().numpy()
    ref = M.forward(p0, x, NORM)
    print(f"[case] predict n={n} max err {np.abs(y - ref).max():.2e}", flush=True)
    assert np.all(np.abs(y - ref) <= 1e-5 * (1.0 + np.abs(ref)))


def test_used_params_are_bf16_rounded(mlp):
    p0 = W.mlp_init(1)
    net = mlp.Mlp(p0, NORM)
    p, q, _, _, _ = net.read()
    assert np.array_equal(p, p0)
    assert np.array_equal(q, M.bf16_round(p0))


@pytest.mark.parametrize("batch", [256, 37, 1])
def test_gradients_match_oracle(mlp, batch):
    rng = np.random.default_rng(batch)
    p0 = W.mlp_init(2)
    net = mlp.Mlp(p0, NORM)
    x = W.mlp_queries(batch, seed=100 + batch)
    t = rng.normal(size=batch).astype(np.float32)
    net.train_step(_dev(x), _dev(t), update=False)
    _, _, g, loss, steps = net.read()
    lref, gref = M.loss_and_grad(p0, x, t, NORM)
    err = np.abs(g - gref)
    print(f"[case] grad batch={batch} loss {loss} vs {lref}, max err {err.max():.2e} "
          f"of max |g| {np.abs(gref).max():.2e}", flush=True)
    assert steps == 0
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    assert np.all(err <= 1e-4 * np.abs(gref).max())
    assert np.linalg.norm(g - gref) <= 1e-5 * np.linalg.norm(gref)


def test_adam_step_matches_oracle(mlp):
    rng = np.random.default_rng(7)
    p0 = W.mlp_init(3)
    net = mlp.Mlp(p0, NORM, lr=1e-3)
    opt = M.Adam(p0, lr=1e-3)
    x = W.mlp_queries(256, seed=8)
    t = rng.normal(size=256).astype(np.float32)
    for step in range(3):
        _, gref = M.loss_and_grad(opt.p, x, t, NORM)
        net.train_step(_dev(x), _dev(t), update=True)
        pref = opt.step(gref)
        p, q, g, _, steps = net.read()
        assert steps == step + 1
        firm = np.abs(gref) > 1e-5 * np.abs(gref).max()
        if step == 0:
            # from identical parameters the step agrees to float32 rounding
            assert np.allclose(p[firm], pref[firm], rtol=0, atol=2e-7 + 1e-6 * 1e-3)
        assert np.array_equal(q, M.bf16_round(p))
        # keep the oracle on the GPU's parameters so the comparison stays local
        opt.p = p.copy()


def test_training_reduces_loss_like_the_oracle(mlp):
    x = W.mlp_queries(256, seed=11)
    t = (np.sin(3 * x[:, 0]) + 0.1 * x[:, 1] - 0.2 * x[:, 3]).astype(np.float32)
    p0 = W.mlp_init(7)
    net = mlp.Mlp(p0, NORM, lr=3e-3)
    opt = M.Adam(p0, lr=3e-3)
    xd, td = _dev(x), _dev(t)
    lg, lo = [], []
    for _ in range(200):
        net.train_step(xd, td, update=True)
        lg.append(net.read()[3])
        l, g = M.loss_and_grad(opt.p, x, t, NORM)
        opt.step(g)
        lo.append(l)
    print(f"[case] training loss gpu {lg[0]:.4f} -> {lg[-1]:.5f}, oracle {lo[0]:.4f} -> "
          f"{lo[-1]:.5f}", flush=True)
    assert lg[-1] < 0.1 * lg[0]
    assert abs(lg[-1] - lo[-1]) <= 0.1 * lo[-1] + 1e-4


def test_predict_is_repeatable(mlp):
    net = mlp.Mlp(W.mlp_init(4), NORM)
    x = _dev(W.mlp_queries(5000, seed=3))
    a = net.predict(x).cpu().numpy()
    b = net.predict(x).cpu().numpy()
    assert np.array_equal(a, b)
