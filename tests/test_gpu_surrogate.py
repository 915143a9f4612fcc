"""The surrogate workflow end to end on the GPU: viscosities measured by the
batched viscometer, the network trained on them by its own kernels, the
plain simulation answering outside the training box, and what the network
gains over running the simulation."""
import math
import time

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu

KW = dict(side=(10, 12), shear=(3e-2, 1e-1), steps=600)


@pytest.fixture(scope="module")
def SG():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import surrogate
    return surrogate


@pytest.fixture(scope="module")
def trained(SG):
    _, cells = W.viscometer_batch(96, seed=21, **KW)
    print(f"[case] measuring {len(cells)} cells", flush=True)
    eta, se = SG.measure(cells, KW["steps"])
    x = SG.features([c[2] for c in cells])
    ok = eta > 0
    y = np.log(eta[ok]).astype(np.float32)
    net, hist = SG.train(x[ok], y, epochs=300, seed=3)
    return net, x[ok], y, hist


def test_training_fits_the_measured_viscosities(SG, trained):
    net, x, y, hist = trained
    sur = SG.Surrogate(net, SG.BOX_LO, SG.BOX_HI)
    pred = np.log(sur.predict(x))
    resid = np.mean((pred - y) ** 2)
    spread = np.var(y)
    print(f"[case] loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}, residual {resid:.4f} of "
          f"variance {spread:.4f}", flush=True)
    assert hist[-1][1] < hist[0][1]
    assert resid < spread  # better than the mean of the data


def test_outside_the_box_the_plain_simulation_answers(SG, trained):
    net = trained[0]
    cell_kw = dict(n_side=10, steps=KW["steps"])
    sur = SG.Surrogate(net, SG.BOX_LO, SG.BOX_HI, cell_kw=cell_kw, fallback_steps=KW["steps"])
    q = np.array([[0.2, 3.0, 1e-3, math.log(5e-2)],     # inside
                  [0.45, 3.0, 1e-3, math.log(5e-2)]],   # phi above the box
                 np.float32)
    out, sim = sur.query(q, seed=77)
    assert list(sim) == [False, True]
    # the same cell built from the query's float32 values, run directly
    direct = SG.measure([W.shear_cell(phi=float(q[1, 0]), d=float(q[1, 1]), kBT=float(q[1, 2]),
                                      shear_rate=float(math.exp(q[1, 3])), seed=77, **cell_kw)],
                        KW["steps"])[0]
    assert out[1] == direct[0]
    assert out[0] == sur.predict(q[:1])[0]


def test_network_answers_far_faster_than_the_simulation(SG, trained):
    import torch
    net = trained[0]
    q = torch.from_numpy(W.mlp_queries(1 << 20, seed=1)).cuda()
    net.predict(q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.predict(q)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    t0 = time.perf_counter()
    SG.measure([W.shear_cell(12, 0.2, 3.0, seed=5)], 200)
    t_sim = time.perf_counter() - t0
    print(f"[case] 2^20 network answers in {t_net * 1e3:.3f} ms; one 200-step plain run "
          f"{t_sim * 1e3:.1f} ms", flush=True)
    assert t_net < t_sim
