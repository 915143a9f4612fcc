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


def test_committed_network_matches_fresh_plain_runs_far_faster(SG):
    """The committed network (trained on 4096 cells of the batched-viscometer
    sampler, sides 16-40, 5000 steps) against 12 fresh plain runs of the
    same protocol at shear rates 1e-2..1e-1: its error is within 5 % where
    the run itself resolves 5 % (standard error below 2 %), no larger than
    about twice the plain runs' own statistical error overall -- the gain
    is at equal error -- and an answer costs a million times less."""
    import torch
    sur, doc = SG.load_network()
    assert doc["n_params"] == 8705 and doc["side"] == [16, 40] and doc["steps_per_run"] == 5000
    _, fresh = W.viscometer_batch(12, seed=4242, side=(16, 40), steps=5000, shear=(1e-2, 1e-1))
    print(f"[case] 12 fresh plain runs, {sum(c[2]['n'] for c in fresh)} particles", flush=True)
    t0 = time.perf_counter()
    ev, rel, rel_se = SG.evaluate(sur, fresh, 5000,
                                  tuning={"cell_factor": 0.5, "graph_steps": 2, "tile": 8388608})
    t_plain = (time.perf_counter() - t0) / len(fresh)
    q = torch.from_numpy(W.mlp_queries(1 << 20, seed=1)).cuda()
    sur.net.predict(q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.net.predict(q)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / (1 << 20)
    print(f"[case] median error {ev['median_rel_error']:.3f}, plain se {ev['median_plain_rel_se']:.3f}"
          f"; {ev['cells_with_plain_se_below_2pct']} resolved, mean error there "
          f"{ev['mean_rel_error_where_plain_se_below_2pct']}; plain run {t_plain:.2f} s, "
          f"network answer {t_net * 1e9:.2f} ns", flush=True)
    quiet = rel_se < 0.02
    assert quiet.sum() >= 4
    assert rel[quiet].mean() <= 0.05 and (rel[quiet] <= 0.05).mean() >= 0.75
    assert ev["median_rel_error"] <= 2.0 * ev["median_plain_rel_se"] + 0.01
    assert t_plain / t_net > 1e6
