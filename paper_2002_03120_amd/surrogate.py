"""The viscometer workflow: effective viscosities measured by batched
Lees-Edwards shear cells, a surrogate MLP trained on them on the GPU, and
queries answered by the network inside its training box and by the plain
simulation (the batched viscometer) outside it.

Every number comes from the HIP library (libsdpdem.so): the cells run on
sdpdem_create_batch / sdpdem_step / sdpdem_box_stress, the network on the
sdpdem_mlp_* kernels; this module only arranges inputs and averages the
per-box stress samples the library returns.

Viscosity: eta_eff = -<P_zx> / shear_rate over the second half of a run,
<.> the mean of the per-step samples; its standard error from block means
(blocks of `block` steps).  The network's target is log(eta_eff / eta).

    python -m paper_2002_03120_amd.surrogate --cells 4096 --steps 5000

The measurement can be split over several runs: --measure-only --range A B
writes the measured cells A..B-1 (features, eta_eff/eta, standard error) to
--data; a later run given those files with --train-from trains, evaluates
on fresh plain runs and writes the trained parameters (--save).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import autotune as AT
from . import mlp as MLP
from . import sdpdem as S
from . import workloads as W

# the sampling box of the viscometer (phi, d/dx, kT, log shear rate)
BOX_LO = np.array([0.0, 2.0, 5e-4, math.log(1e-3)])
BOX_HI = np.array([0.4, 6.0, 5e-3, math.log(1e-1)])


def features(infos):
    """(phi, d/dx, kT, log shear rate) of measured cells (the achieved phi)."""
    return np.array([[i["phi"], i["d"], i["kBT"], math.log(i["shear_rate"])] for i in infos],
                    np.float32)


def measure(cells, steps, block=50, chunk_particles=4_000_000, tuning=None, log=None):
    """Run the cells as batches of at most chunk_particles particles (on a
    side stream, the step loop replayed from captured graphs of 10 steps).
    A `tuning` from autotune.tune replaces the batch tile, the graph length
    and the cell size by its choice (graph length 0: eager steps with
    neighbour-candidate reuse).  Returns (eta_eff / eta, standard error
    of it) per cell."""
    import torch
    cell_factor, graph_steps = 1.0, 10
    if tuning is not None:
        cell_factor, graph_steps = tuning["cell_factor"], tuning["graph_steps"]
        chunk_particles = tuning["tile"]
    # stress is read every `block` steps: a whole number of graphs
    block = AT.steps_per_call(graph_steps, block)
    stream = torch.cuda.Stream()
    eta_rel = np.empty(len(cells))
    se_rel = np.empty(len(cells))
    for start, stop, n in AT.split(cells, chunk_particles):
        part = cells[start:stop]
        parts, boxes, box_of = W.stack_cells(part)
        p = AT.launch_params(part[0][0], cell_factor, graph_steps)
        g = S.System(p, parts, boxes=boxes, box_of=box_of, stream=stream)
        g.set_stress(True)
        g.set_graph(graph_steps)
        nb = len(part)
        sums = []
        prev = np.zeros(nb)
        for _ in range(steps // block):
            g.step(block)
            _, tot, _ = g.box_stress()
            sums.append(tot - prev)
            prev = tot
        del g
        torch.cuda.empty_cache()
        blocks = np.array(sums) / block  # block means of P_zx, [nblocks, nb]
        half = blocks[blocks.shape[0] // 2:]
        gd = np.array([c[2]["shear_rate"] for c in part])
        eta0 = np.array([c[0]["eta"] for c in part])
        mean = half.mean(axis=0)
        se = half.std(axis=0, ddof=1) / math.sqrt(max(half.shape[0], 2))
        eta_rel[start:stop] = -mean / gd / eta0
        se_rel[start:stop] = se / np.abs(gd) / eta0
        if log:
            log(f"measured cells {start}..{stop - 1} ({n} particles)")
    return eta_rel, se_rel


def normalisation(lo=BOX_LO, hi=BOX_HI):
    """Mean and standard deviation of the uniform sampling box (the inputs'
    fixed normalisation)."""
    mean = 0.5 * (lo + hi)
    std = (hi - lo) / math.sqrt(12.0)
    return np.concatenate([mean, std]).astype(np.float32)


class Surrogate:
    """The trained network plus the plain simulation as its fallback."""

    def __init__(self, net, lo, hi, cell_kw=None, fallback_steps=2000):
        self.net = net
        self.lo = np.asarray(lo, np.float32)
        self.hi = np.asarray(hi, np.float32)
        self.cell_kw = dict(cell_kw or {})
        self.fallback_steps = fallback_steps

    def inside(self, q):
        q = np.asarray(q, np.float32)
        return np.all((q >= self.lo) & (q <= self.hi), axis=1)

    def predict(self, q):
        """eta_eff / eta by the network (inputs as features())."""
        import torch
        x = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
        return np.exp(self.net.predict(x).cpu().numpy().astype(np.float64))

    def query(self, q, seed=12345):
        """Answers inside the training box from the network, the others by
        running the plain simulation for them.  Returns (eta_eff / eta,
        mask of the answers that came from the simulation)."""
        q = np.asarray(q, np.float32)
        ins = self.inside(q)
        out = np.empty(q.shape[0])
        if ins.any():
            out[ins] = self.predict(q[ins])
        if (~ins).any():
            cells = []
            for k, row in enumerate(q[~ins]):
                cells.append(W.shear_cell(phi=float(row[0]), d=float(row[1]), kBT=float(row[2]),
                                          shear_rate=float(math.exp(row[3])),
                                          seed=seed + k, **self.cell_kw))
            out[~ins] = measure(cells, self.fallback_steps)[0]
        return out, ~ins


def train(x, y, epochs=300, batch=256, lr=3e-3, seed=0, log=None):
    """Adam on the GPU over shuffled mini-batches; returns the network and
    the per-epoch mean training loss."""
    import torch
    net = MLP.Mlp(W.mlp_init(seed), normalisation(), lr=lr)
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    rng = np.random.default_rng(seed)
    hist = []
    n = x.shape[0]
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).cuda()
        tot = 0.0
        nb = 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            net.train_step(xd[idx], yd[idx], update=True)
            if ep == epochs - 1 or ep % 50 == 0:
                tot += net.read()[3]
                nb += 1
        if nb:
            hist.append((ep, tot / nb))
            if log:
                log(f"epoch {ep} loss {tot / nb:.5f}")
    return net, hist


PARAMS_PATH = __import__("os").path.join(__import__("os").path.dirname(__file__),
                                         "surrogate_params.json")


def save_params(path, net, meta):
    """The trained network: float32 master parameters (the bfloat16 values
    the kernels use are their rounding) and how they were made."""
    p = net.read()[0]
    doc = dict(meta, n_params=int(p.size), norm=[float(v) for v in normalisation()],
               box_lo=[float(v) for v in BOX_LO], box_hi=[float(v) for v in BOX_HI],
               params=[float(v) for v in p])
    with open(path, "w") as f:
        json.dump(doc, f, separators=(",", ":"))


def load_params(path=PARAMS_PATH):
    with open(path) as f:
        doc = json.load(f)
    return np.asarray(doc["params"], np.float32), doc


def load_network(path=PARAMS_PATH):
    """The committed trained network as a Surrogate (None if absent)."""
    import os
    if not os.path.exists(path):
        return None, None
    p, doc = load_params(path)
    net = MLP.Mlp(p, np.asarray(doc["norm"], np.float32))
    return Surrogate(net, doc["box_lo"], doc["box_hi"]), doc


def evaluate(sur, fresh, steps, tuning=None, log=None):
    """Relative error of the network against fresh plain runs of `steps`
    steps: all runs, and the runs whose own relative standard error is below
    2 % (where a 5 % error is resolvable)."""
    eta_f, se_f = measure(fresh, steps, tuning=tuning, log=log)
    pred = sur.predict(features([c[2] for c in fresh]))
    rel = np.abs(pred / eta_f - 1.0)
    rel_se = se_f / np.abs(eta_f)
    quiet = rel_se < 0.02
    return {
        "eval_cells": len(fresh), "eval_steps": steps,
        "median_rel_error": float(np.median(rel)),
        "mean_rel_error": float(rel.mean()),
        "median_plain_rel_se": float(np.median(rel_se)),
        "cells_with_plain_se_below_2pct": int(quiet.sum()),
        "mean_rel_error_where_plain_se_below_2pct": float(rel[quiet].mean()) if quiet.any() else None,
        "median_rel_error_where_plain_se_below_2pct":
            float(np.median(rel[quiet])) if quiet.any() else None,
        "frac_within_5pct_where_plain_se_below_2pct":
            float((rel[quiet] <= 0.05).mean()) if quiet.any() else None,
    }, rel, rel_se


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--cells", type=int, default=4096, help="training cells")
    ap.add_argument("--eval-cells", type=int, default=64, help="fresh plain runs for the error")
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--eval-steps", type=int, default=5000,
                    help="steps of the fresh plain runs the error is judged against (the "
                         "training protocol's: the viscosity still relaxes after 5000 steps "
                         "from the initial lattice, so longer runs measure another quantity)")
    ap.add_argument("--eval-shear", type=float, nargs=2, default=[1e-2, 1e-1],
                    help="shear-rate range of a second set of fresh runs (their own standard "
                         "error resolves 5 %% in most)")
    ap.add_argument("--side", type=int, nargs=2, default=[16, 40])
    ap.add_argument("--measure-only", action="store_true")
    ap.add_argument("--range", type=int, nargs=2, default=None,
                    help="with --measure-only: the training cells A..B-1 of the sampler")
    ap.add_argument("--data", default=None, help="npz file written by --measure-only")
    ap.add_argument("--train-from", nargs="*", default=None,
                    help="npz files of measured cells (no measuring)")
    ap.add_argument("--save", default=None, help="write the trained parameters (json)")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--queries", type=int, default=1 << 20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-rel-se", type=float, default=0.1,
                    help="train only on cells whose relative standard error is below this "
                         "(the low-shear cells are dominated by thermal noise)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape (cell = h, 10-step graphs, 4M-particle batches)")
    args = ap.parse_args(argv)
    log = lambda m: print(f"# {m}", file=sys.stderr, flush=True)
    import torch
    torch.cuda.set_device(0)
    kw = dict(side=tuple(args.side), steps=args.steps)
    t0 = time.perf_counter()
    tuning = None
    if args.train_from:
        parts = [np.load(f) for f in args.train_from]
        x = np.concatenate([d["x"] for d in parts]).astype(np.float32)
        eta = np.concatenate([d["eta"] for d in parts])
        se = np.concatenate([d["se"] for d in parts])
        t_meas = float(sum(float(d["seconds"]) for d in parts))
        if not args.no_autotune:
            _, some = W.viscometer_batch(min(args.cells, 512), seed=args.seed, **kw)
            tuning = AT.tune(some, args.steps, log=log)
    else:
        _, cells = W.viscometer_batch(args.cells, seed=args.seed, **kw)
        if args.range:
            cells = cells[args.range[0]:args.range[1]]
        tuning = None if args.no_autotune else AT.tune(cells, args.steps, log=log)
        eta, se = measure(cells, args.steps, tuning=tuning, log=log)
        torch.cuda.synchronize()
        t_meas = time.perf_counter() - t0
        x = features([c[2] for c in cells])
        if args.measure_only:
            np.savez(args.data, x=x, eta=eta, se=se, seconds=t_meas)
            print(json.dumps({"measured": len(cells), "seconds": round(t_meas, 2),
                              "launch_shape": None if tuning is None else
                              {k: tuning[k] for k in ("cell_factor", "graph_steps", "tile")}}),
                  flush=True)
            return None
    ok = (eta > 0) & (se < args.max_rel_se * np.abs(eta))
    y = np.log(np.where(ok, eta, 1.0)).astype(np.float32)
    t0 = time.perf_counter()
    net, hist = train(x[ok], y[ok], epochs=args.epochs, seed=args.seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # fresh plain runs, never seen in training, run longer than the training
    # cells so that most resolve a 5 % error
    _, fresh = W.viscometer_batch(args.eval_cells, seed=args.seed + 999,
                                  **dict(kw, steps=args.eval_steps))
    sur = Surrogate(net, BOX_LO, BOX_HI)
    ev, rel, rel_se = evaluate(sur, fresh, args.eval_steps, tuning=tuning, log=log)
    _, fresh2 = W.viscometer_batch(args.eval_cells, seed=args.seed + 1999,
                                   **dict(kw, steps=args.eval_steps, shear=tuple(args.eval_shear)))
    ev2 = evaluate(sur, fresh2, args.eval_steps, tuning=tuning, log=log)[0]
    ev["eval_high_shear"] = dict(ev2, shear=list(args.eval_shear))
    q = W.mlp_queries(args.queries, seed=args.seed + 7)
    qd = torch.from_numpy(q).cuda()
    net.predict(qd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net.predict(qd)
    torch.cuda.synchronize()
    t_q = (time.perf_counter() - t0) / 10
    res = dict({
        "train_cells": int(x.shape[0]), "steps_per_run": args.steps, "side": args.side,
        "trained_on": int(ok.sum()), "max_rel_se": args.max_rel_se,
        "measure_s": round(t_meas, 2), "train_s": round(t_train, 2),
        "launch_shape": None if tuning is None else
            {k: tuning[k] for k in ("cell_factor", "graph_steps", "tile", "tune_s")},
        "final_train_loss": hist[-1][1],
    }, **ev)
    res.update({
        "queries": args.queries, "query_s": t_q, "queries_per_s": args.queries / t_q,
        "plain_runs_per_s": x.shape[0] / t_meas,
    })
    if args.save:
        save_params(args.save, net, {
            "train_cells": int(x.shape[0]), "trained_on": int(ok.sum()),
            "steps_per_run": args.steps, "side": list(args.side), "seed": args.seed,
            "epochs": args.epochs, "max_rel_se": args.max_rel_se,
            "final_train_loss": float(hist[-1][1])})
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
