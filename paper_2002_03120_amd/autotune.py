"""Autotuner of the batched viscometer's launch shape.

Three knobs decide how fast a set of Lees-Edwards shear cells runs on the
GPU; none of them changes what is computed (the neighbour sets are fixed by
the cut-off h, so results move only by FP32 summation order):

* the fluid cell size, cell_factor x h: cells of h or more are searched as
  the 27-cell stencil, smaller ones as the rows and x cells within h of the
  particle (fewer candidate pairs outside the cut-off, more cells to bin and
  more row set-ups);
* the batch tile, the number of particles advanced together by one batched
  system (cells are packed in order up to it): one big batch fills the chip
  best, smaller ones keep the working set in the L2 caches;
* the steps captured per HIP graph (the launch overhead per step), or
  none: eager steps with neighbour-candidate reuse (a skin of h/15; the
  host decides each step whether to search, which a captured graph cannot).

Every candidate is created and timed on the GPU itself over a short sample
of the same cells (graph capture in the warm-up, `sample_steps` timed
steps); the choice minimises the predicted wall time of the whole run,
  sum over batches of (create time + run_steps x step time).
The search is coordinate-wise: the cell size, then the graph length, on the
first batch of the largest tile, then the tile at the chosen pair.

    python -m paper_2002_03120_amd.autotune --cells 256
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import sdpdem as S
from . import workloads as W

CELL_FACTORS = (0.34, 0.5, 0.55, 0.67, 0.75, 1.0, 1.25)
# the first is used while the cell size is tuned; 0: eager steps with
# neighbour-candidate reuse
GRAPH_STEPS = (10, 2, 20, 0)
REUSE_SKIN_H = 1.0 / 15.0  # the skin of the eager shape, as a fraction of h
TILES = (1 << 20, 1 << 21, 1 << 22, 1 << 23)


def split(cells, tile):
    """Consecutive runs of cells with at most `tile` particles each (a cell
    larger than the tile forms a batch of its own)."""
    out, start = [], 0
    while start < len(cells):
        stop, n = start, 0
        while stop < len(cells) and (stop == start or n + cells[stop][2]["n"] <= tile):
            n += cells[stop][2]["n"]
            stop += 1
        out.append((start, stop, n))
        start = stop
    return out


def fits(cells, cell_factor):
    """Whether every periodic cell keeps at least three fluid cells per
    axis at this cell size (the 27-cell stencil needs them)."""
    for p, _parts, _info in cells:
        cs = max(1.0, cell_factor) * p["h"] * (1.0 + 1e-6)
        for a in range(3):
            if p["periodic"][a] and int(p["L"][a] // cs) < 3:
                return False
    return True


def launch_params(p, cell_factor, graph_steps):
    """The parameters of a system at a launch shape: the cell size, and
    for eager steps (graph_steps 0) the candidate skin."""
    skin = REUSE_SKIN_H * p["h"] if graph_steps == 0 else 0.0
    return dict(p, cell_factor=float(cell_factor), skin=skin)


def steps_per_call(graph_steps, steps):
    """The largest whole number of graphs within `steps` (at least one),
    or `steps` itself for eager stepping."""
    if graph_steps == 0:
        return max(1, steps)
    return max(graph_steps, (steps // graph_steps) * graph_steps)


def time_batch(cells, cell_factor, graph_steps, sample_steps, stream):
    """(create seconds, seconds per step) of one batched system of `cells`
    at this cell size and graph length, stress sampling on."""
    import torch
    parts, boxes, box_of = W.stack_cells(cells)
    p = launch_params(cells[0][0], cell_factor, graph_steps)
    stream.synchronize()
    t0 = time.perf_counter()
    g = S.System(p, parts, stream=stream, boxes=boxes, box_of=box_of)
    g.set_stress(True)
    g.set_graph(graph_steps)
    g.step(1)  # first neighbour build
    stream.synchronize()
    t_create = time.perf_counter() - t0
    g.step(graph_steps)  # capture and first replay
    k = steps_per_call(graph_steps, sample_steps)
    stream.synchronize()
    t0 = time.perf_counter()
    g.step(k)
    stream.synchronize()
    t_step = (time.perf_counter() - t0) / k
    g.close()
    del g
    torch.cuda.empty_cache()
    return t_create, t_step


def tune(cells, run_steps, sample_steps=40, cell_factors=CELL_FACTORS,
         graph_steps=GRAPH_STEPS, tiles=TILES, log=None):
    """Pick (cell_factor, graph_steps, tile) for running `cells` for
    `run_steps` steps each, one knob at a time in that order, the others at
    their current choice (graph_steps[0], the largest tile to begin with).
    Returns a dict with the choice, its predicted wall time, that of the
    default shape (cell = h, 10-step graphs, largest tile) when it was among
    the trials, and every trial."""
    import torch
    stream = torch.cuda.Stream()
    t_start = time.perf_counter()
    trials = []
    n_all = sum(c[2]["n"] for c in cells)
    big = max(tiles)

    def trial(cf, gs, tile):
        a, b, n = split(cells, tile)[0]
        tc, ts = time_batch(cells[a:b], cf, gs, sample_steps, stream)
        # the first batch's per-particle rate stands for every batch of the tile
        tw = len(split(cells, tile)) * tc + run_steps * ts * n_all / n
        trials.append(dict(cell_factor=cf, graph_steps=gs, tile=tile, particles=n,
                           create_s=tc, step_ms=ts * 1e3, predicted_s=tw))
        if log:
            log(f"cell {cf:.2f}h graph {gs:2d} tile {tile} ({n} particles): "
                f"{ts * 1e3:.3f} ms/step, predicted {tw:.1f} s")
        return tw

    best = None
    gs0 = graph_steps[0]
    for cf in cell_factors:
        if not fits(cells, cf):
            trials.append(dict(cell_factor=cf, skipped="fewer than 3 cells on a periodic axis"))
            continue
        tw = trial(cf, gs0, big)
        if best is None or tw < best[0]:
            best = (tw, cf, gs0, big)
    if best is None:
        raise ValueError("no cell size fits the cells")
    for gs in graph_steps[1:]:
        tw = trial(best[1], gs, big)
        if tw < best[0]:
            best = (tw, best[1], gs, big)
    for tile in sorted(tiles):
        if tile != big:
            tw = trial(best[1], best[2], tile)
            if tw < best[0]:
                best = (tw, best[1], best[2], tile)
    default = next((t["predicted_s"] for t in trials if t.get("cell_factor") == 1.0
                    and t.get("graph_steps") == 10 and t.get("tile") == big), None)
    return {
        "cell_factor": best[1], "graph_steps": best[2], "tile": best[3],
        "skin": launch_params(cells[0][0], best[1], best[2])["skin"],
        "predicted_s": best[0], "default_predicted_s": default,
        "tune_s": time.perf_counter() - t_start, "trials": trials,
    }


def tune_system(p, parts, sample_steps=20, cell_factors=CELL_FACTORS, log=None):
    """The cell size of one plain system (the dam break, say): each
    candidate is created and run for sample_steps steps after one warm-up
    step, eager on the default stream; the fastest step wins.  Returns a
    dict with the choice and the trials."""
    import torch
    trials = []
    best = None
    for cf in cell_factors:
        if not fits([(p, None, None)], cf):
            trials.append(dict(cell_factor=cf, skipped="fewer than 3 cells on a periodic axis"))
            continue
        g = S.System(dict(p, cell_factor=float(cf)), parts)
        g.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(sample_steps)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / sample_steps
        g.close()
        del g
        torch.cuda.empty_cache()
        trials.append(dict(cell_factor=cf, step_ms=ts * 1e3))
        if log:
            log(f"cell {cf:.2f}h: {ts * 1e3:.3f} ms/step")
        if best is None or ts < best[0]:
            best = (ts, cf)
    if best is None:
        raise ValueError("no cell size fits the box")
    return {"cell_factor": best[1], "step_ms": best[0] * 1e3, "trials": trials}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--steps", type=int, default=5000, help="steps per run")
    ap.add_argument("--sample-steps", type=int, default=40)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    _, cells = W.viscometer_batch(args.cells, seed=args.seed, steps=args.steps)
    res = tune(cells, args.steps, args.sample_steps,
               log=lambda m: print(f"# {m}", file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
