"""Throughput of the SDPD-DEM hot path on one MI355X.

Workload: the dam break with rigid particles at 1M moving particles
(1,028,576 SDPD fluid + 20,000 DEM spheres of diameter 3dx, 485,592 wall
particles, 1,534,168 in all), seeded synthetic inputs.  A step is one
iteration of Algorithm 1: two velocity-Verlet passes, each running the
whole force evaluation of Algorithm 2, with the cell sort, neighbour
build, density and pressure smoothing once per step.

Prints one JSON line: particle-steps/s of the moving particles, the
roofline of the dominant kernel (the SDPD pair-force kernel), measured with
HIP events on its launch stream over the timed region, and the FP64 CPU
oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# the pair kernel's launches timed by HIP events: one in seven (odd, so the
# timed launches alternate between the two passes of a step, whose pair
# kernels differ: pass 1 shares the chip with the contacts)
PROF_EVERY = 7
# plain (unpacked) VALU issue: 256 CUs x 64 lanes x 2.4 GHz, one op per lane-cycle
VALU_PEAK_GOPS = 256 * 64 * 2.4


def pair_kernel_bytes(n, n_act, nnz_act, noise):
    """Algorithmic HBM bytes of one launch of the pair-force kernel: every
    particle's type and its 9 FP32 outputs; for each fluid/inner-wall
    particle its own FP64 position, the two FP32 pair records, its row
    length and its neighbour indices (plus its id with noise).  Neighbour
    records themselves come from cache and are not counted."""
    return n * (1 + 36) + n_act * (32 + 16 + 16 + 4 + (4 if noise else 0)) + 4 * nnz_act


# device helpers the pair kernel calls (hashed with it; the rest of their
# header does not change the kernel)
PAIR_KERNEL_HELPERS = ("xcd_tid", "logical_block", "blk_box", "geo_of", "min_img_box",
                       "min_img_fast", "load_pr", "philox10", "u01", "pair_normals")


def _function_text(src, name):
    """The definition of a __device__ function `name` in `src`, from its
    declaration line to the brace that closes its body."""
    import re
    m = re.search(r"^__device__[^\n]*\b" + re.escape(name) + r"\(", src, flags=re.M)
    if not m:
        raise KeyError(name)
    i = src.index("{", m.end())
    depth = 0
    for k in range(i, len(src)):
        if src[k] == "{":
            depth += 1
        elif src[k] == "}":
            depth -= 1
            if depth == 0:
                return src[m.start():k + 1]
    raise KeyError(name)


def pair_kernel_sha256():
    """Hash of what the pair kernel is made of: its own source (the pair-force
    section of sdpdem_neighbors.hip to the end of its launcher), the device
    helpers it calls and the pair record it loads.  Counter figures taken
    with other sources are not used."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2002_03120_amd", "csrc")
    nb = open(os.path.join(csrc, "sdpdem_neighbors.hip")).read()
    a = nb.index("// (a5) SDPD+a pair forces")
    b = nb.index("}  // namespace sdpdem", a)
    dev = open(os.path.join(csrc, "sdpdem_device.h")).read()
    internal = open(os.path.join(csrc, "sdpdem_internal.h")).read()
    c = internal.index("struct __align__(64) PR {")
    e = internal.index("static_assert(sizeof(PR)", c)
    h = hashlib.sha256()
    h.update(nb[a:b].encode())
    for name in PAIR_KERNEL_HELPERS:
        h.update(_function_text(dev, name).encode())
    h.update(internal[c:e].encode())
    return h.hexdigest()


def profiled_counters(name="fluid_forces_dam_break_pmc.md"):
    """Counter figures of the pair kernel from a committed rocprofv3 summary
    in profiles/ (its machine-readable block).  Returned only while the
    kernel sources hash to the value recorded with the counters (a changed
    kernel invalidates them); otherwise None."""
    import re
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(re.findall(r"^\s{4}(\w+): (\S+)\s*$", open(path).read(), flags=re.M))
    if kv.get("source_sha256") != pair_kernel_sha256():
        return None
    return {k: float(v) for k, v in kv.items() if k not in ("kernel", "source_sha256")}


def viscometer_leg(k_steps, n_cells=256, run_steps=5000, graph_steps=10, tune=True):
    """Batched viscometer: the 256 Lees-Edwards shear cells of uneven size
    advanced together (one launch per kernel for all cells of a batch)
    against the same cells run one after another as plain systems.  All run
    on a side stream with the step loop replayed from captured HIP graphs and
    stress sampling on; each system is timed over k_steps steps after a
    warm-up that includes the capture; runs/hr extrapolates to run_steps
    steps per run.  The batched figure is taken twice: at the default launch
    shape (cell = h, graph_steps steps per graph, all cells in one batch) and
    at the shape the autotuner picks (its own trials are not timed here;
    graph length 0 there means eager steps with neighbour-candidate reuse,
    timed over 3 k_steps steps)."""
    import torch

    from paper_2002_03120_amd import autotune as AT
    from paper_2002_03120_amd import sdpdem as S
    from paper_2002_03120_amd import workloads as W

    st = torch.cuda.Stream()

    def timed(p, parts, cell_factor=1.0, gs=graph_steps, **kw):
        # eager steps with candidate reuse (graph length 0) search every few
        # dozen steps: they are timed over three times as many steps
        k = AT.steps_per_call(gs, k_steps if gs else 3 * k_steps)
        p = AT.launch_params(p, cell_factor, gs)
        g = S.System(p, parts, stream=st, **kw)
        g.set_stress(True)
        g.set_graph(gs)
        g.step(1 + gs)  # first build, capture, one replay
        st.synchronize()
        t0 = time.perf_counter()
        g.step(k)
        st.synchronize()
        t = (time.perf_counter() - t0) / k
        g.close()
        del g
        torch.cuda.empty_cache()
        return t

    def batched(cs, cell_factor=1.0, gs=graph_steps):
        parts, boxes, box_of = W.stack_cells(cs)
        return timed(cs[0][0], parts, cell_factor, gs, boxes=boxes, box_of=box_of)

    shared, cells = W.viscometer_batch(n_cells, seed=0, steps=run_steps)
    n_all = sum(c[2]["n"] for c in cells)
    t_batch = batched(cells)
    out = {}
    if tune:
        tun = AT.tune(cells, run_steps)
        t_tuned = sum(batched(cells[a:b], tun["cell_factor"], tun["graph_steps"])
                      for a, b, _n in AT.split(cells, tun["tile"]))
        out["autotuned"] = {
            "cell_factor": tun["cell_factor"], "graph_steps": tun["graph_steps"],
            "skin": round(tun["skin"], 4),
            "tile_particles": tun["tile"], "tune_s": round(tun["tune_s"], 2),
            "trials": len(tun["trials"]),
            "batched_ms_per_step": round(t_tuned * 1e3, 3),
            "batched_runs_per_hour": round(n_cells / (t_tuned * run_steps) * 3600.0, 1),
        }
    t_cells = [timed(p, pp) for p, pp, _info in cells]
    t_plain = sum(t_cells)
    rb = n_cells / (t_batch * run_steps) * 3600.0
    rp = n_cells / (t_plain * run_steps) * 3600.0
    res = {
        "cells": n_cells, "particles": n_all, "steps_per_run": run_steps,
        "batched_runs_per_hour": round(rb, 1), "plain_runs_per_hour": round(rp, 1),
        "speedup": round(rb / rp, 2),
        "batched_ms_per_step": round(t_batch * 1e3, 3),
        "plain_ms_per_step_all_cells": round(t_plain * 1e3, 3),
        "batched_particle_steps_per_s": round(n_all / t_batch, 1),
        "graph_steps": graph_steps,
        "sample": f"{k_steps} timed steps per system after a warm-up of 1 + graph length "
                  f"steps (graph capture included), extrapolated to {run_steps} steps per run",
    }
    if "autotuned" in out:
        res["autotuned"] = out["autotuned"]
        res["autotuned"]["speedup_vs_plain"] = round(out["autotuned"]["batched_runs_per_hour"] / rp, 2)
        # the plain runs at their own best too: each cell alone at the tuned
        # cell size and step mode as well, the faster of the two shapes kept
        # per cell, so that the gain above is the batching's, not the tuning's
        t_best = sum(min(t0, timed(p, pp, tun["cell_factor"], tun["graph_steps"]))
                     for (p, pp, _info), t0 in zip(cells, t_cells))
        rbest = n_cells / (t_best * run_steps) * 3600.0
        res["autotuned"]["plain_best_runs_per_hour"] = round(rbest, 1)
        res["autotuned"]["speedup_vs_best_plain"] = round(
            out["autotuned"]["batched_runs_per_hour"] / rbest, 2)
    return res


def surrogate_leg(n_cells=64, steps=5000, seed=1999, shear=(1e-2, 1e-1)):
    """The committed viscosity surrogate (trained on 4096 batched-viscometer
    cells of the batched-viscometer sampling, sides 16-40, 5000 steps) judged
    against fresh plain runs of the same protocol: n_cells cells (the same
    sampler, shear rates in `shear`, another seed), run batched on the GPU;
    the network's relative error against each run's measured viscosity,
    also on the runs whose own standard error is below 2 %; and the rate of
    network answers against plain runs."""
    import numpy as np
    import torch

    from paper_2002_03120_amd import surrogate as SG
    from paper_2002_03120_amd import workloads as W
    sur, doc = SG.load_network()
    if sur is None:
        return None
    _, fresh = W.viscometer_batch(n_cells, seed=seed, side=tuple(doc["side"]), steps=steps,
                                  shear=shear)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, rel, rel_se = SG.evaluate(sur, fresh, steps, tuning={"cell_factor": 0.5,
                                                              "graph_steps": 2,
                                                              "tile": 8388608})
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    q = torch.from_numpy(W.mlp_queries(1 << 20, seed=7)).cuda()
    sur.net.predict(q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        sur.net.predict(q)
    torch.cuda.synchronize()
    t_q = (time.perf_counter() - t0) / 10
    flop = 2 * (4 * 64 + 64 * 64 + 64 * 64 + 64) * (1 << 20)
    ev.update({
        "shear": list(shear), "trained_on": doc["trained_on"], "train_cells": doc["train_cells"],
        "plain_runs_per_s": round(n_cells / t_plain, 2),
        "network_answers_per_s": round((1 << 20) / t_q, 1),
        "gain_answers_per_plain_run": round((1 << 20) / t_q / (n_cells / t_plain), 1),
        "inference_roofline": {"bound": "mfma", "achieved": round(flop / t_q / 1e12, 2),
                               "unit": "TFLOP/s", "peak_bf16_mfma": 2500.0,
                               "frac_bf16_mfma": round(flop / t_q / 2.5e15, 4)},
    })
    return ev


def scale_leg(steps, cell_factor, skin, warmup=2):
    """The scale run: a fully periodic SDPD lattice of 256 x 256 x 128 =
    8,388,608 particles (the reverse-Poiseuille constants, kT = 1e-3, so the
    thermal pair forces are on), timed over `steps` eager steps after
    `warmup`, with neighbour-candidate reuse at `skin` as in the main figure
    (and the same steps searching after every drift beside it); the pair
    kernel timed by HIP events as in the main figure."""
    import torch

    from paper_2002_03120_amd import sdpdem as S
    from paper_2002_03120_amd import workloads as W

    p, parts, info = W.periodic_scale()

    def timed(sk, profile):
        g = S.System(dict(p, cell_factor=cell_factor, skin=sk), parts)
        g.step(warmup)
        if profile:
            g.set_profiling("fluid_forces", every=PROF_EVERY)
        inf0 = g.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        k = g.kernel_time() if profile else (0.0, 0)
        inf = g.info()
        g.close()
        del g
        torch.cuda.empty_cache()
        return wall, k, inf, inf0

    wall, (k_ms, k_launches), inf, inf0 = timed(skin, True)
    nnz = int(inf[9])
    n = int(info["n"])
    k_avg_s = k_ms / max(k_launches, 1) / 1e3
    res = {
        "particles": n, "steps": steps, "warmup": warmup, "kT": p["kBT"],
        "cell_factor": cell_factor, "skin": skin,
        "ms_per_step": round(wall / steps * 1e3, 4),
        "particle_steps_per_s": round(n * steps / wall, 1),
        "pair_interactions_per_s": round(2 * nnz * steps / wall, 1),
        "pair_kernel_ms": round(k_avg_s * 1e3, 4),
        "pair_slots": nnz,
        "neighbour_searches": int(inf[13] - inf0[13]),
        "lists_from_candidates": int(inf[14] - inf0[14]),
    }
    if skin > 0:
        wall0 = timed(0.0, False)[0]
        res["ms_per_step_without_reuse"] = round(wall0 / steps * 1e3, 4)
    # With thermal noise the pair kernel is bound by vector-ALU issue: its
    # roofline is VALU lane-instructions per second against the plain issue
    # peak, the instructions per neighbour slot taken from the committed
    # counter run (SQ_INSTS_VALU x 64 / slots) while the sources match it.
    prof = profiled_counters("fluid_forces_noise_scale_pmc.md")
    if prof and "valu_lane_instr_per_slot" in prof:
        achieved = prof["valu_lane_instr_per_slot"] * nnz / k_avg_s / 1e9
        res["roofline"] = {
            "kernel": "fluid_forces (thermal)", "bound": "alu", "unit": "G lane-instr/s",
            "achieved": round(achieved, 1), "peak": VALU_PEAK_GOPS,
            "frac": round(achieved / VALU_PEAK_GOPS, 4),
            "instr_per_slot": prof["valu_lane_instr_per_slot"],
            # measured HBM bytes per launch (FETCH_SIZE, WRITE_SIZE), profiles/
            "traffic": round(prof["traffic_bytes_per_launch"]),
            "hbm_frac_from_traffic": round(prof["traffic_bytes_per_launch"] / k_avg_s / 1e9
                                           / HBM_PEAK_GBS, 4),
            "slots_per_launch": nnz, "avg_launch_ms": round(k_avg_s * 1e3, 4),
            "valu_busy_counter": prof.get("valu_busy"),
        }
    return res


def measured_peaks():
    """The chip's measured plain-FMA issue rates (FP32 and FP64, 8 chains of
    dependent fused multiply-adds per thread, unpacked) and device copy
    bandwidth (2 GiB, read + write), from the benchmark's helper library."""
    import ctypes

    import torch

    from paper_2002_03120_amd import build as B
    if not os.path.exists(B.PEAKS_LIB):
        return None
    L = ctypes.CDLL(B.PEAKS_LIB)
    L.sdpdem_peak_fma.restype = ctypes.c_double
    L.sdpdem_peak_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p]
    L.sdpdem_peak_copy.restype = ctypes.c_double
    L.sdpdem_peak_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p]
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks = 256 * 32
    out = torch.empty(blocks, dtype=torch.float64, device="cuda")
    f32 = L.sdpdem_peak_fma(0, blocks, 4096, ctypes.c_void_p(out.data_ptr()), st)
    f64 = L.sdpdem_peak_fma(1, blocks, 2048, ctypes.c_void_p(out.data_ptr()), st)
    nbytes = 2 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    cp = L.sdpdem_peak_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                            nbytes, st)
    torch.cuda.synchronize()
    del src, dst, out
    torch.cuda.empty_cache()
    return {"fp32_fma_lane_ops_per_s": round(f32, 1), "fp64_fma_lane_ops_per_s": round(f64, 1),
            "copy_bytes_per_s": round(cp, 1),
            "note": "8 chains of dependent unpacked FMAs per thread, 8192 x 256 threads; "
                    "a 2 GiB device copy (read + write bytes)"}


def window_leg(sysm, p, start_step, steps, n_moving):
    """A timing window later in the dam break: the system is advanced
    (untimed) to start_step, then `steps` steps are timed; the neighbour
    slots per active particle show how the collapse changes the work."""
    import torch
    cur = sysm.current_step
    if start_step > cur:
        sysm.step(start_step - cur)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    inf = sysm.info()
    tot = sysm.totals()
    return {"from_step": start_step, "steps": steps, "ms_per_step": round(wall / steps * 1e3, 4),
            "moving_particle_steps_per_s": round(n_moving * steps / wall, 1),
            "pair_slots": int(inf[9]), "max_speed": round(float(tot[8]), 4),
            "time": round(start_step * p["dt"], 3)}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo), with lscpu's
    family / model / stepping numbers (a virtual machine may report only a
    generic name)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {}
        for ln in out.splitlines():
            if ":" in ln:
                k, v = ln.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if "Model name" in f:
            ids = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if k in f)
            return f["Model name"] + (f" ({ids})" if ids else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                        None)
    except OSError:
        return None


def eager_ms_per_step(p, parts, steps, warmup):
    """The same workload and steps with other parameters (the eager step
    loop on the caller's stream, as in the headline figure)."""
    import torch

    from paper_2002_03120_amd import sdpdem as S

    g = S.System(p, parts)
    g.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    del g
    torch.cuda.empty_cache()
    return t * 1e3


def graph_ms_per_step(p, parts, steps, graph_steps=10):
    """The same workload with its step loop replayed from captured graphs
    (the same neighbour sets; every replayed step searches the cell grid,
    since no host decision can be made inside a graph); reported beside the
    eager figure."""
    import torch

    from paper_2002_03120_amd import sdpdem as S

    st = torch.cuda.Stream()
    g = S.System(p, parts, stream=st)
    g.set_graph(graph_steps)
    g.step(1 + graph_steps)
    st.synchronize()
    steps = max(graph_steps, (steps // graph_steps) * graph_steps)
    t0 = time.perf_counter()
    g.step(steps)
    st.synchronize()
    t = (time.perf_counter() - t0) / steps
    del g
    return t * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--kT", type=float, default=0.0, help="thermal energy (0: the dam break as defined)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the CPU-oracle sample (0 disables it)")
    ap.add_argument("--small", action="store_true", help="a small tank, for quick checks")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    ap.add_argument("--cell-factor", type=float, default=0.55,
                    help="fluid cell size in units of h; the default is the fastest of a sweep "
                         "over 0.5-0.75 h with candidate reuse at the default skin, 0 runs the "
                         "tuner (without reuse) before the timed region")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="steps per captured graph for the graph-replay figure (0: skip)")
    ap.add_argument("--scale-steps", type=int, default=20,
                    help="timed steps of the 8,388,608-particle periodic scale run (0: skip)")
    ap.add_argument("--viscometer-steps", type=int, default=20,
                    help="timed steps per configuration of the batched-viscometer leg (0: skip)")
    ap.add_argument("--skin", type=float, default=0.1,
                    help="neighbour-candidate margin of the dam break and the scale box (0: sort "
                         "and search after every drift); "
                         "the default, h/15, is the fastest of 0.05 h, h/15, 0.1 h, 0.15 h, "
                         "0.2 h here")
    ap.add_argument("--surrogate-cells", type=int, default=64,
                    help="fresh plain runs the committed surrogate is judged against (0: skip)")
    ap.add_argument("--window-step", type=int, default=2000,
                    help="also time --window-steps steps from this step of the collapse (0: skip)")
    ap.add_argument("--window-steps", type=int, default=20)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; a run over several GPUs "
                                   "(slab decomposition with halo exchange) is not implemented",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_03120_amd import sdpdem as S
    from paper_2002_03120_amd import workloads as W

    torch.cuda.set_device(0)
    peaks = measured_peaks()
    if args.calibrate_copy_mib:
        src = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.small:
        p, parts, info = W.dam_break(tank=(64, 32, 48), column=(32, 32, 32), n_rigid=600,
                                     kBT=args.kT)
    else:
        p, parts, info = W.dam_break(kBT=args.kT)
    print(f"# workload {info}", file=sys.stderr, flush=True)
    tuned = None
    if args.cell_factor <= 0.0:
        from paper_2002_03120_amd import autotune as AT
        tuned = AT.tune_system(p, parts, log=lambda m: print(f"# {m}", file=sys.stderr, flush=True))
        args.cell_factor = tuned["cell_factor"]
    pg = dict(p, cell_factor=args.cell_factor, skin=args.skin)  # the GPU system's parameters
    sysm = S.System(pg, parts)
    sysm.step(args.warmup)
    torch.cuda.synchronize()
    inf0 = sysm.info()
    noise = args.kT > 0

    # timed region: exactly `steps` steps, the pair kernel timed by events
    # on the first of every PROF_EVERY launches (the timing events stall the
    # stream a little; sampling keeps the step time close to untimed runs)
    sysm.set_profiling("fluid_forces", every=PROF_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysm.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = sysm.kernel_time()
    sysm.set_profiling("none")
    wall = t1 - t0

    inf = sysm.info()
    typ = parts["type"]
    n = int(info["n"])
    n_act = int(((typ == W.FLUID) | (typ == W.INNER_WALL)).sum())
    nnz = int(inf[9])
    value = info["n_moving"] * args.steps / wall
    pair_rate = 2 * nnz * args.steps / wall
    k_avg_s = (k_ms / max(k_launches, 1)) / 1e3
    kbytes = pair_kernel_bytes(n, n_act, nnz, noise)
    achieved = kbytes / k_avg_s / 1e9
    prof = profiled_counters() if not noise else None
    roof = {
        "kernel": "fluid_forces",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        # measured HBM bytes per launch (rocprofv3 counters, profiles/)
        "traffic": round(prof["traffic_bytes_per_launch"]) if prof else None,
        "avg_launch_ms": round(k_avg_s * 1e3, 4),
        "launches": k_launches,
        "timed_every": PROF_EVERY,
        "bytes_per_launch": kbytes,
    }
    if prof:
        roof["valu_busy"] = prof["valu_busy"]
        roof["valu_lane_use"] = prof["lane_use"]
        # the unit the divergent gathers keep busy: texture addressing, from
        # the same counter profile
        if "ta_busy" in prof:
            roof["ta_busy"] = prof["ta_busy"]
    if prof:
        # the same fraction from the measured HBM bytes of the counter
        # profile (re-fetched partner records included) instead of the
        # algorithmic ones
        roof["frac_from_traffic"] = round(prof["traffic_bytes_per_launch"] / k_avg_s / 1e9
                                          / HBM_PEAK_GBS, 4)
    if peaks and peaks["copy_bytes_per_s"] > 0:
        roof["frac_of_measured_copy"] = round(achieved * 1e9 / peaks["copy_bytes_per_s"], 4)
    tot = sysm.totals()
    status_after = {"max_speed": float(tot[8]), "rho_min": float(tot[9]), "rho_max": float(tot[10])}
    slots_first = nnz
    windows = [{"from_step": args.warmup, "steps": args.steps,
                "ms_per_step": round(wall / args.steps * 1e3, 4), "pair_slots": slots_first,
                "note": "the headline window above"}]
    if args.window_step > 0 and args.window_steps > 0:
        windows.append(window_leg(sysm, p, max(args.window_step, args.warmup + args.steps),
                                  args.window_steps, info["n_moving"]))
    result = {
        "metric": "particle-steps/s at 1M SDPD+20k DEM",
        "value": round(value, 1),
        "unit": "moving-particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 pair forces, fp64 state",
        "data": "synthetic",
        "config": {
            "workload": "dam break with rigid particles" + (" (small)" if args.small else ""),
            "n_fluid": info["n_fluid"], "n_rigid": info["n_rigid"],
            "n_wall": info["n_inner_wall"] + info["n_outer_wall"], "n_total": n,
            "kT": args.kT, "dt": p["dt"], "h": p["h"], "cell_factor": args.cell_factor,
            "skin": args.skin,
        },
        "pair_interactions_per_s": round(pair_rate, 1),
        # cell-grid searches (sort + search) and list builds from the
        # candidates of an earlier search in the timed steps (skin > 0)
        "neighbour_searches": int(inf[13] - inf0[13]),
        "lists_from_candidates": int(inf[14] - inf0[14]),
        "cell_size_trials": None if tuned is None else
            {f"{t['cell_factor']}h": round(t["step_ms"], 4) for t in tuned["trials"] if "step_ms" in t},
        "roofline": roof,
        "measured_peaks": peaks,
        "status_after": status_after,
        "windows": windows,
    }

    del sysm
    torch.cuda.empty_cache()
    if args.skin > 0:
        # the same steps with every list taken from a fresh search
        result["ms_per_step_without_reuse"] = round(
            eager_ms_per_step(dict(pg, skin=0.0), parts, args.steps, args.warmup), 4)
    if args.graph_steps > 0:
        result["ms_per_step_graph"] = round(graph_ms_per_step(pg, parts, args.steps,
                                                              args.graph_steps), 4)
    if args.scale_steps > 0:
        result["scale"] = scale_leg(args.scale_steps, args.cell_factor, args.skin)
    if args.viscometer_steps > 0:
        result["viscometer"] = viscometer_leg(args.viscometer_steps)
    if args.surrogate_cells > 0:
        result["surrogate"] = surrogate_leg(args.surrogate_cells)

    if args.cpu_seconds > 0:
        from oracle import oracle as O
        O.build()
        o = O.Oracle(p, parts)
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        more = max(0, int(args.cpu_seconds / max(one, 1e-9)) - 1)
        more = min(more, 50)
        t0 = time.perf_counter()
        if more:
            o.step(more)
        t_more = time.perf_counter() - t0
        steps_cpu = 1 + more
        t_cpu = one + t_more
        cores = O.num_threads()
        # the same oracle on one core, one step further on
        O.set_num_threads(1)
        t0 = time.perf_counter()
        o.step(1)
        t_one_core = time.perf_counter() - t0
        O.set_num_threads(cores)
        del o
        # the reverse-Poiseuille box (8,000 particles, 200 steps) in full
        pc, partsc, infoc = W.reverse_poiseuille()
        oc = O.Oracle(pc, partsc)
        t0 = time.perf_counter()
        oc.step(infoc["steps"])
        t_c1 = time.perf_counter() - t0
        del oc
        model = cpu_model()
        result["cpu_baseline"] = {
            "value": round(info["n_moving"] * steps_cpu / t_cpu, 1),
            "unit": "moving-particle-steps/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"{steps_cpu} step(s) of the same workload from its initial state "
                      f"({t_cpu:.1f} s, FP64 oracle, OpenMP)",
            "one_core_value": round(info["n_moving"] / t_one_core, 1),
            "one_core_sample": f"the next step on one thread ({t_one_core:.1f} s)",
            "cpu_model": model,
            "reverse_poiseuille_full": {
                "particles": int(infoc["n"]), "steps": int(infoc["steps"]),
                "seconds": round(t_c1, 2),
                "particle_steps_per_s": round(infoc["n"] * infoc["steps"] / t_c1, 1),
                "cores": cores},
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
