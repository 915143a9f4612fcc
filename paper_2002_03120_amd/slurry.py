"""The reverse-Poiseuille viscometer of Sec. 4.1 and the slurry experiment
of Sec. 4.3, run on the GPU path.

A channel of height Lz = 2D is driven along y by an acceleration g of
opposite sign in its two halves.  With no-slip planes at z = 0, D and 2D
(periodic images or wall particles at z = 0 and 2D, symmetry at the middle)
each half carries the plane Poiseuille profile of Eq. poiseuanasol,
    v(zeta) = s rho g zeta (D - zeta) / (2 mu),   zeta in [0, D],
with s = +1 in the upper half and -1 in the lower; its mean over a half is
Eq. poiseuave, V = rho g D^2 / (12 mu).  The viscosity follows from a
least-squares fit of c = rho g / (2 mu) to both halves at once (the convex
and the concave curve), with rho the mean density of the moving matter
(fluid plus rigid particles: the acceleration drives both).  Wall particles
need not put the no-slip plane exactly on the box face (the inner wall
layer's velocity is integrated like a fluid particle's, Sec. 2.5), so a
second fit leaves that plane free and reports its offset.

Sec. 4.1 compares the fully periodic box with the wall-periodic one (walls
on the z faces); Sec. 4.3 adds rigid particles interleaved with the fluid
lattice at concentrations 3.67, 5.5 and 11 % and reports the viscosity
relative to the particle-free channel.

    python -m paper_2002_03120_amd.slurry
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import sdpdem as S
from . import workloads as W


def half_profile_basis(z, D):
    """(sign, zeta (D - zeta)) of points at heights z in a channel [0, 2D]."""
    z = np.asarray(z, dtype=np.float64)
    upper = z >= D
    zeta = np.where(upper, z - D, z)
    return np.where(upper, 1.0, -1.0), zeta * (D - zeta)


def fit_viscosity(z, v, D, rho, g, weights=None):
    """Least-squares viscosity of a reverse-Poiseuille profile: v(z) samples
    (bin centres z, mean velocities v along the drive) fitted by
    c s(z) zeta (D - zeta) over both halves, mu = rho g / (2 c).  Returns
    (mu, c)."""
    s, phi = half_profile_basis(z, D)
    w = np.ones_like(phi) if weights is None else np.asarray(weights, np.float64)
    c = float(np.sum(w * s * np.asarray(v) * phi) / np.sum(w * phi * phi))
    return rho * g / (2.0 * c), c


def fit_viscosity_slip(z, v, D, rho, g):
    """The same fit with the no-slip plane of the outer faces left free: in
    the lower half v = -c (z + delta)(D - z), zero at z = -delta and at the
    middle (where the antisymmetric drive forces v = 0), mirrored in the
    upper half.  Linear least squares in (c, c delta).  Returns
    (mu, c, delta); delta > 0 puts the plane outside the box (slip)."""
    z = np.asarray(z, dtype=np.float64)
    upper = z >= D
    zeta = np.where(upper, 2.0 * D - z, z)  # distance from the nearer outer face
    s = np.where(upper, 1.0, -1.0)
    A = np.stack([zeta * (D - zeta), D - zeta], axis=1)
    (c, b), *_ = np.linalg.lstsq(A, s * np.asarray(v, np.float64), rcond=None)
    return rho * g / (2.0 * c), float(c), float(b / c)


def mean_half_velocity(c, D):
    """Eq. poiseuave from the fitted profile: V = c D^2 / 6."""
    return c * D * D / 6.0


def run(p, parts, info, steps=None, sample_every=20, nbins=None, cell_factor=0.5,
        block=10, log=None):
    """Run one channel on the GPU and measure its viscosity from the
    velocity profile of the moving particles (mass-weighted mean of v_y per
    z bin) sampled every sample_every steps over the second half of the run.
    The standard error comes from fits to blocks of `block` samples."""
    steps = info["steps"] if steps is None else steps
    typ = parts["type"]
    moving = (typ == W.FLUID) | (typ == W.RIGID)
    mass = parts["mass"][moving]
    Lz, D, g = p["L"][2], info["D"], info["drive"]
    nbins = int(round(Lz / p["dx"])) if nbins is None else nbins
    rho_mix = mass.sum() / (p["L"][0] * p["L"][1] * p["L"][2])
    edges = np.linspace(0.0, Lz, nbins + 1)
    zc = 0.5 * (edges[1:] + edges[:-1])
    sysm = S.System(dict(p, cell_factor=cell_factor), parts)
    t0 = time.perf_counter()
    done = 0
    prof_sum = np.zeros(nbins)
    nsamp = 0
    blocks, cur, ncur = [], np.zeros(nbins), 0
    while done < steps:
        k = min(sample_every, steps - done)
        sysm.step(k)
        done += k
        if done <= steps // 2:
            continue
        x = sysm.read_field("POS")[moving]
        v = sysm.read_field("VEL")[moving]
        b = np.clip(np.floor(x[:, 2] / Lz * nbins).astype(int), 0, nbins - 1)
        mom = np.bincount(b, weights=mass * v[:, 1], minlength=nbins)
        mb = np.bincount(b, weights=mass, minlength=nbins)
        prof = mom / np.maximum(mb, 1e-300)
        prof_sum += prof
        nsamp += 1
        cur += prof
        ncur += 1
        if ncur == block:
            blocks.append(cur / ncur)
            cur, ncur = np.zeros(nbins), 0
    totals = sysm.totals()
    sysm.close()
    wall = time.perf_counter() - t0
    if nsamp == 0:
        raise ValueError("no samples: the run is shorter than two sampling intervals")
    prof = prof_sum / nsamp
    mu, c = fit_viscosity(zc, prof, D, rho_mix, g)
    mu_slip, _, delta = fit_viscosity_slip(zc, prof, D, rho_mix, g)
    cb = np.array([fit_viscosity(zc, pb, D, rho_mix, g)[1] for pb in blocks])
    se_mu = float(mu * cb.std(ddof=1) / math.sqrt(len(cb)) / abs(c)) if len(cb) > 1 else None
    res = dict(mu=float(mu), se_mu=se_mu, c=c, V_rp=mean_half_velocity(c, D),
               mu_fitted_plane=float(mu_slip), slip_delta=delta,
               rho_mix=float(rho_mix), steps=steps, samples=nsamp,
               seconds=round(wall, 3), profile_z=zc.tolist(), profile_vy=prof.tolist(),
               max_speed=float(totals[8]))
    if log:
        log(f"{info['name']} interval {info['interval']} walls {info['walls']}: mu {mu:.3f} "
            f"(se {se_mu if se_mu is None else round(se_mu, 3)}), {wall:.1f} s")
    return res


def experiment(steps=None, intervals=(15, 10, 5), seed=0, log=None, **kw):
    """Sec. 4.1: the particle-free channel fully periodic and wall-periodic;
    Sec. 4.3: the wall-periodic slurry at every interval.  Returns a dict of
    viscosities and their ratios."""
    out = {}
    eta = None
    runs = {}
    for walls in (False, True):
        p, parts, info = W.slurry_channel(0, walls=walls, seed=seed, **kw)
        eta = p["eta"]
        runs[("fluid", walls)] = run(p, parts, info, steps, log=log)
    mp, mw = runs[("fluid", False)]["mu"], runs[("fluid", True)]["mu"]
    out["eta"] = eta
    out["mu_periodic"] = mp
    out["mu_wall_periodic"] = mw
    out["rel_diff_wall_vs_periodic"] = (mw - mp) / mp
    out["se_mu_periodic"] = runs[("fluid", False)]["se_mu"]
    out["se_mu_wall_periodic"] = runs[("fluid", True)]["se_mu"]
    # the same comparison with each run's no-slip plane fitted
    fp, fw = runs[("fluid", False)], runs[("fluid", True)]
    out["mu_periodic_fitted_plane"] = fp["mu_fitted_plane"]
    out["mu_wall_periodic_fitted_plane"] = fw["mu_fitted_plane"]
    out["wall_slip_delta"] = fw["slip_delta"]
    out["periodic_slip_delta"] = fp["slip_delta"]
    out["rel_diff_wall_vs_periodic_fitted_plane"] = (
        (fw["mu_fitted_plane"] - fp["mu_fitted_plane"]) / fp["mu_fitted_plane"])
    slurry = []
    for iv in intervals:
        p, parts, info = W.slurry_channel(iv, walls=True, seed=seed, **kw)
        r = run(p, parts, info, steps, log=log)
        slurry.append(dict(interval=iv, concentration=info["concentration"], mu=r["mu"],
                           se_mu=r["se_mu"], relative_viscosity=r["mu"] / mw,
                           relative_viscosity_fitted_plane=(
                               r["mu_fitted_plane"] / fw["mu_fitted_plane"]),
                           slip_delta=r["slip_delta"],
                           V_rp=r["V_rp"], rho_mix=r["rho_mix"]))
    out["slurry"] = sorted(slurry, key=lambda s: s["concentration"])
    out["profiles"] = {f"{k[0]}_{'wall' if k[1] else 'periodic'}":
                       dict(z=v["profile_z"], vy=v["profile_vy"]) for k, v in runs.items()}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=None, help="steps per run (default 3500)")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    res = experiment(args.steps, seed=args.seed,
                     log=lambda m: print(f"# {m}", file=sys.stderr, flush=True))
    res.pop("profiles")
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
