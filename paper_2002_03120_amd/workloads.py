"""Seeded synthetic inputs for the SDPD-DEM hot path.

This module only places particles and states physical constants; it holds
none of the method's arithmetic and imports nothing else from the package,
so both the GPU path and the CPU oracle can take their inputs from it.

Every generator returns ``(params, particles, info)``:

* ``params`` -- a plain dict whose keys are the fields of the parameter
  struct of the C ABI (names follow the command-line table of Sec. 3.2 of
  the paper);
* ``particles`` -- numpy arrays in id order: ``id`` (int64), ``type``
  (uint8: 0 fluid, 1 rigid, 2 inner wall, 3 outer wall), ``pos``, ``vel``,
  ``angvel`` (n x 3 float64), ``mass``, ``inertia``, ``radius`` (n float64);
* ``info`` -- counts and the number of steps the workload runs.

Ids are assigned in the order: fluid lattice (x fastest, sites taken by a
rigid particle skipped), rigid particles (placement order), inner walls,
outer walls.  The paper uses no dataset; these boxes stand in for its
validation cases (Sec. 4) at the sizes of the workloads measured here.
"""
from __future__ import annotations

import math

import numpy as np

FLUID, RIGID, INNER_WALL, OUTER_WALL = 0, 1, 2, 3


def base_params(**over) -> dict:
    """Fluid constants of the reverse-Poiseuille box (eta = 0.1, xi = 20 eta/21
    as in Sec. 4.1, alpha = 7, p0 = beta = 1 so that p(rho0) = 0)."""
    eta = 0.1
    p = dict(
        org=[0.0, 0.0, 0.0], L=[20.0, 20.0, 20.0], periodic=[1, 1, 1], noslip=1,
        dx=1.0, h=1.5, rho0=1.0, p0=1.0, alpha=7.0, beta_eos=1.0,
        eta=eta, xi=20.0 * eta / 21.0, kBT=1e-3, dt=1e-3,
        g=[0.0, 0.0, 0.0], f=[0.0, 0.0, 0.0], gravity_type=0, gravity_axis=2,
        coeff_c=1.0, coeff_d=1.0, coeff_r=1.0, coeff_t=1.0,
        # Young modulus picked so that k_n is about 5000 for d = 3 spheres
        E_dem=7881.0, nu_dem=0.3, mu_fric=0.3, dem_damping=1.0,
        mass_fluid=1.0, inertia_fluid=0.1,
        enable_kernel_norm=1, enable_pres_smooth=1, enable_neg_p_clamp=0,
        enable_lub=1, eps_min=0.2, lub_gap_min=0.01,
        itr_start=0, itr_actv_rigid=0, seed=0, max_neighbors=64, max_contacts=16,
        shear_rate=0.0,
    )
    p.update(over)
    return p


def _lattice(nx, ny, nz, dx, org=(0.0, 0.0, 0.0)):
    """Sites (k + 1/2) dx of an nx x ny x nz block, x fastest."""
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1).astype(np.float64)
    pos = (pos + 0.5) * dx + np.asarray(org, dtype=np.float64)
    return pos


def _walls(ncell, periodic, layers, dx, org=(0.0, 0.0, 0.0)):
    """Wall lattice sites around a box of ncell sites per axis: `layers`
    layers on every non-periodic face; layer 1 (touching the box) is the
    inner wall, the others are outer walls.  Returns (pos, type)."""
    lo = [0 if periodic[a] else -layers for a in range(3)]
    hi = [ncell[a] if periodic[a] else ncell[a] + layers for a in range(3)]
    kz, ky, kx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                             np.arange(lo[0], hi[0]), indexing="ij")
    k = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    depth = np.zeros(k.shape[0], dtype=np.int64)
    for a in range(3):
        below = -k[:, a]
        above = k[:, a] - (ncell[a] - 1)
        depth = np.maximum(depth, np.maximum(below, above))
    keep = depth >= 1
    k, depth = k[keep], depth[keep]
    pos = (k.astype(np.float64) + 0.5) * dx + np.asarray(org, dtype=np.float64)
    typ = np.where(depth == 1, INNER_WALL, OUTER_WALL).astype(np.uint8)
    # inner walls first, then outer walls (id order)
    order = np.argsort(typ, kind="stable")
    return pos[order], typ[order]


def _assemble(params, fluid_pos, rigid_pos, rigid_d, ratio, wall_pos, wall_type,
              steps, name):
    rho0, dx = params["rho0"], params["dx"]
    nf, nr, nw = fluid_pos.shape[0], rigid_pos.shape[0], wall_pos.shape[0]
    n = nf + nr + nw
    typ = np.concatenate([np.full(nf, FLUID, np.uint8), np.full(nr, RIGID, np.uint8),
                          wall_type.astype(np.uint8)])
    pos = np.concatenate([fluid_pos, rigid_pos, wall_pos]).astype(np.float64)
    mass = np.full(n, params["mass_fluid"], dtype=np.float64)
    inertia = np.full(n, params["inertia_fluid"], dtype=np.float64)
    radius = np.full(n, 0.5 * dx, dtype=np.float64)
    if nr:
        R = 0.5 * np.asarray(rigid_d, dtype=np.float64) * np.ones(nr)
        vs = 4.0 / 3.0 * math.pi * R ** 3
        ms = ratio * rho0 * vs
        mass[nf:nf + nr] = ms
        inertia[nf:nf + nr] = 0.4 * ms * R ** 2
        radius[nf:nf + nr] = R
    parts = dict(
        id=np.arange(n, dtype=np.int64), type=typ, pos=np.ascontiguousarray(pos),
        vel=np.zeros((n, 3)), angvel=np.zeros((n, 3)), mass=mass, inertia=inertia,
        radius=radius,
    )
    info = dict(name=name, n=n, n_fluid=nf, n_rigid=nr,
                n_inner_wall=int((wall_type == INNER_WALL).sum()),
                n_outer_wall=int((wall_type == OUTER_WALL).sum()),
                n_moving=nf + nr, steps=steps)
    return params, parts, info


def reverse_poiseuille(n_side=(20, 20, 20), dx=1.0, g=1e-3, kBT=1e-3, dt=1e-3,
                       steps=200, seed=0, **over):
    """Fully periodic SDPD box driven by +g along y in the upper half of z
    and -g in the lower half (the reverse-Poiseuille viscometer of Sec. 4.1
    with the 20x20x20 lattice, h = 1.5 dx, eta = 0.1, kT = 1e-3)."""
    nx, ny, nz = n_side
    p = base_params(org=[0.0, 0.0, 0.0], L=[nx * dx, ny * dx, nz * dx],
                    periodic=[1, 1, 1], dx=dx, h=1.5 * dx, kBT=kBT, dt=dt,
                    g=[0.0, g, 0.0], gravity_type=1, gravity_axis=2, seed=seed,
                    mass_fluid=1.0 * dx ** 3, inertia_fluid=0.1 * dx ** 5)
    p.update(over)
    fluid = _lattice(nx, ny, nz, dx)
    return _assemble(p, fluid, np.zeros((0, 3)), 0.0, 0.0, np.zeros((0, 3)),
                     np.zeros(0, np.uint8), steps, "reverse_poiseuille")


def sedimentation(n_fluid=(32, 32, 64), d=8.0, ratio=2.5, center=None, g=2e-5,
                  dt=0.025, steps=20000, layers=3, **over):
    """Single DEM sphere released at rest near the top of a walled fluid box
    (the sedimentation test of Sec. 4.2, moved to the Stokes regime): 3 wall
    layers on all faces, the sphere replaces the lattice site at its
    centre, gravity -z, kT = 0."""
    nx, ny, nz = n_fluid
    dx = 1.0
    if center is None:
        center = ((nx // 2 - 1) + 0.5, (ny // 2 - 1) + 0.5, nz - 8.5)
    p = base_params(org=[0.0, 0.0, 0.0], L=[nx * dx, ny * dx, nz * dx],
                    periodic=[0, 0, 0], kBT=0.0, dt=dt, g=[0.0, 0.0, -g],
                    gravity_type=0)
    p.update(over)
    fluid = _lattice(nx, ny, nz, dx)
    c = np.asarray(center, dtype=np.float64)
    site = np.argmin(((fluid - c) ** 2).sum(axis=1))
    fluid = np.delete(fluid, site, axis=0)
    wp, wt = _walls((nx, ny, nz), (0, 0, 0), layers, dx)
    return _assemble(p, fluid, c[None, :], d, ratio, wp, wt, steps, "sedimentation")


def slurry_channel(interval=0, walls=False, L=(21.0, 41.0, 10.0), dx=0.5, h_over_dx=2.0,
                   kBT=1.0, dt=2e-3, steps=3500, seed=0, layers=3, ratio=2.7,
                   site_volume_fraction=0.55, **over):
    """The reverse-Poiseuille channel of Sec. 4.1 and its slurry version of
    Sec. 4.3 at the paper's constants: box (20, 40, 10), eta = 25,
    xi = 20 eta / 21, rho0 = 3, p0 = beta = 100, no gravity, driving
    acceleration 1.5 along y, +y in the upper half of z and -y in the lower
    half.  Fully periodic (walls=False) or wall-periodic (walls=True: wall
    particles on the z faces, periodic in x and y).

    interval > 0 interleaves rigid particles with the fluid lattice: every
    interval-th site in id order (x fastest) becomes a rigid particle of
    volume site_volume_fraction dx^3 and density ratio `ratio`, so the
    concentration (rigid volume over box volume) is
    site_volume_fraction / interval: 3.67 %, 5.5 % and 11 % at intervals 15,
    10 and 5.  interval = 0 (or -1) places none.

    Spacing, support and thermal energy are not stated in the paper (they
    live in its parameter files): dx = 0.5, h = 2 dx and kBT = 1 here, the
    fluid particle mass rho0 dx^3.  The box is 42 x 82 x 20 sites
    (21 x 41 x 10): spheres of 1.016 dx touch only across faces of sites,
    and with these counts no two face neighbours (periodic wraps included)
    are both interleaved sites at intervals 5, 10 and 15 (at 40 x 80 sites
    intervals 5 and 10 stack the spheres into sheets of overlapping
    spheres, and such runs blow up).  Runs 7 time units in 3500 steps of
    0.002: a sphere's Stokes drag 3 pi eta d relaxes its velocity in
    m_s / (3 pi eta d) = 0.0046, which the step must resolve.  The
    lubrication gap is floored at dx / 8: the explicit step resolves the
    lubrication coefficient 6 pi eta R*^2 / gap only down to about that gap
    at eta = 25."""
    eta = 25.0
    nx, ny, nz = (int(round(L[a] / dx)) for a in range(3))
    periodic = [1, 1, 0 if walls else 1]
    m_f = 3.0 * dx ** 3
    p = base_params(org=[0.0, 0.0, 0.0], L=[nx * dx, ny * dx, nz * dx], periodic=periodic,
                    dx=dx, h=h_over_dx * dx, rho0=3.0, p0=100.0, alpha=7.0, beta_eos=100.0,
                    eta=eta, xi=20.0 * eta / 21.0, kBT=kBT, dt=dt,
                    g=[0.0, 0.0, 0.0], f=[0.0, 1.5, 0.0], gravity_type=1, gravity_axis=2,
                    seed=seed, mass_fluid=m_f, inertia_fluid=0.4 * m_f * (0.5 * dx) ** 2,
                    # stiffness for spheres of about one lattice site
                    E_dem=788.0, lub_gap_min=0.125 * dx)
    p.update(over)
    sites = _lattice(nx, ny, nz, dx)
    rig = np.zeros(sites.shape[0], bool)
    if interval and interval > 0:
        rig[interval - 1::interval] = True
    d = (6.0 * site_volume_fraction / math.pi) ** (1.0 / 3.0) * dx
    if walls:
        wp, wt = _walls((nx, ny, nz), periodic, layers, dx)
    else:
        wp, wt = np.zeros((0, 3)), np.zeros(0, np.uint8)
    p_, parts, info = _assemble(p, sites[~rig], sites[rig], d, ratio, wp, wt, steps,
                                "slurry_channel")
    vol = p["L"][0] * p["L"][1] * p["L"][2]
    nr = int(rig.sum())
    info.update(interval=int(interval or 0), walls=bool(walls), rigid_d=d,
                concentration=nr * math.pi * d ** 3 / 6.0 / vol, D=0.5 * p["L"][2],
                drive=1.5)
    return p_, parts, info


def _rsa(n, lo, hi, d, rng, max_tries=500_000):
    """Random sequential addition of n non-overlapping spheres of diameter d
    with centres uniform in the box [lo, hi]."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    cs = d
    ncell = np.maximum(1, np.floor((hi - lo) / cs).astype(int))
    grid: dict = {}
    out = []
    tries = 0
    batch = 4096
    while len(out) < n:
        cand = lo + rng.random((batch, 3)) * (hi - lo)
        for x in cand:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random sequential addition did not converge")
            c = tuple(np.minimum(((x - lo) / cs).astype(int), ncell - 1))
            ok = True
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dxx in (-1, 0, 1):
                        for y in grid.get((c[0] + dxx, c[1] + dy, c[2] + dz), ()):
                            if ((x - y) ** 2).sum() < d * d:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                grid.setdefault(c, []).append(x)
                out.append(x)
                if len(out) == n:
                    break
    return np.asarray(out)


def dam_break(tank=(256, 64, 192), column=(128, 64, 128), n_rigid=20000, d=3.0,
              ratio=2.5, g=1e-3, c0=5.0, dt=0.005, steps=10000, layers=3,
              kBT=0.0, seed=0, **over):
    """Dam break with rigid particles (Sec. 4.4): a fluid column in one
    corner of a walled tank, DEM spheres placed by seeded random sequential
    addition inside the column, each replacing its nearest fluid site; free
    surface (negative-pressure clamp on), friction 0.3, kT = 0."""
    dx = 1.0
    alpha = 7.0
    p0 = 1.0 * c0 * c0 / alpha
    p = base_params(org=[0.0, 0.0, 0.0], L=[float(t) for t in tank],
                    periodic=[0, 0, 0], kBT=kBT, dt=dt, g=[0.0, 0.0, -g],
                    gravity_type=0, p0=p0, beta_eos=p0, alpha=alpha,
                    enable_neg_p_clamp=1, seed=seed)
    p.update(over)
    fluid = _lattice(*column, dx)
    rng = np.random.default_rng(seed)
    R = 0.5 * d
    if n_rigid:
        rig = _rsa(n_rigid, [R, R, R], [column[0] - R, column[1] - R, column[2] - R], d, rng)
        k = np.clip(np.floor(rig / dx).astype(np.int64), 0, np.asarray(column) - 1)
        sites = (k[:, 2] * column[1] + k[:, 1]) * column[0] + k[:, 0]
        if np.unique(sites).size != sites.size:
            raise RuntimeError("two spheres share a lattice site")
        keep = np.ones(fluid.shape[0], bool)
        keep[sites] = False
        fluid = fluid[keep]
    else:
        rig = np.zeros((0, 3))
    wp, wt = _walls(tank, (0, 0, 0), layers, dx)
    return _assemble(p, fluid, rig, d, ratio, wp, wt, steps, "dam_break")


def shear_cell(n_side=16, phi=0.2, d=4.0, kBT=1e-3, shear_rate=1e-2, ratio=1.0, dt=5e-3,
               seed=0, steps=5000, **over):
    """A periodic Lees-Edwards shear cell (the batched viscometer's unit):
    an n_side^3 fluid lattice with DEM spheres of diameter d on a jittered
    cubic sub-lattice of spacing (V_s/phi)^(1/3) (dense enough for phi up to
    0.4, where random sequential addition would jam), each replacing its
    nearest fluid site.  Velocities follow the linear shear profile
    v_x = shear_rate (z - L/2) plus Maxwellian noise of variance kBT/m; spins
    are shear_rate/2 about y (half the vorticity)."""
    dx = 1.0
    n = int(n_side)
    L = float(n)
    rng = np.random.default_rng(seed)
    p = base_params(org=[0.0, 0.0, 0.0], L=[L, L, L], periodic=[1, 1, 1], kBT=kBT, dt=dt,
                    g=[0.0, 0.0, 0.0], shear_rate=shear_rate, seed=seed)
    p.update(over)
    fluid = _lattice(n, n, n, dx)
    rig = np.zeros((0, 3))
    if phi > 0.0 and d > 0.0:
        vs = math.pi * d ** 3 / 6.0
        a = (vs / phi) ** (1.0 / 3.0)
        m = int(math.floor(L / a))
        if m >= 1:
            a = L / m
            g = (np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"),
                          axis=-1).reshape(-1, 3) + 0.5) * a
            jit = 0.45 * max(a - d, 0.0)
            rig = g + rng.uniform(-jit, jit, size=g.shape)
            k = np.floor(rig / dx).astype(np.int64) % n
            sites = (k[:, 2] * n + k[:, 1]) * n + k[:, 0]
            if np.unique(sites).size != sites.size:
                raise RuntimeError("two spheres share a lattice site")
            keep = np.ones(fluid.shape[0], bool)
            keep[sites] = False
            fluid = fluid[keep]
    params, parts, info = _assemble(p, fluid, rig, d, ratio, np.zeros((0, 3)),
                                    np.zeros(0, np.uint8), steps, "shear_cell")
    z = parts["pos"][:, 2]
    m_ = parts["mass"]
    parts["vel"][:, 0] = shear_rate * (z - 0.5 * L)
    if kBT > 0.0:
        parts["vel"] += rng.normal(size=(z.size, 3)) * np.sqrt(kBT / m_)[:, None]
    parts["angvel"][:, 1] = 0.5 * shear_rate
    info.update(phi=float(rig.shape[0] * math.pi * d ** 3 / 6.0 / L ** 3), d=float(d),
                kBT=float(kBT), shear_rate=float(shear_rate), L=L)
    return params, parts, info


def viscometer_batch(n_cells=256, seed=0, side=(16, 40), phi=(0.0, 0.4), d=(2.0, 6.0),
                     kBT=(5e-4, 5e-3), shear=(1e-3, 1e-1), dt=5e-3, steps=5000, **over):
    """Independent Lees-Edwards shear cells of uneven size for the batched
    viscometer: side ~ U{side}, volume fraction ~ U[phi], sphere diameter
    ~ U[d], kT ~ U[kBT], shear rate log-uniform in [shear].  Returns
    (params shared by all cells, list of per-cell (params, particles, info))."""
    rng = np.random.default_rng(seed)
    cells = []
    for c in range(n_cells):
        L = int(rng.integers(side[0], side[1] + 1))
        ph = float(rng.uniform(*phi))
        dd = float(rng.uniform(*d))
        kt = float(rng.uniform(*kBT))
        gd = float(math.exp(rng.uniform(math.log(shear[0]), math.log(shear[1]))))
        cells.append(shear_cell(L, ph, dd, kt, gd, dt=dt, seed=seed * 1000003 + c, steps=steps,
                                **over))
    shared = dict(cells[0][0]) if cells else base_params(dt=dt)
    return shared, cells


def stack_cells(cells):
    """Concatenate shear cells into one batch: particles with ids offset per
    cell, the box list and the per-particle box index."""
    ids, types, pos, vel, ang, mass, iner, rad, box_of, boxes = ([] for _ in range(10))
    off = 0
    for b, (p, parts, info) in enumerate(cells):
        n = parts["id"].shape[0]
        ids.append(parts["id"] + off)
        for lst, k in ((types, "type"), (pos, "pos"), (vel, "vel"), (ang, "angvel"),
                       (mass, "mass"), (iner, "inertia"), (rad, "radius")):
            lst.append(parts[k])
        box_of.append(np.full(n, b, np.int32))
        boxes.append(dict(org=p["org"], L=p["L"], periodic=p["periodic"],
                          shear_rate=p["shear_rate"], kBT=p["kBT"], seed=p["seed"]))
        off += n
    parts = dict(id=np.concatenate(ids), type=np.concatenate(types), pos=np.concatenate(pos),
                 vel=np.concatenate(vel), angvel=np.concatenate(ang), mass=np.concatenate(mass),
                 inertia=np.concatenate(iner), radius=np.concatenate(rad))
    return parts, boxes, np.concatenate(box_of)


# ---- the viscosity surrogate's inputs -------------------------------------

MLP_LAYERS = (4, 64, 64, 64, 1)


def mlp_param_count(layers=MLP_LAYERS):
    return sum(a * b + b for a, b in zip(layers[:-1], layers[1:]))


def mlp_init(seed=0, layers=MLP_LAYERS):
    """Initial parameters of the surrogate MLP as one flat float32 array in
    the order W1 [in x out] row-major, b1, W2, b2, ...: weights uniform in
    +-sqrt(6 / (fan_in + fan_out)) (Glorot), biases zero.  Seeded random
    numbers only; no arithmetic of the network."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(layers[:-1], layers[1:]):
        lim = math.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def mlp_queries(n, seed=0, phi=(0.0, 0.4), d=(2.0, 6.0), kBT=(5e-4, 5e-3), shear=(1e-3, 1e-1)):
    """Query points (phi, d/dx, kT, log shear rate) uniform over the
    viscometer's sampling box (log-uniform in the shear rate)."""
    rng = np.random.default_rng(seed)
    q = np.empty((n, 4), np.float32)
    q[:, 0] = rng.uniform(*phi, size=n)
    q[:, 1] = rng.uniform(*d, size=n)
    q[:, 2] = rng.uniform(*kBT, size=n)
    q[:, 3] = rng.uniform(math.log(shear[0]), math.log(shear[1]), size=n)
    return q


def periodic_scale(n_side=(256, 256, 128), **over):
    """Scale run: a fully periodic SDPD lattice at density 1 with the
    reverse-Poiseuille constants (2^23 particles at the default size)."""
    return reverse_poiseuille(n_side=n_side, steps=100, **over)


def random_box(n, L, periodic, h=1.5, seed=0, exact_pairs=0, wall=False):
    """Uniformly random fluid positions in a box, for brute-force neighbour
    checks; `exact_pairs` pairs are planted at separation exactly h along an
    axis, and `wall` marks a random tenth of the particles as inner walls."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L, float)
    pos = rng.random((n, 3)) * L
    for k in range(min(exact_pairs, n // 2)):
        a = int(rng.integers(0, 3))
        # dyadic coordinates make the separation exactly h in floating point
        pos[2 * k] = np.floor(pos[2 * k] * 1024.0) / 1024.0
        q = pos[2 * k].copy()
        q[a] = q[a] + h
        if q[a] >= L[a]:
            q[a] = pos[2 * k][a] - h
        pos[2 * k + 1] = q
    p = base_params(org=[0.0, 0.0, 0.0], L=list(L), periodic=list(periodic), h=h)
    typ = np.full(n, FLUID, np.uint8)
    if wall:
        typ[rng.random(n) < 0.1] = INNER_WALL
    parts = dict(id=np.arange(n, dtype=np.int64), type=typ, pos=pos,
                 vel=np.zeros((n, 3)), angvel=np.zeros((n, 3)),
                 mass=np.full(n, p["mass_fluid"]), inertia=np.full(n, p["inertia_fluid"]),
                 radius=np.full(n, 0.5 * p["dx"]))
    info = dict(name="random_box", n=n, n_fluid=n, n_rigid=0, n_moving=n, steps=1)
    return p, parts, info


def perturb(parts, params, jitter=0.1, kT=None, seed=1, types=(FLUID, RIGID),
            spin=False):
    """Jitter the moving particles' positions uniformly by +-jitter*dx
    (seed) and give them Gaussian velocities of variance kT/m (seed + 1),
    and spins of variance kT/I if `spin`.  Returns a new particle dict."""
    out = {k: np.array(v, copy=True) for k, v in parts.items()}
    sel = np.isin(out["type"], np.asarray(types, np.uint8))
    rng = np.random.default_rng(seed)
    dx = params["dx"]
    if jitter:
        out["pos"][sel] += (rng.random((int(sel.sum()), 3)) * 2.0 - 1.0) * jitter * dx
        for a in range(3):
            lo, L = params["org"][a], params["L"][a]
            x = out["pos"][:, a]
            if params["periodic"][a]:
                x[sel] = lo + np.mod(x[sel] - lo, L)
            else:
                x[sel] = np.clip(x[sel], lo, lo + L)
    if kT:
        rng2 = np.random.default_rng(seed + 1)
        m = out["mass"][sel][:, None]
        out["vel"][sel] = rng2.standard_normal((int(sel.sum()), 3)) * np.sqrt(kT / m)
        if spin:
            inert = out["inertia"][sel][:, None]
            out["angvel"][sel] = rng2.standard_normal((int(sel.sum()), 3)) * np.sqrt(kT / inert)
    return out


CONFIGS = {
    "reverse_poiseuille": reverse_poiseuille,
    "sedimentation": sedimentation,
    "dam_break": dam_break,
    "periodic_scale": periodic_scale,
}
