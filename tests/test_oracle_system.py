"""System-level pins of the oracle: conservation laws, the Hamiltonian
structure of the conservative force, equipartition, Archimedes, Stokes drag,
the action/reaction balance of the coupling, velocity Verlet, the boundary
treatment, error codes, restart and thread-count invariance."""
import math

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W


def _fluid_box(n=8, kT=1e-3, jitter=0.15, seed=1, **over):
    p, parts, info = W.reverse_poiseuille(n_side=(n, n, n), kBT=kT, g=0.0, **over)
    parts = W.perturb(parts, p, jitter=jitter, kT=max(kT, 1e-4), seed=seed, spin=True)
    return p, parts


def test_pair_forces_conserve_momentum(oracle_lib):
    p, parts = _fluid_box()
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    F = o.read_field("F_SDPD")
    scale = o.read_field("F_SDPD_ABS").sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-14 * scale
    P0 = o.totals()[:3]
    o.step(30)
    assert np.abs(o.totals()[:3] - P0).max() < 1e-13 * scale * 30 * p["dt"]


def _energy(oracle_lib, o, p):
    """Kinetic energy plus U/C_W with U = sum_i m u(rho_i), du/drho = p/rho^2."""
    tot = o.totals()
    rho = o.read_field("DENS")
    a, p0, b, r0 = p["alpha"], p["p0"], p["beta_eos"], p["rho0"]
    u = p0 * rho ** (a - 1) / ((a - 1) * r0 ** a) + b / rho
    cw = r0 / (p["mass_fluid"] * oracle_lib.lattice_w_sum(p["h"], p["dx"]))
    return tot[6] + p["mass_fluid"] * u.sum() / cw


def test_conservative_force_is_hamiltonian(oracle_lib):
    """With only F^C, no smoothing: E = KE + U/C_W is conserved, with a
    velocity-Verlet error that falls as dt^2."""
    drifts = []
    for dt in (2e-3, 1e-3):
        p, parts = _fluid_box(n=7, kT=0.0, jitter=0.2, seed=4, coeff_d=0.0, coeff_r=0.0,
                              coeff_t=0.0, enable_pres_smooth=0, dt=dt)
        parts["vel"] = np.random.default_rng(5).standard_normal(parts["vel"].shape) * 0.05
        o = oracle_lib.Oracle(p, parts)
        o.compute_forces()
        e0 = _energy(oracle_lib, o, p)
        ke0 = o.totals()[6]
        es = []
        for k in range(int(round(0.4 / dt))):
            o.step(1)
            o.compute_forces()
            es.append(_energy(oracle_lib, o, p))
        drifts.append(np.max(np.abs(np.asarray(es) - e0)) / ke0)
    assert drifts[0] < 5e-4
    # second-order integrator: halving dt cuts the energy error 4x; a wrong
    # force (sign, factor, missing term) leaves an error that does not shrink
    assert 3.5 < drifts[0] / drifts[1] < 4.5


def test_equipartition_translational(oracle_lib):
    """Periodic box at kT: (1/3) <m v^2> -> kT.  The rotational coupling is
    switched off so the translational dynamics satisfy the FDT alone."""
    kT = 1e-3
    p, parts = _fluid_box(n=6, kT=kT, jitter=0.05, seed=7, coeff_r=0.0, dt=5e-3)
    o = oracle_lib.Oracle(p, parts)
    o.step(400)
    temps = []
    n = parts["id"].shape[0]
    for k in range(60):
        o.step(40)
        temps.append(2.0 * o.totals()[6] / (3.0 * (n - 1)))
    t = np.mean(temps)
    assert abs(t / kT - 1.0) < 0.06, t / kT


def test_archimedes_in_hydrostatic_equilibrium(oracle_lib):
    """Relax a periodic column under opposite body forces in its two halves
    to rest; a sphere put in place of one fluid particle then feels
    F^PG = -rho0 V_s g_eff (buoyancy) from Eq. F_fpi_PG."""
    g = 0.01
    # a positive background pressure (beta = 0) keeps the stretched half of
    # the column free of the SPH tensile instability
    p, parts, _ = W.reverse_poiseuille(n_side=(6, 6, 12), kBT=0.0, g=0.0, eta=1.0, xi=20.0 / 21.0,
                                       dt=0.01, beta_eos=0.0)
    p["g"] = [0.0, 0.0, g]
    o = oracle_lib.Oracle(p, parts)
    o.step(3500)
    vmax = o.totals()[8]
    assert vmax < 2e-6
    pos, vel = o.read_field("POS"), o.read_field("VEL")
    k = int(np.argmin(((pos - np.array([3.0, 3.0, 3.0])) ** 2).sum(axis=1)))
    d, ratio = 2.0, 2.5
    R = d / 2
    vs = 4.0 / 3.0 * math.pi * R ** 3
    parts2 = {key: np.array(v, copy=True) for key, v in parts.items()}
    parts2["pos"], parts2["vel"] = pos, vel
    parts2["type"][k] = W.RIGID
    parts2["mass"][k] = ratio * vs
    parts2["inertia"][k] = 0.4 * ratio * vs * R * R
    parts2["radius"][k] = R
    o2 = oracle_lib.Oracle(p, parts2)
    o2.compute_forces()
    fpg = o2.read_field("F_PG")[k]
    # lower half (z < L/2): g_eff = -g z, buoyancy +rho0 V_s g z
    expect = np.array([0.0, 0.0, p["rho0"] * vs * g])
    assert np.allclose(fpg, expect, atol=5e-3 * np.linalg.norm(expect))


def _sphere_in_still_fluid(v_s, d=2.0, n=12):
    p, parts, _ = W.reverse_poiseuille(n_side=(n, n, n), kBT=0.0, g=0.0)
    c = np.array([n / 2 + 0.5] * 3)
    k = int(np.argmin(((parts["pos"] - c) ** 2).sum(axis=1)))
    R = d / 2
    vs = 4.0 / 3.0 * math.pi * R ** 3
    parts["type"][k] = W.RIGID
    parts["mass"][k] = 2.5 * vs
    parts["inertia"][k] = 0.4 * 2.5 * vs * R * R
    parts["radius"][k] = R
    parts["vel"][k] = v_s
    return p, parts, k


def test_isolated_sphere_feels_stokes_drag(oracle_lib):
    v = np.array([1e-4, -2e-4, 5e-5])
    p, parts, k = _sphere_in_still_fluid(v)
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    assert o.read_field("EPS")[k] == 1.0
    d, mu, rho = 2.0, p["eta"], p["rho0"]
    re = rho * d * np.linalg.norm(v) / mu
    expect = -3.0 * math.pi * mu * d * (1.0 + 0.15 * re ** 0.687) * v
    assert np.allclose(o.read_field("F_DG")[k], expect, rtol=1e-12, atol=0)
    # the reaction returns exactly the same momentum to the fluid
    rxn = o.read_field("F_RXN")
    assert np.allclose(rxn.sum(axis=0), -expect, rtol=1e-12, atol=1e-20)
    assert np.count_nonzero(np.abs(rxn).sum(axis=1)) > 20


def test_reaction_balances_drag_with_many_spheres(oracle_lib):
    p, parts, info = W.dam_break(tank=(24, 12, 20), column=(12, 12, 12), n_rigid=20, seed=3)
    parts = W.perturb(parts, p, jitter=0.0, kT=1e-3, seed=2)
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    fdg = o.read_field("F_DG")
    rxn = o.read_field("F_RXN")
    scale = np.abs(fdg).sum()
    assert scale > 0
    assert np.abs(rxn.sum(axis=0) + fdg.sum(axis=0)).max() < 1e-13 * scale
    eps = o.read_field("EPS")[parts["type"] == W.RIGID]
    assert np.all((eps >= p["eps_min"]) & (eps <= 1.0))


def test_free_flight_under_constant_force(oracle_lib):
    """A lone particle: velocity Verlet is exact for constant acceleration."""
    p, parts, _ = W.random_box(1, (10.0, 10.0, 10.0), (1, 1, 1), seed=0)
    p.update(kBT=0.0, dt=0.01, g=[0.001, -0.002, 0.0005], gravity_type=0)
    parts["pos"][0] = [2.0, 7.0, 4.0]
    parts["vel"][0] = [0.1, 0.05, -0.02]
    o = oracle_lib.Oracle(p, parts)
    o.step(300)
    t = 3.0
    g = np.array(p["g"])
    x = np.array([2.0, 7.0, 4.0]) + np.array([0.1, 0.05, -0.02]) * t + 0.5 * g * t * t
    x = np.mod(x, 10.0)
    assert np.allclose(o.read_field("POS")[0], x, rtol=0, atol=1e-12)
    assert np.allclose(o.read_field("VEL")[0], np.array([0.1, 0.05, -0.02]) + g * t, atol=1e-14)


@pytest.mark.parametrize("noslip", [1, 0])
def test_wall_reflection(oracle_lib, noslip):
    p, parts, _ = W.random_box(1, (10.0, 10.0, 10.0), (0, 1, 1), seed=0)
    p.update(kBT=0.0, dt=0.1, noslip=noslip)
    parts["pos"][0] = [9.5, 5.0, 5.0]
    parts["vel"][0] = [1.0, 0.3, 0.0]
    o = oracle_lib.Oracle(p, parts)
    o.step(10)  # leaves [0, 10] in the drift of step 6, then mirrored
    x = o.read_field("POS")[0]
    v = o.read_field("VEL")[0]
    assert x[0] == pytest.approx(10.0 - 0.5, abs=1e-12)
    assert v[0] == -1.0
    assert v[1] == (-0.3 if noslip else 0.3)
    assert x[1] == pytest.approx(5.0 + 0.3 * 0.6 + (-0.3 if noslip else 0.3) * 0.4, abs=1e-12)


@pytest.mark.parametrize("noslip", [1, 0])
def test_wall_corner_reflection(oracle_lib, noslip):
    """A drift that crosses two wall faces at once (an edge of the box):
    both coordinates are mirrored; no-slip reverses the whole velocity once
    (a second reversal would leave it unchanged), slip reverses the two
    normal components (Sec. 2.5)."""
    p, parts, _ = W.random_box(1, (10.0, 10.0, 10.0), (0, 0, 1), seed=0)
    p.update(kBT=0.0, dt=0.1, noslip=noslip)
    parts["pos"][0] = [9.95, 0.08, 5.0]
    parts["vel"][0] = [1.0, -1.0, 0.25]
    o = oracle_lib.Oracle(p, parts)
    o.step(1)
    x = o.read_field("POS")[0]
    v = o.read_field("VEL")[0]
    assert x[0] == pytest.approx(2 * 10.0 - 10.05, abs=1e-12)
    assert x[1] == pytest.approx(-(0.08 - 0.1), abs=1e-12)
    assert x[2] == pytest.approx(5.025, abs=1e-12)
    expect = [-1.0, 1.0, -0.25] if noslip else [-1.0, 1.0, 0.25]
    assert list(v) == expect


def test_error_codes(oracle_lib):
    O = oracle_lib
    p, parts, _ = W.reverse_poiseuille(n_side=(6, 6, 6), kBT=0.0)
    with pytest.raises(O.OracleError) as e:
        O.Oracle(dict(p, xi=0.0), parts)
    assert e.value.code == O.E_INVALID_ARG
    with pytest.raises(O.OracleError) as e:
        O.Oracle(dict(p, L=[4.0, 6.0, 6.0]), parts)
    assert e.value.code == O.E_INVALID_ARG
    bad = {k: np.array(v, copy=True) for k, v in parts.items()}
    bad["id"][3] = bad["id"][4]
    with pytest.raises(O.OracleError) as e:
        O.Oracle(p, bad)
    assert e.value.code == O.E_INVALID_ARG
    o = O.Oracle(dict(p, max_neighbors=10), parts)
    assert o.compute_forces(check=False) == O.E_NBR_OVERFLOW
    nan = {k: np.array(v, copy=True) for k, v in parts.items()}
    nan["vel"][5, 1] = np.nan
    assert O.Oracle(p, nan).step(1, check=False) == O.E_NONFINITE
    p2, one, _ = W.random_box(1, (10.0, 10.0, 10.0), (0, 0, 0), seed=0)
    p2.update(kBT=0.0, dt=1.0)
    one["vel"][0] = [100.0, 0.0, 0.0]
    assert O.Oracle(p2, one).step(1, check=False) == O.E_OUT_OF_DOMAIN


def _small_dam(oracle_lib, seed=0, lub=0):
    """A periodic fluid box with two pairs of d = 2 spheres set on collision
    courses with some tangential slip, so that DEM contacts form (with
    lubrication off: its 1/gap resistance would keep them apart)."""
    p, parts, _ = W.reverse_poiseuille(n_side=(10, 10, 10), kBT=1e-3, g=0.0, dt=0.01, seed=seed,
                                       enable_lub=lub)
    parts = W.perturb(parts, p, jitter=0.0, kT=1e-3, seed=11)
    centres = [(3.0, 5.0, 5.0), (5.02, 5.3, 5.0), (3.0, 2.0, 8.0), (3.1, 4.02, 8.2)]
    vels = [(0.1, 0.0, 0.05), (-0.1, 0.0, -0.05), (0.0, 0.1, 0.02), (0.03, -0.1, 0.0)]
    R = 1.0
    vs = 4.0 / 3.0 * math.pi * R ** 3
    for c, v in zip(centres, vels):
        k = int(np.argmin(((parts["pos"] - np.asarray(c)) ** 2).sum(axis=1)))
        parts["type"][k] = W.RIGID
        parts["pos"][k] = c
        parts["vel"][k] = v
        parts["mass"][k] = 2.5 * vs
        parts["inertia"][k] = 0.4 * 2.5 * vs * R * R
        parts["radius"][k] = R
    return p, parts


def test_restart_is_bit_exact(oracle_lib):
    p, parts = _small_dam(oracle_lib)
    a = oracle_lib.Oracle(p, parts)
    a.step(40)
    b = oracle_lib.Oracle(p, parts)
    b.step(20)
    saved = {k: np.array(v, copy=True) for k, v in parts.items()}
    saved["pos"], saved["vel"], saved["angvel"] = (b.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    pairs, dts = b.read_contacts()
    c = oracle_lib.Oracle(dict(p, itr_start=b.current_step), saved)
    c.load_contacts(pairs, dts)
    c.step(20)
    for f in ("POS", "VEL", "ANGVEL"):
        assert np.array_equal(a.read_field(f), c.read_field(f))
    pa, da = a.read_contacts()
    pc, dc = c.read_contacts()
    assert np.array_equal(pa, pc) and np.array_equal(da, dc)


def test_dem_contacts_form_and_persist(oracle_lib):
    p, parts = _small_dam(oracle_lib)
    o = oracle_lib.Oracle(p, parts)
    o.step(40)
    pairs, dts = o.read_contacts()
    pos = o.read_field("POS")
    rad = parts["radius"]
    assert pairs.shape[0] == 2
    assert np.all(np.linalg.norm(dts, axis=1) > 0)
    eps = o.read_field("EPS")
    for (i, j) in pairs:
        # overlapping spheres lie inside each other's coupling support
        assert eps[i] < 1.0 and eps[j] < 1.0
        assert np.linalg.norm(pos[i] - pos[j]) < rad[i] + rad[j]
        assert parts["type"][i] == W.RIGID and parts["type"][j] == W.RIGID


def test_thread_count_does_not_change_results(oracle_lib):
    p, parts = _small_dam(oracle_lib, seed=1)
    outs = []
    for nt in (1, 3):
        oracle_lib.set_num_threads(nt)
        o = oracle_lib.Oracle(p, parts)
        o.step(10)
        o.compute_forces()
        outs.append([o.read_field(f) for f in ("POS", "VEL", "F_SDPD", "F_DG", "F_DEM")])
    oracle_lib.set_num_threads(8)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_lubrication_resists_approach(oracle_lib):
    p, parts = _small_dam(oracle_lib, lub=1)
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    rig = np.nonzero(parts["type"] == W.RIGID)[0]
    fl = o.read_field("F_LUB")
    pos = parts["pos"]
    i, j = rig[0], rig[1]
    n = (pos[i] - pos[j]) / np.linalg.norm(pos[i] - pos[j])
    # closing pair: the lubrication force on i points away from j
    assert np.dot(fl[i], n) > 0 and np.dot(fl[j], n) < 0
    # pairwise and antisymmetric: the total vanishes
    assert np.abs(fl.sum(axis=0)).max() < 1e-13 * np.abs(fl).sum()
    o.step(40)
    assert o.read_contacts()[0].shape[0] == 0
