"""Pins of the oracle's SDPD pair force (Eqs. FijC, FijD, FijR, FijT).

None of these re-types the formulas: they check symmetries that the paper's
forces must have (antisymmetry, Galilean invariance, zero viscous force under
solid-body rotation with matching spin) and the fluctuation-dissipation
relation between the dissipative and the random force.
"""
import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W


def _params(**over):
    p = W.base_params(kBT=1e-3, dt=1e-3)
    p.update(over)
    return p


def _rand_pair(rng, h=1.5):
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    r = rng.uniform(0.2, 0.95) * h
    return (r * e, rng.standard_normal(3) * 0.1, rng.standard_normal(3) * 0.1,
            rng.standard_normal(3) * 0.1, rng.standard_normal(3) * 0.1,
            rng.uniform(0.9, 1.1), rng.uniform(0.9, 1.1),
            rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2))


def test_pair_antisymmetry_is_exact(oracle_lib):
    rng = np.random.default_rng(0)
    p = _params(xi=0.13)
    for k in range(200):
        rij, vi, vj, wi, wj, di, dj, pi, pj = _rand_pair(rng)
        a = oracle_lib.pair_force(p, rij, vi, vj, wi, wj, di, dj, pi, pj, 11, 93, k)
        b = oracle_lib.pair_force(p, -rij, vj, vi, wj, wi, dj, di, pj, pi, 93, 11, k)
        for fa, fb in zip(a, b):
            assert np.array_equal(fa, -fb)


def test_galilean_invariance(oracle_lib):
    rng = np.random.default_rng(1)
    p = _params(kBT=0.0)
    for k in range(50):
        rij, vi, vj, wi, wj, di, dj, pi, pj = _rand_pair(rng)
        u = rng.standard_normal(3)
        a = oracle_lib.pair_force(p, rij, vi, vj, wi, wj, di, dj, pi, pj, 1, 2, 0)
        b = oracle_lib.pair_force(p, rij, vi + u, vj + u, wi, wj, di, dj, pi, pj, 1, 2, 0)
        for fa, fb in zip(a, b):
            assert np.allclose(fa, fb, rtol=1e-12, atol=1e-14)


def test_solid_body_rotation_feels_no_viscous_force(oracle_lib):
    # v = Omega x r with spin Omega on both particles: F^D + F^R = 0
    rng = np.random.default_rng(2)
    p = _params(kBT=0.0, xi=0.11)
    for k in range(50):
        om = rng.standard_normal(3)
        xi_ = rng.standard_normal(3) * 3
        rij = _rand_pair(rng)[0]
        xj_ = xi_ - rij
        vi, vj = np.cross(om, xi_), np.cross(om, xj_)
        fc, fd, fr, ft = oracle_lib.pair_force(p, rij, vi, vj, om, om, 1.0, 1.0, 0.0, 0.0, 3, 4, 0)
        assert np.linalg.norm(fd) > 1e-3
        assert np.allclose(fd + fr, 0.0, atol=1e-14 * np.linalg.norm(fd) + 1e-16)
        # a wrong sign of the rotational term would double it instead
        assert np.linalg.norm(fd - fr) > 1.5 * np.linalg.norm(fd)


@pytest.mark.parametrize("xi_frac", [20.0 / 21.0, 0.9, 1.4])
def test_fluctuation_dissipation(oracle_lib, xi_frac):
    """Cov(F^T dt) = 2 kT dt Gamma, Gamma read off the dissipative force."""
    eta, kT, dt = 0.1, 2e-3, 1e-3
    p = _params(eta=eta, xi=xi_frac * eta, kBT=kT, dt=dt)
    pd = dict(p, kBT=0.0, coeff_c=0.0, coeff_r=0.0)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    rij = 0.8 * e
    z3 = np.zeros(3)
    # friction matrix: F^D = -Gamma v_ij
    G = np.zeros((3, 3))
    for a in range(3):
        v = np.zeros(3)
        v[a] = 1.0
        fd = oracle_lib.pair_force(pd, rij, v, z3, z3, z3, 1.0, 1.0, 0.0, 0.0, 1, 2, 0)[1]
        G[:, a] = -fd
    assert np.allclose(G, G.T, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(G) > 0)
    n = 40000
    samples = np.empty((n, 3))
    for k in range(n):
        ft = oracle_lib.pair_force(p, rij, z3, z3, z3, z3, 1.0, 1.0, 0.0, 0.0, 5, 6, k)[3]
        samples[k] = ft * dt
    cov = samples.T @ samples / n
    target = 2.0 * kT * dt * G
    scale = np.sqrt(np.outer(np.diag(target), np.diag(target)))
    # statistical tolerance: 5 standard errors of a covariance estimate
    tol = 5.0 * np.sqrt(2.0 / n) * scale
    assert np.all(np.abs(cov - target) < tol + 1e-3 * scale.max())
    assert np.abs(samples.mean(axis=0)).max() < 5.0 * np.sqrt(np.diag(target).max() / n)


@pytest.mark.parametrize("xi_frac", [20.0 / 21.0, 1.4])
def test_thermal_force_has_the_law_of_the_matrix_form(oracle_lib, xi_frac):
    """The thermal force the oracle draws from four normals against Eq. FijT
    written out with a full matrix of independent standard increments
    (numpy draws Z, forms (sa (sym Z - tr Z/3 1) + sb tr Z/3 1) e / sqrt dt
    with the sigma coefficients of Sec. 2.1): the same mean and the same
    covariance matrix, component by component."""
    eta, kT, dt, h = 0.1, 2e-3, 1e-3, 1.5
    xi = xi_frac * eta
    p = _params(eta=eta, xi=xi, kBT=kT, dt=dt)
    rng = np.random.default_rng(11)
    e = rng.standard_normal(3)
    e /= np.linalg.norm(e)
    r = 0.7
    F = oracle_lib.lucy_f(r, h)
    ga = (20.0 * eta / 3.0 - 4.0 * xi) * F
    gb = (17.0 * xi - 40.0 * eta / 3.0) * F
    sa, sb = 2.0 * np.sqrt(kT * ga), 2.0 * np.sqrt(kT * gb)
    z3 = np.zeros(3)
    n = 40000
    drawn = np.array([oracle_lib.pair_force(p, r * e, z3, z3, z3, z3, 1.0, 1.0, 0.0, 0.0, 8, 3, k)[3]
                      for k in range(n)])
    Z = rng.standard_normal((n, 3, 3))
    S = 0.5 * (Z + np.transpose(Z, (0, 2, 1)))
    t = np.trace(Z, axis1=1, axis2=2) / 3.0
    D = S - t[:, None, None] * np.eye(3)
    ref = (sa * (D @ e) + sb * t[:, None] * e) / np.sqrt(dt)
    ca, cr = drawn.T @ drawn / n, ref.T @ ref / n
    scale = np.sqrt(np.outer(np.diag(cr), np.diag(cr)))
    tol = 7.0 * np.sqrt(2.0 / n) * scale  # two independent estimates
    assert np.all(np.abs(ca - cr) < tol)
    assert np.abs(drawn.mean(axis=0)).max() < 5.0 * np.sqrt(np.diag(cr).max() / n)
    # the part along e carries sa^2 2/3 + sb^2 1/3, each direction across e sa^2/2
    par = drawn @ e
    assert abs(par.var() * dt / (sa * sa * 2.0 / 3.0 + sb * sb / 3.0) - 1.0) < 5.0 * np.sqrt(2.0 / n)
