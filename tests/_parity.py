"""Comparison helpers for GPU-vs-oracle parity tests (not a test module)."""
import numpy as np

# Single-step FP32 force fields: per particle, |X_gpu - X_ref| must stay
# below REL_FORCE times the oracle's sum of |pair term| for that particle,
# the scale that remains meaningful where X itself cancels to ~0.
REL_FORCE = 1e-5
# the same over the whole system, in the 2-norm
REL_FORCE_GLOBAL = 1e-6

VECTOR_FIELDS = ["F_SDPD", "F_CD", "N_SDPD", "F_DG", "F_PG", "F_RXN", "F_DEM", "F_LUB", "N_DEM"]


def force_errors(gpu, ref, name):
    a = gpu.read_field(name)
    b = ref.read_field(name)
    scale = ref.read_field(name + "_ABS")
    err = np.linalg.norm(a - b, axis=1)
    return a, b, scale, err


def assert_force_field(gpu, ref, name, rel=REL_FORCE, rel_global=REL_FORCE_GLOBAL):
    a, b, scale, err = force_errors(gpu, ref, name)
    tiny = 1e-30 + 1e-12 * (scale.max() if scale.size else 0.0)
    bad = err > rel * scale + tiny
    if bad.any():
        k = int(np.argmax(err / (scale + tiny)))
        raise AssertionError(
            f"{name}: {int(bad.sum())} particles beyond {rel} x sum|pair term|; worst id {k} "
            f"gpu {a[k]} ref {b[k]} scale {scale[k]}")
    tot = np.linalg.norm(scale)
    if tot > 0:
        g = np.linalg.norm(err) / tot
        assert g <= rel_global, f"{name}: global error {g}"
    return float((err / (scale + tiny)).max()) if err.size else 0.0


def assert_scalar_fields(gpu, ref, params):
    rho_g, rho_o = gpu.read_field("DENS"), ref.read_field("DENS")
    assert np.allclose(rho_g, rho_o, rtol=1e-12, atol=0), np.abs(rho_g / rho_o - 1).max()
    p_g, p_o = gpu.read_field("PRES"), ref.read_field("PRES")
    # d p = alpha p0 (rho/rho0)^(alpha-1) d rho / rho0: scale by alpha p0
    pscale = params["alpha"] * params["p0"] * np.maximum(1.0, (rho_o / params["rho0"]) ** (params["alpha"] - 1))
    assert np.all(np.abs(p_g - p_o) <= 1e-12 * pscale), np.abs(p_g - p_o).max()
    ps_g, ps_o = gpu.read_field("PRES_SMOOTH"), ref.read_field("PRES_SMOOTH")
    # stored in FP32: one rounding of |p~| plus the FP64 differences above
    tol = 1.2e-7 * np.abs(ps_o) + 1e-12 * pscale
    assert np.all(np.abs(ps_g - ps_o) <= tol), np.abs(ps_g - ps_o).max()
    eps_g, eps_o = gpu.read_field("EPS"), ref.read_field("EPS")
    assert np.allclose(eps_g, eps_o, rtol=1e-14, atol=0)


def assert_same_neighbors(gpu, ref):
    rg, cg = gpu.read_neighbors()
    ro, co = ref.read_neighbors()
    assert np.array_equal(rg, ro), "row lengths differ"
    assert np.array_equal(cg, co), "neighbour ids differ"
    return int(co.size)
