"""ctypes binding of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of the benchmark use this module; the product path never imports it.  It
imports nothing from the GPU package, and the GPU package imports nothing
from here.  Inputs come as plain numpy arrays (from the seeded generators);
every output is returned in id order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sdpdem_oracle.c")

OK = 0
E_INVALID_ARG = -1
E_NBR_OVERFLOW = -3
E_CONTACT_OVERFLOW = -4
E_NONFINITE = -5
E_OUT_OF_DOMAIN = -6
E_NOMEM = -8

FLUID, RIGID, INNER_WALL, OUTER_WALL = 0, 1, 2, 3

FIELDS = {
    "POS": 0, "VEL": 1, "ANGVEL": 2, "DENS": 3, "PRES": 4, "PRES_SMOOTH": 5,
    "F_SDPD": 6, "F_CD": 7, "N_SDPD": 8, "F_DG": 9, "F_PG": 10, "F_RXN": 11,
    "F_DEM": 12, "F_LUB": 13, "N_DEM": 14, "F_TOTAL": 15, "N_TOTAL": 16,
    "EPS": 17,
    "F_SDPD_ABS": 32, "F_CD_ABS": 33, "N_SDPD_ABS": 34, "F_DG_ABS": 35,
    "F_PG_ABS": 36, "F_RXN_ABS": 37, "F_DEM_ABS": 38, "F_LUB_ABS": 39,
    "N_DEM_ABS": 40,
}


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("org", ctypes.c_double * 3), ("L", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32 * 3), ("noslip", ctypes.c_int32),
        ("dx", ctypes.c_double), ("h", ctypes.c_double),
        ("rho0", ctypes.c_double), ("p0", ctypes.c_double),
        ("alpha", ctypes.c_double), ("beta_eos", ctypes.c_double),
        ("eta", ctypes.c_double), ("xi", ctypes.c_double),
        ("kBT", ctypes.c_double), ("dt", ctypes.c_double),
        ("g", ctypes.c_double * 3), ("f", ctypes.c_double * 3),
        ("gravity_type", ctypes.c_int32), ("gravity_axis", ctypes.c_int32),
        ("coeff_c", ctypes.c_double), ("coeff_d", ctypes.c_double),
        ("coeff_r", ctypes.c_double), ("coeff_t", ctypes.c_double),
        ("E_dem", ctypes.c_double), ("nu_dem", ctypes.c_double),
        ("mu_fric", ctypes.c_double), ("dem_damping", ctypes.c_double),
        ("mass_fluid", ctypes.c_double), ("inertia_fluid", ctypes.c_double),
        ("enable_kernel_norm", ctypes.c_int32),
        ("enable_pres_smooth", ctypes.c_int32),
        ("enable_neg_p_clamp", ctypes.c_int32), ("enable_lub", ctypes.c_int32),
        ("eps_min", ctypes.c_double), ("lub_gap_min", ctypes.c_double),
        ("itr_start", ctypes.c_int64), ("itr_actv_rigid", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("max_neighbors", ctypes.c_int32), ("max_contacts", ctypes.c_int32),
        ("shear_rate", ctypes.c_double),
    ]


def make_params(d: dict) -> OracleParams:
    """Fill the C parameter struct from a plain dict of named values."""
    p = OracleParams()
    names = {f[0] for f in OracleParams._fields_}
    for k, v in d.items():
        if k not in names:
            raise KeyError(f"unknown parameter {k!r}")
        attr = getattr(p, k)
        if isinstance(attr, ctypes.Array):
            for i, x in enumerate(v):
                attr[i] = x
        else:
            setattr(p, k, v)
    return p


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_lucy_w.restype = ctypes.c_double
        L.oracle_lucy_w.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_lucy_f.restype = ctypes.c_double
        L.oracle_lucy_f.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_lattice_w_sum.restype = ctypes.c_double
        L.oracle_lattice_w_sum.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_drag_b.restype = ctypes.c_double
        L.oracle_drag_b.argtypes = [ctypes.c_double] * 5
        L.oracle_pair_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int64, dp]
        L.oracle_create.argtypes = [ctypes.POINTER(OracleParams), ctypes.c_int64] + [
            ctypes.c_void_p] * 8 + [ctypes.POINTER(ctypes.c_void_p)]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_destroy.restype = None
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.oracle_compute_forces.argtypes = [ctypes.c_void_p]
        L.oracle_read_field.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.oracle_read_neighbors.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64)]
        L.oracle_read_contacts.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64)]
        L.oracle_load_contacts.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int64]
        L.oracle_totals.argtypes = [ctypes.c_void_p, dp]
        L.oracle_stress.argtypes = [ctypes.c_void_p, dp]
        L.oracle_get_step.restype = ctypes.c_int64
        L.oracle_get_step.argtypes = [ctypes.c_void_p]
        L.oracle_field_comps.argtypes = [ctypes.c_int]
        L.oracle_philox4x32_10.argtypes = [ctypes.c_void_p] * 3
        L.oracle_pair_force.argtypes = [ctypes.POINTER(OracleParams)] + [dp] * 5 + [
            ctypes.c_double] * 4 + [ctypes.c_int64] * 3 + [dp] * 4
        L.oracle_dem_pair.argtypes = [ctypes.POINTER(OracleParams)] + [dp] * 5 + [
            ctypes.c_double] * 4 + [dp] * 4 + [ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with oracle status {code}")
        self.code = code


class Oracle:
    """One oracle system, created from a params dict and particle arrays."""

    def __init__(self, params: dict, particles: dict):
        L = lib()
        self._p = make_params(params)
        n = int(particles["id"].shape[0])
        self.n = n
        self._arr = {
            "id": np.ascontiguousarray(particles["id"], dtype=np.int64),
            "type": np.ascontiguousarray(particles["type"], dtype=np.uint8),
        }
        for k in ("pos", "vel", "angvel"):
            self._arr[k] = np.ascontiguousarray(particles[k], dtype=np.float64).reshape(n, 3)
        for k in ("mass", "inertia", "radius"):
            self._arr[k] = np.ascontiguousarray(particles[k], dtype=np.float64).reshape(n)
        h = ctypes.c_void_p()
        a = self._arr
        rc = L.oracle_create(ctypes.byref(self._p), n, _ptr(a["id"]), _ptr(a["type"]),
                             _ptr(a["pos"]), _ptr(a["vel"]), _ptr(a["angvel"]),
                             _ptr(a["mass"]), _ptr(a["inertia"]), _ptr(a["radius"]),
                             ctypes.byref(h))
        if rc != OK:
            raise OracleError(rc, "oracle_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps: int = 1, check: bool = True) -> int:
        rc = lib().oracle_step(self._h, int(nsteps))
        if check and rc != OK:
            raise OracleError(rc, "oracle_step")
        return rc

    def compute_forces(self, check: bool = True) -> int:
        rc = lib().oracle_compute_forces(self._h)
        if check and rc != OK:
            raise OracleError(rc, "oracle_compute_forces")
        return rc

    def read_field(self, name: str) -> np.ndarray:
        f = FIELDS[name]
        c = lib().oracle_field_comps(f)
        out = np.empty((self.n, c), dtype=np.float64)
        rc = lib().oracle_read_field(self._h, f, _ptr(out))
        if rc != OK:
            raise OracleError(rc, "oracle_read_field")
        return out if c > 1 else out[:, 0]

    def read_neighbors(self):
        rp = np.empty(self.n + 1, dtype=np.int64)
        nnz = ctypes.c_int64()
        lib().oracle_read_neighbors(self._h, _ptr(rp), None, 0, ctypes.byref(nnz))
        cols = np.empty(max(nnz.value, 1), dtype=np.int32)
        rc = lib().oracle_read_neighbors(self._h, _ptr(rp), _ptr(cols), nnz.value,
                                         ctypes.byref(nnz))
        if rc != OK:
            raise OracleError(rc, "oracle_read_neighbors")
        return rp, cols[: nnz.value]

    def read_contacts(self):
        m = ctypes.c_int64()
        lib().oracle_read_contacts(self._h, None, None, 0, ctypes.byref(m))
        pairs = np.empty((max(m.value, 1), 2), dtype=np.int32)
        dt = np.empty((max(m.value, 1), 3), dtype=np.float64)
        rc = lib().oracle_read_contacts(self._h, _ptr(pairs), _ptr(dt), m.value,
                                        ctypes.byref(m))
        if rc != OK:
            raise OracleError(rc, "oracle_read_contacts")
        return pairs[: m.value], dt[: m.value]

    def load_contacts(self, pairs, delta_t):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        dt = np.ascontiguousarray(delta_t, dtype=np.float64).reshape(-1, 3)
        rc = lib().oracle_load_contacts(self._h, _ptr(pairs), _ptr(dt), pairs.shape[0])
        if rc != OK:
            raise OracleError(rc, "oracle_load_contacts")

    def totals(self) -> np.ndarray:
        out = np.zeros(16, dtype=np.float64)
        lib().oracle_totals(self._h, _dp(out))
        return out

    def stress(self) -> np.ndarray:
        """Pressure tensor (3x3) of the box: kinetic part from the current
        velocities, virial of the last force evaluation."""
        out = np.zeros(9)
        rc = lib().oracle_stress(self._h, _dp(out))
        if rc:
            raise OracleError(rc, "stress")
        return out.reshape(3, 3)

    @property
    def current_step(self) -> int:
        return int(lib().oracle_get_step(self._h))


# ---- pure functions ------------------------------------------------------

def lucy_w(r, h):
    return lib().oracle_lucy_w(float(r), float(h))


def lucy_f(r, h):
    return lib().oracle_lucy_f(float(r), float(h))


def lattice_w_sum(h, dx):
    return lib().oracle_lattice_w_sum(float(h), float(dx))


def drag_b(eps, dv, d, rho, mu):
    return lib().oracle_drag_b(float(eps), float(dv), float(d), float(rho), float(mu))


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def pair_normals(seed, id_a, id_b, step):
    z = np.zeros(4, dtype=np.float64)
    lib().oracle_pair_normals(int(seed), int(id_a), int(id_b), int(step), _dp(z))
    return z


def pair_force(params: dict, rij, vi, vj, wi, wj, di, dj, psi, psj, idi, idj, step):
    """Returns (F^C, F^D, F^R, F^T) of one pair as four 3-vectors."""
    p = make_params(params)
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (rij, vi, vj, wi, wj)]
    outs = [np.zeros(3) for _ in range(4)]
    lib().oracle_pair_force(ctypes.byref(p), *[_dp(a) for a in arrs], float(di), float(dj),
                            float(psi), float(psj), int(idi), int(idj), int(step),
                            *[_dp(o) for o in outs])
    return outs


def dem_pair(params: dict, dij, vi, vj, wi, wj, Ri, Rj, mi, mj, dt_in):
    """Returns (F_n, F_t, delta_t_new, sliding) of one rigid contact."""
    p = make_params(params)
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (dij, vi, vj, wi, wj)]
    dti = np.ascontiguousarray(dt_in, dtype=np.float64)
    fn, ft, dto = np.zeros(3), np.zeros(3), np.zeros(3)
    sl = ctypes.c_int()
    lib().oracle_dem_pair(ctypes.byref(p), *[_dp(a) for a in arrs], float(Ri), float(Rj),
                          float(mi), float(mj), _dp(dti), _dp(fn), _dp(ft), _dp(dto),
                          ctypes.byref(sl))
    return fn, ft, dto, bool(sl.value)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib().oracle_set_num_threads.restype = None
    lib().oracle_set_num_threads(int(n))
