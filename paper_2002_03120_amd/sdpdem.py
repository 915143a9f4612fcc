"""Python binding of the C ABI in include/sdpdem.h (libsdpdem.so).

Argument marshalling only: every step of the SDPD-DEM path runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the
stream.  The functions carry the C names; :class:`System` bundles a handle
with the workspace tensor that must outlive it.

Importing this module does not load the library; the first call does, and
raises if ``libsdpdem.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdpdem.so")

OK = 0
E_INVALID_ARG = -1
E_WORKSPACE_TOO_SMALL = -2
E_NBR_OVERFLOW = -3
E_CONTACT_OVERFLOW = -4
E_NONFINITE = -5
E_OUT_OF_DOMAIN = -6
E_HIP = -7

FIELDS = {
    "POS": 0, "VEL": 1, "ANGVEL": 2, "DENS": 3, "PRES": 4, "PRES_SMOOTH": 5,
    "F_SDPD": 6, "F_CD": 7, "N_SDPD": 8, "F_DG": 9, "F_PG": 10, "F_RXN": 11,
    "F_DEM": 12, "F_LUB": 13, "N_DEM": 14, "F_TOTAL": 15, "N_TOTAL": 16, "EPS": 17,
}
KERNELS = {
    "none": 0, "bin": 1, "sort": 2, "permute": 3, "neighbors_density": 4, "smooth": 5,
    "fluid_forces": 6, "fpi_action": 7, "fpi_reaction": 8, "dem": 9, "integrate": 10,
    "rigid_grid": 11,
}


class Params(ctypes.Structure):
    """sdpdem_params (field order is part of the ABI)."""
    _fields_ = [
        ("org", ctypes.c_double * 3), ("L", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32 * 3), ("noslip", ctypes.c_int32),
        ("dx", ctypes.c_double), ("h", ctypes.c_double),
        ("rho0", ctypes.c_double), ("p0", ctypes.c_double),
        ("alpha", ctypes.c_double), ("beta_eos", ctypes.c_double),
        ("eta", ctypes.c_double), ("xi", ctypes.c_double), ("kBT", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("g", ctypes.c_double * 3), ("f", ctypes.c_double * 3),
        ("gravity_type", ctypes.c_int32), ("gravity_axis", ctypes.c_int32),
        ("coeff_c", ctypes.c_double), ("coeff_d", ctypes.c_double),
        ("coeff_r", ctypes.c_double), ("coeff_t", ctypes.c_double),
        ("E_dem", ctypes.c_double), ("nu_dem", ctypes.c_double),
        ("mu_fric", ctypes.c_double), ("dem_damping", ctypes.c_double),
        ("mass_fluid", ctypes.c_double), ("inertia_fluid", ctypes.c_double),
        ("enable_kernel_norm", ctypes.c_int32), ("enable_pres_smooth", ctypes.c_int32),
        ("enable_neg_p_clamp", ctypes.c_int32), ("enable_lub", ctypes.c_int32),
        ("eps_min", ctypes.c_double), ("lub_gap_min", ctypes.c_double),
        ("itr_start", ctypes.c_int64), ("itr_actv_rigid", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("max_neighbors", ctypes.c_int32), ("max_contacts", ctypes.c_int32),
        ("shear_rate", ctypes.c_double),
        ("cell_factor", ctypes.c_double), ("skin", ctypes.c_double),
    ]


class Particles(ctypes.Structure):
    """sdpdem_particles (host pointers)."""
    _fields_ = [
        ("n", ctypes.c_int64), ("id", ctypes.c_void_p), ("type", ctypes.c_void_p),
        ("pos", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("angvel", ctypes.c_void_p),
        ("mass", ctypes.c_void_p), ("inertia", ctypes.c_void_p), ("radius", ctypes.c_void_p),
    ]


class Box(ctypes.Structure):
    """sdpdem_box: one box of a batch."""
    _fields_ = [
        ("org", ctypes.c_double * 3), ("L", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
        ("shear_rate", ctypes.c_double), ("kBT", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_2002_03120_amd/build.py "
                "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        L.sdpdem_workspace_bytes.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Particles),
                                             ctypes.POINTER(sz)]
        L.sdpdem_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Particles), vp, sz,
                                    vp, ctypes.POINTER(vp)]
        L.sdpdem_create_static.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Particles),
                                           vp, ctypes.POINTER(vp)]
        L.sdpdem_batch_workspace_bytes.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Box),
                                                   ctypes.c_int32, ctypes.POINTER(Particles),
                                                   vp, ctypes.POINTER(sz)]
        L.sdpdem_create_batch.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Box),
                                          ctypes.c_int32, ctypes.POINTER(Particles), vp, vp, sz,
                                          vp, ctypes.POINTER(vp)]
        L.sdpdem_set_stress.argtypes = [vp, ctypes.c_int, vp]
        L.sdpdem_set_graph.argtypes = [vp, ctypes.c_int]
        L.sdpdem_box_stress.argtypes = [vp, vp, vp, ctypes.POINTER(i64), vp]
        L.sdpdem_step.argtypes = [vp, i64, vp]
        L.sdpdem_compute_forces.argtypes = [vp, vp]
        L.sdpdem_read_field.argtypes = [vp, ctypes.c_int, vp, sz, ctypes.c_int, vp]
        L.sdpdem_field_comps.argtypes = [ctypes.c_int]
        L.sdpdem_read_neighbors.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64), vp]
        L.sdpdem_read_contacts.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64), vp]
        L.sdpdem_load_contacts.argtypes = [vp, vp, vp, i64, vp]
        L.sdpdem_totals.argtypes = [vp, vp, vp]
        L.sdpdem_get_step.argtypes = [vp]
        L.sdpdem_get_step.restype = i64
        L.sdpdem_info.argtypes = [vp, vp, vp]
        L.sdpdem_set_profiling.argtypes = [vp, ctypes.c_int]
        L.sdpdem_set_profiling_every.argtypes = [vp, ctypes.c_int]
        L.sdpdem_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.sdpdem_destroy.argtypes = [vp]
        L.sdpdem_destroy.restype = None
        L.sdpdem_status_string.argtypes = [ctypes.c_int]
        L.sdpdem_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


class SdpdemError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {sdpdem_status_string(code)} ({code})")
        self.code = code


def _check(code, what):
    if code != OK:
        raise SdpdemError(code, what)
    return code


def make_params(d: dict) -> Params:
    p = Params()
    names = {f[0] for f in Params._fields_}
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


def make_particles(parts: dict):
    """Contiguous host copies and the sdpdem_particles struct pointing at them."""
    n = int(parts["id"].shape[0])
    keep = {
        "id": np.ascontiguousarray(parts["id"], dtype=np.int64),
        "type": np.ascontiguousarray(parts["type"], dtype=np.uint8),
        "pos": np.ascontiguousarray(parts["pos"], dtype=np.float64).reshape(n, 3),
        "vel": np.ascontiguousarray(parts["vel"], dtype=np.float64).reshape(n, 3),
        "angvel": np.ascontiguousarray(parts["angvel"], dtype=np.float64).reshape(n, 3),
        "mass": np.ascontiguousarray(parts["mass"], dtype=np.float64).reshape(n),
        "inertia": np.ascontiguousarray(parts["inertia"], dtype=np.float64).reshape(n),
        "radius": np.ascontiguousarray(parts["radius"], dtype=np.float64).reshape(n),
    }
    q = Particles(n, *(keep[k].ctypes.data for k in
                       ("id", "type", "pos", "vel", "angvel", "mass", "inertia", "radius")))
    return q, keep


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---- functions with the C names ------------------------------------------

def sdpdem_status_string(code: int) -> str:
    return lib().sdpdem_status_string(int(code)).decode()


def sdpdem_workspace_bytes(params: dict, parts: dict) -> int:
    p = make_params(params)
    q, _keep = make_particles(parts)
    out = ctypes.c_size_t()
    _check(lib().sdpdem_workspace_bytes(ctypes.byref(p), ctypes.byref(q), ctypes.byref(out)),
           "sdpdem_workspace_bytes")
    return int(out.value)


def sdpdem_create(params: dict, parts: dict, workspace, stream=None) -> ctypes.c_void_p:
    """workspace: a device tensor of at least sdpdem_workspace_bytes bytes."""
    p = make_params(params)
    q, _keep = make_particles(parts)
    h = ctypes.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().sdpdem_create(ctypes.byref(p), ctypes.byref(q),
                               ctypes.c_void_p(workspace.data_ptr()), nbytes,
                               _stream(stream), ctypes.byref(h)), "sdpdem_create")
    return h


def sdpdem_create_static(params: dict, parts: dict, stream=None) -> ctypes.c_void_p:
    """A system in the library's own static device array (no workspace)."""
    p = make_params(params)
    q, _keep = make_particles(parts)
    h = ctypes.c_void_p()
    _check(lib().sdpdem_create_static(ctypes.byref(p), ctypes.byref(q), _stream(stream),
                                      ctypes.byref(h)), "sdpdem_create_static")
    return h


def make_boxes(boxes):
    """Array of sdpdem_box from a list of dicts (org, L, periodic, shear_rate,
    kBT, seed)."""
    arr = (Box * len(boxes))()
    for b, d in zip(arr, boxes):
        for a in range(3):
            b.org[a] = float(d["org"][a])
            b.L[a] = float(d["L"][a])
            b.periodic[a] = int(d["periodic"][a])
        b.reserved = 0
        b.shear_rate = float(d.get("shear_rate", 0.0))
        b.kBT = float(d.get("kBT", 0.0))
        b.seed = int(d.get("seed", 0))
    return arr


def sdpdem_batch_workspace_bytes(params: dict, boxes, parts: dict, box_of) -> int:
    p = make_params(params)
    bx = make_boxes(boxes)
    q, _keep = make_particles(parts)
    bo = np.ascontiguousarray(box_of, dtype=np.int32)
    out = ctypes.c_size_t()
    _check(lib().sdpdem_batch_workspace_bytes(ctypes.byref(p), bx, len(boxes), ctypes.byref(q),
                                              bo.ctypes.data, ctypes.byref(out)),
           "sdpdem_batch_workspace_bytes")
    return int(out.value)


def sdpdem_create_batch(params: dict, boxes, parts: dict, box_of, workspace,
                        stream=None) -> ctypes.c_void_p:
    p = make_params(params)
    bx = make_boxes(boxes)
    q, _keep = make_particles(parts)
    bo = np.ascontiguousarray(box_of, dtype=np.int32)
    h = ctypes.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().sdpdem_create_batch(ctypes.byref(p), bx, len(boxes), ctypes.byref(q),
                                     bo.ctypes.data, ctypes.c_void_p(workspace.data_ptr()),
                                     nbytes, _stream(stream), ctypes.byref(h)),
           "sdpdem_create_batch")
    return h


def sdpdem_set_stress(h, on: bool, stream=None):
    _check(lib().sdpdem_set_stress(h, 1 if on else 0, _stream(stream)), "sdpdem_set_stress")


def sdpdem_box_stress(h, nbox: int, stream=None):
    """(last P_zx sample per box, running sums per box, number of samples)"""
    inst = np.zeros(nbox)
    tot = np.zeros(nbox)
    m = ctypes.c_int64()
    _check(lib().sdpdem_box_stress(h, inst.ctypes.data, tot.ctypes.data, ctypes.byref(m),
                                   _stream(stream)), "sdpdem_box_stress")
    return inst, tot, int(m.value)


def sdpdem_step(h, nsteps: int, stream=None) -> int:
    return lib().sdpdem_step(h, int(nsteps), _stream(stream))


def sdpdem_compute_forces(h, stream=None) -> int:
    return lib().sdpdem_compute_forces(h, _stream(stream))


def sdpdem_read_field(h, name: str, n: int, stream=None, out=None):
    """Host copy (numpy) of a field in id order; with `out` a float64 device
    tensor of n x comps elements the rows are written there instead and the
    copy is only enqueued on the stream."""
    f = FIELDS[name]
    c = lib().sdpdem_field_comps(f)
    if out is not None:
        if not out.is_cuda or out.dtype.itemsize != 8 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor")
        _check(lib().sdpdem_read_field(h, f, ctypes.c_void_p(out.data_ptr()),
                                       out.numel() * 8, 1, _stream(stream)),
               "sdpdem_read_field")
        return out
    host = np.empty((n, c), dtype=np.float64)
    _check(lib().sdpdem_read_field(h, f, host.ctypes.data, host.nbytes, 0, _stream(stream)),
           "sdpdem_read_field")
    return host if c > 1 else host[:, 0]


def sdpdem_read_neighbors(h, n: int, stream=None):
    rp = np.empty(n + 1, dtype=np.int64)
    nnz = ctypes.c_int64()
    st = _stream(stream)
    _check(lib().sdpdem_read_neighbors(h, rp.ctypes.data, None, 0, ctypes.byref(nnz), st),
           "sdpdem_read_neighbors")
    cols = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().sdpdem_read_neighbors(h, rp.ctypes.data, cols.ctypes.data, nnz.value,
                                       ctypes.byref(nnz), st), "sdpdem_read_neighbors")
    return rp, cols[: nnz.value]


def sdpdem_read_contacts(h, stream=None):
    m = ctypes.c_int64()
    st = _stream(stream)
    _check(lib().sdpdem_read_contacts(h, None, None, 0, ctypes.byref(m), st),
           "sdpdem_read_contacts")
    pairs = np.empty((max(m.value, 1), 2), dtype=np.int32)
    dt = np.empty((max(m.value, 1), 3), dtype=np.float64)
    _check(lib().sdpdem_read_contacts(h, pairs.ctypes.data, dt.ctypes.data, m.value,
                                      ctypes.byref(m), st), "sdpdem_read_contacts")
    return pairs[: m.value], dt[: m.value]


def sdpdem_load_contacts(h, pairs, delta_t, stream=None):
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    dt = np.ascontiguousarray(delta_t, dtype=np.float64).reshape(-1, 3)
    _check(lib().sdpdem_load_contacts(h, pairs.ctypes.data, dt.ctypes.data, pairs.shape[0],
                                      _stream(stream)), "sdpdem_load_contacts")


def sdpdem_totals(h, stream=None) -> np.ndarray:
    out = np.zeros(16, dtype=np.float64)
    _check(lib().sdpdem_totals(h, out.ctypes.data, _stream(stream)), "sdpdem_totals")
    return out


def sdpdem_get_step(h) -> int:
    return int(lib().sdpdem_get_step(h))


def sdpdem_info(h, stream=None) -> np.ndarray:
    out = np.zeros(16, dtype=np.int64)
    _check(lib().sdpdem_info(h, out.ctypes.data, _stream(stream)), "sdpdem_info")
    return out


def sdpdem_set_profiling(h, kernel: str):
    _check(lib().sdpdem_set_profiling(h, KERNELS[kernel]), "sdpdem_set_profiling")


def sdpdem_kernel_time(h):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().sdpdem_kernel_time(h, ctypes.byref(ms), ctypes.byref(n)), "sdpdem_kernel_time")
    return ms.value, int(n.value)


def sdpdem_destroy(h):
    lib().sdpdem_destroy(h)


# ---- convenience wrapper --------------------------------------------------

class System:
    """A system plus the device workspace it lives in (torch uint8 tensor)."""

    def __init__(self, params: dict, parts: dict, device="cuda", stream=None, boxes=None,
                 box_of=None, static=False):
        """boxes/box_of: a batch of independent boxes (sdpdem_create_batch);
        static: no workspace, the library's static array (sdpdem_create_static)."""
        import torch
        self.n = int(parts["id"].shape[0])
        self.params = dict(params)
        self.stream = stream
        self.nbox = len(boxes) if boxes is not None else 1
        if static:
            self.workspace = None
            self.h = sdpdem_create_static(params, parts, stream)
        elif boxes is None:
            nbytes = sdpdem_workspace_bytes(params, parts)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
            self.h = sdpdem_create(params, parts, self.workspace, stream)
        else:
            nbytes = sdpdem_batch_workspace_bytes(params, boxes, parts, box_of)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
            self.h = sdpdem_create_batch(params, boxes, parts, box_of, self.workspace, stream)

    def close(self):
        if getattr(self, "h", None):
            sdpdem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1, check=True):
        rc = sdpdem_step(self.h, nsteps, self.stream)
        if check:
            _check(rc, "sdpdem_step")
        return rc

    def compute_forces(self, check=True):
        rc = sdpdem_compute_forces(self.h, self.stream)
        if check:
            _check(rc, "sdpdem_compute_forces")
        return rc

    def read_field(self, name, out=None):
        return sdpdem_read_field(self.h, name, self.n, self.stream, out=out)

    def read_neighbors(self):
        return sdpdem_read_neighbors(self.h, self.n, self.stream)

    def read_contacts(self):
        return sdpdem_read_contacts(self.h, self.stream)

    def load_contacts(self, pairs, delta_t):
        sdpdem_load_contacts(self.h, pairs, delta_t, self.stream)

    def totals(self):
        return sdpdem_totals(self.h, self.stream)

    def info(self):
        return sdpdem_info(self.h, self.stream)

    @property
    def current_step(self):
        return sdpdem_get_step(self.h)

    def set_profiling(self, kernel, every=1):
        """Time the launches of `kernel` (the first of every `every`)."""
        _check(lib().sdpdem_set_profiling_every(self.h, int(every)), "sdpdem_set_profiling_every")
        sdpdem_set_profiling(self.h, kernel)

    def set_graph(self, steps_per_graph):
        """Replay steps from a captured graph (needs a non-null stream)."""
        _check(lib().sdpdem_set_graph(self.h, int(steps_per_graph)), "sdpdem_set_graph")

    def set_stress(self, on=True):
        sdpdem_set_stress(self.h, on, self.stream)

    def box_stress(self):
        return sdpdem_box_stress(self.h, self.nbox, self.stream)

    def kernel_time(self):
        return sdpdem_kernel_time(self.h)
