"""Host-side checks of the C-ABI library that need no GPU: it loads,
exports every symbol declared in include/*.h, sizes workspaces and rejects bad
arguments before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2002_03120_amd import sdpdem as S
from paper_2002_03120_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    import glob
    src = "".join(open(f).read() for f in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    return sorted(set(re.findall(r"\b(sdpdem_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        from paper_2002_03120_amd import build as B
        B.build()
    return S.lib()


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 15
    for name in syms:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert S.sdpdem_status_string(code) not in ("", "unknown status")
    assert S.sdpdem_status_string(-99) == "unknown status"


def test_field_comps(lib):
    for name, f in S.FIELDS.items():
        c = lib.sdpdem_field_comps(f)
        assert c == (1 if name in ("DENS", "PRES", "PRES_SMOOTH", "EPS") else 3)
    assert lib.sdpdem_field_comps(99) == 0


def test_workspace_scales_with_problem(lib):
    p, parts, _ = W.reverse_poiseuille(n_side=(10, 10, 10))
    small = S.sdpdem_workspace_bytes(p, parts)
    p2, parts2, _ = W.reverse_poiseuille(n_side=(20, 20, 20))
    big = S.sdpdem_workspace_bytes(p2, parts2)
    assert 6 * small < big < 10 * small
    p3 = dict(p2, max_neighbors=128)
    assert S.sdpdem_workspace_bytes(p3, parts2) > big


def test_cell_factor_grows_the_grid_below_h(lib):
    p, parts, _ = W.reverse_poiseuille(n_side=(20, 20, 20))
    base = S.sdpdem_workspace_bytes(p, parts)
    assert S.sdpdem_workspace_bytes(dict(p, cell_factor=1.0), parts) == base  # 0 means 1
    half = S.sdpdem_workspace_bytes(dict(p, cell_factor=0.5), parts)
    quarter = S.sdpdem_workspace_bytes(dict(p, cell_factor=0.25), parts)
    assert base < half < quarter  # the cell arrays grow with the number of cells


def test_skin_adds_candidate_rows(lib):
    """Candidate reuse keeps a second column-major table of the partners
    within h + skin (rows of max_neighbors ((h + skin)/h)^3) and the
    positions of the last search."""
    p, parts, _ = W.reverse_poiseuille(n_side=(20, 20, 20))
    base = S.sdpdem_workspace_bytes(p, parts)
    assert S.sdpdem_workspace_bytes(dict(p, skin=0.0), parts) == base
    n = parts["id"].shape[0]
    g = (p["h"] + 0.3) / p["h"]
    rows = math.ceil(p["max_neighbors"] * g ** 3)
    grown = S.sdpdem_workspace_bytes(dict(p, skin=0.3), parts) - base
    need = 4 * rows * n + 4 * n + 32 * n  # candidates, their counts, reference positions
    assert abs(grown - need) <= 3 * 256  # 256-byte pieces (one each without reuse)


@pytest.mark.parametrize("bad", [
    dict(xi=0.0), dict(xi=1.0), dict(h=0.0), dict(dt=-1.0), dict(L=[4.0, 10.0, 10.0]),
    dict(max_neighbors=0), dict(gravity_axis=3), dict(rho0=0.0),
    dict(cell_factor=0.2), dict(cell_factor=-1.0), dict(cell_factor=float("nan")),
    dict(cell_factor=17.0), dict(cell_factor=4.0),  # 4 h cells: fewer than 3 on a 10-site axis
    dict(skin=-0.1), dict(skin=0.76), dict(skin=float("nan")),  # 0 <= skin <= h/2 = 0.75
])
def test_rejects_bad_params(lib, bad):
    p, parts, _ = W.reverse_poiseuille(n_side=(10, 10, 10))
    p.update(bad)
    with pytest.raises(S.SdpdemError) as e:
        S.sdpdem_workspace_bytes(p, parts)
    assert e.value.code == S.E_INVALID_ARG


def test_rejects_bad_particles(lib):
    p, parts, _ = W.reverse_poiseuille(n_side=(6, 6, 6))
    dup = {k: np.array(v, copy=True) for k, v in parts.items()}
    dup["id"][0] = dup["id"][1]
    badt = {k: np.array(v, copy=True) for k, v in parts.items()}
    badt["type"][3] = 7
    rig = {k: np.array(v, copy=True) for k, v in parts.items()}
    rig["type"][3] = W.RIGID
    rig["radius"][3] = 0.0
    for q in (dup, badt, rig):
        with pytest.raises(S.SdpdemError):
            S.sdpdem_workspace_bytes(p, q)


def test_create_rejects_small_workspace_without_device(lib):
    p, parts, _ = W.reverse_poiseuille(n_side=(6, 6, 6))
    pp = S.make_params(p)
    q, keep = S.make_particles(parts)
    h = ctypes.c_void_p()
    # a fake non-null pointer with too few bytes is refused before any HIP call
    rc = lib.sdpdem_create(ctypes.byref(pp), ctypes.byref(q), ctypes.c_void_p(256), 1024,
                           None, ctypes.byref(h))
    assert rc == S.E_WORKSPACE_TOO_SMALL
    rc = lib.sdpdem_create(ctypes.byref(pp), ctypes.byref(q), None, 1 << 30, None,
                           ctypes.byref(h))
    assert rc == S.E_INVALID_ARG


_CITE = re.compile(r"\b(Sec\.|Secs\.|Eq\.|Eqs\.|Alg\.|Algs\.|Algorithms?|Table|Fig\.)\s")


def _declarations_with_comments():
    """(header, symbol, the comment block that precedes its declaration)."""
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = open(f).read()
        # top-level declarations: a line that starts with a type and names sdpdem_*(
        for m in re.finditer(r"^(?:const\s+)?[a-z_0-9]+\s*\**\s*(sdpdem_[a-z_]+)\s*\(", src,
                             re.M):
            before = src[:m.start()]
            end = before.rfind("*/")
            start = before.rfind("/*", 0, end) if end >= 0 else -1
            out.append((os.path.basename(f), m.group(1),
                        before[start:end] if start >= 0 else ""))
    return out


def test_every_declaration_cites_its_passage():
    decls = _declarations_with_comments()
    assert len(decls) >= 25
    # the one allocation-free variant names its callers instead of a passage
    missing = [(h, name) for h, name, c in decls
               if not _CITE.search(c) and "cannot allocate" not in c]
    assert not missing, missing
