"""sdpdem_create_static (no workspace: the library's static device array)
against sdpdem_create with a caller workspace: the same kernels on the same
input, so every field matches bit for bit.  Two systems in a row through
the static array, the second smaller, and an oversize request refused."""
import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("POS", "VEL", "ANGVEL", "DENS", "PRES_SMOOTH", "F_SDPD", "F_DG", "F_PG", "F_RXN",
          "F_DEM", "N_DEM")


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import sdpdem
    sdpdem.lib()
    return sdpdem


def _compare(S, p, parts, steps, label):
    print(f"[case] {label}: n={parts['id'].shape[0]}, workspace "
          f"{S.sdpdem_workspace_bytes(p, parts)} bytes", flush=True)
    ref = S.System(p, parts)
    st = S.System(p, parts, static=True)
    assert st.workspace is None
    for sysm in (ref, st):
        sysm.compute_forces()
    for f in FIELDS:
        assert np.array_equal(ref.read_field(f), st.read_field(f)), f
    ref.step(steps)
    st.step(steps)
    for f in FIELDS:
        assert np.array_equal(ref.read_field(f), st.read_field(f)), f
    rr, cr = ref.read_neighbors()
    rs, cs = st.read_neighbors()
    assert np.array_equal(rr, rs) and np.array_equal(cr, cs)
    assert np.array_equal(ref.totals(), st.totals())
    ref.close()
    st.close()


def test_static_matches_workspace_twice_second_smaller(S):
    p, parts, _ = W.dam_break(tank=(24, 12, 20), column=(12, 12, 12), n_rigid=12, seed=1,
                              kBT=1e-4)
    parts = W.perturb(parts, p, jitter=0.1, kT=1e-4, seed=2)
    _compare(S, dict(p, cell_factor=0.5), parts, 4, "dam break 24x12x20, 12 spheres")
    p2, parts2, _ = W.reverse_poiseuille(n_side=(9, 9, 9), kBT=1e-3)
    parts2 = W.perturb(parts2, p2, jitter=0.1, kT=1e-3, seed=3, spin=True)
    _compare(S, p2, parts2, 3, "reverse Poiseuille 9^3 (smaller)")


def test_static_with_candidate_reuse(S):
    """With a skin the allocation-free system reads the moved flag through a
    synchronised copy instead of a pinned word; it searches at the same
    steps and matches the workspace system bit for bit."""
    p, parts, _ = W.dam_break(tank=(24, 12, 20), column=(12, 12, 12), n_rigid=12, seed=4,
                              kBT=1e-4)
    parts = W.perturb(parts, p, jitter=0.1, kT=4e-2, seed=5, spin=True)
    _compare(S, dict(p, skin=0.3), parts, 40, "dam break 24x12x20 with skin 0.3, 40 steps")


def test_static_refuses_oversize(S):
    p, parts, _ = W.reverse_poiseuille(n_side=(64, 64, 64), kBT=0.0)
    need = S.sdpdem_workspace_bytes(p, parts)
    assert need > (64 << 20)
    with pytest.raises(S.SdpdemError) as e:
        S.System(p, parts, static=True)
    assert e.value.code == S.E_WORKSPACE_TOO_SMALL
