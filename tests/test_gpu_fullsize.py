"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark uses (fluid cells of h/2) and at cells of h:
the sedimentation box (101,080 particles), the dam break (1,534,168
particles, 2^20 moving) and the periodic scale box (8,388,608 particles).
The oracle evaluates every particle here; neighbour sets must match bit
for bit."""
import numpy as np
import pytest

from _parity import VECTOR_FIELDS, assert_force_field, assert_same_neighbors, assert_scalar_fields
from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import sdpdem
    sdpdem.lib()
    return sdpdem


@pytest.mark.parametrize("name,cf", [("sedimentation", 0.5), ("sedimentation", 1.0),
                                     ("dam_break", 0.5), ("dam_break", 1.0),
                                     ("periodic_scale", 0.5)])
def test_full_size_single_step(S, oracle_lib, name, cf):
    p, parts, info = W.CONFIGS[name]()
    parts = W.perturb(parts, p, jitter=0.05, kT=1e-4, seed=7)
    print(f"[case] full-size {name}: n={info['n']} cell_factor={cf}", flush=True)
    g = S.System(dict(p, cell_factor=cf), parts)
    o = oracle_lib.Oracle(p, parts)
    assert g.compute_forces(check=False) == 0
    assert o.compute_forces(check=False) == 0
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in VECTOR_FIELDS}
    print("  nnz", nnz, {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
