"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark uses: the sedimentation box (101,080 particles)
and the dam break (1,534,168 particles, 2^20 moving).  The oracle evaluates
every particle here; neighbour sets must match bit for bit."""
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


@pytest.mark.parametrize("name", ["sedimentation", "dam_break"])
def test_full_size_single_step(S, oracle_lib, name):
    p, parts, info = W.CONFIGS[name]()
    parts = W.perturb(parts, p, jitter=0.05, kT=1e-4, seed=7)
    print(f"[case] full-size {name}: n={info['n']}", flush=True)
    g = S.System(p, parts)
    o = oracle_lib.Oracle(p, parts)
    assert g.compute_forces(check=False) == 0
    assert o.compute_forces(check=False) == 0
    nnz = assert_same_neighbors(g, o)
    assert_scalar_fields(g, o, p)
    worst = {f: assert_force_field(g, o, f) for f in VECTOR_FIELDS}
    print("  nnz", nnz, {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
