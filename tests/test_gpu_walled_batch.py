"""Walled boxes in one batch.  Every box keeps its outer walls behind its
active particles (fluid, spheres, inner walls), binned into a second range
of cell keys of its own, and the kernels of every pass launch over the
boxes' active parts only; three dam-break tanks of different sizes, each
with spheres, contacts and thermal noise, exercise that layout box by box.
Without a skin the batch must give every box the bits the box gets alone;
with candidate reuse each box's state is handed to the FP64 oracle, which
searches from scratch (neighbour sets bit for bit, fields and forces to
the single-step tolerances)."""
import numpy as np
import pytest

from _parity import VECTOR_FIELDS, assert_force_field, assert_same_neighbors, assert_scalar_fields
from paper_2002_03120_amd import workloads as W

pytestmark = pytest.mark.gpu

TANKS = [dict(tank=(24, 12, 20), column=(12, 12, 12), n_rigid=12, seed=1),
         dict(tank=(30, 10, 16), column=(14, 10, 10), n_rigid=8, seed=2),
         dict(tank=(18, 14, 22), column=(10, 14, 14), n_rigid=10, seed=3)]


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_03120_amd import sdpdem
    sdpdem.lib()
    return sdpdem


def _tanks():
    cells = []
    for k, t in enumerate(TANKS):
        p, parts, info = W.dam_break(kBT=1e-4, **t)
        parts = W.perturb(parts, p, jitter=0.1, kT=4e-2, seed=20 + k, spin=True)
        cells.append((p, parts, info))
    return cells


class _BoxView:
    """One box of a batch as the parity helpers see a system: fields and
    neighbour lists of its id range, ids shifted to start at zero."""

    def __init__(self, g, off, n):
        self.g, self.off, self.n = g, off, n

    def read_field(self, name):
        return self.g.read_field(name)[self.off:self.off + self.n]

    def read_neighbors(self):
        rows, cols = self.g.read_neighbors()
        r = rows[self.off:self.off + self.n + 1]
        return r - r[0], cols[r[0]:r[-1]] - self.off


def test_walled_batch_gives_every_box_its_own_bits(S):
    cells = _tanks()
    parts, boxes, box_of = W.stack_cells(cells)
    steps = 30
    print(f"[case] batch of {len(cells)} walled tanks, n={parts['id'].shape[0]}, search every step",
          flush=True)
    g = S.System(dict(cells[0][0], cell_factor=0.55), parts, boxes=boxes, box_of=box_of)
    assert g.step(steps) == 0
    state = {f: g.read_field(f) for f in ("POS", "VEL", "ANGVEL")}
    g.close()
    off = 0
    for b, (p, pp, info) in enumerate(cells):
        one = S.System(dict(p, cell_factor=0.55), pp)
        assert one.step(steps) == 0
        n = pp["id"].shape[0]
        for f, v in state.items():
            assert np.array_equal(v[off:off + n], one.read_field(f)), (b, f)
        one.close()
        off += n


def test_walled_batch_with_reuse_matches_the_oracle(S, oracle_lib):
    cells = _tanks()
    parts, boxes, box_of = W.stack_cells(cells)
    print(f"[case] batch of {len(cells)} walled tanks, n={parts['id'].shape[0]}, skin 0.3",
          flush=True)
    g = S.System(dict(cells[0][0], cell_factor=0.55, skin=0.3), parts, boxes=boxes, box_of=box_of)
    assert g.step(80) == 0
    info = g.info()
    print(f"  80 steps: {info[13]} searches, {info[14]} lists from candidates", flush=True)
    assert info[13] >= 2 and info[14] >= 20
    pos, vel, ang = (g.read_field(f) for f in ("POS", "VEL", "ANGVEL"))
    pairs, dts = g.read_contacts()
    assert g.compute_forces(check=False) == 0
    off = 0
    for b, (p, pp, _info) in enumerate(cells):
        n = pp["id"].shape[0]
        st = {k: np.array(v, copy=True) for k, v in pp.items()}
        st["pos"], st["vel"], st["angvel"] = pos[off:off + n], vel[off:off + n], ang[off:off + n]
        o = oracle_lib.Oracle(dict(p, itr_start=g.current_step), st)
        mine = np.all((pairs >= off) & (pairs < off + n), axis=1)
        if mine.any():
            o.load_contacts(pairs[mine] - off, dts[mine])
        assert o.compute_forces(check=False) == 0
        view = _BoxView(g, off, n)
        nnz = assert_same_neighbors(view, o)
        assert_scalar_fields(view, o, p)
        worst = {f: assert_force_field(view, o, f) for f in VECTOR_FIELDS}
        print(f"  box {b}: n {n}, nnz {nnz}, worst rel "
              f"{max(worst.values()):.1e}", flush=True)
        off += n
    g.close()
