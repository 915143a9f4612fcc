"""Host logic of the viscometer autotuner: how cells are packed into batch
tiles and which cell sizes a set of periodic cells admits."""
import numpy as np

from paper_2002_03120_amd import autotune as AT
from paper_2002_03120_amd import workloads as W


def _cells(sizes):
    return [({"h": 1.5, "L": [s, s, s], "periodic": [1, 1, 1]}, None, {"n": s ** 3})
            for s in sizes]


def test_split_packs_consecutive_cells_under_the_tile():
    rng = np.random.default_rng(0)
    sizes = [int(x) for x in rng.integers(10, 40, size=57)]
    cells = _cells(sizes)
    for tile in (1, 5000, 60000, 1 << 20, 1 << 30):
        parts = AT.split(cells, tile)
        assert parts[0][0] == 0 and parts[-1][1] == len(cells)
        for (a, b, n), nxt in zip(parts, parts[1:] + [None]):
            assert b > a
            assert n == sum(s ** 3 for s in sizes[a:b])
            assert n <= tile or b == a + 1  # only a lone oversized cell exceeds it
            if nxt is not None:
                assert nxt[0] == b
                assert n + sizes[b] ** 3 > tile  # greedy: the next cell did not fit
    assert AT.split([], 100) == []
    assert len(AT.split(cells, 1 << 30)) == 1


def test_fits_requires_three_cells_per_periodic_axis():
    cells = _cells([10])
    assert AT.fits(cells, 1.0)          # 10 // 1.5 = 6
    assert AT.fits(cells, 2.2)          # 10 // 3.3 = 3
    assert not AT.fits(cells, 2.3)      # 10 // 3.45 = 2
    walls = [({"h": 1.5, "L": [4.0, 4.0, 4.0], "periodic": [0, 0, 0]}, None, {"n": 8})]
    assert AT.fits(walls, 5.0)


def test_viscometer_cells_admit_the_candidate_cell_sizes():
    _, cells = W.viscometer_batch(8, seed=3, side=(16, 40), steps=10)
    assert all(AT.fits(cells, cf) for cf in AT.CELL_FACTORS)
