"""The oracle's grid + linked-list neighbour search against O(N^2) brute
force with explicit periodic images, on small random boxes."""
import itertools

import numpy as np
import pytest

from paper_2002_03120_amd import workloads as W


def brute_force_neighbors(pos, typ, L, periodic, h):
    """Rows by id, columns ascending: all j != i with r^2 < h^2 for some
    periodic image, r^2 = (dx*dx + dy*dy) + dz*dz; outer walls own no row."""
    n = pos.shape[0]
    shifts = [s for s in itertools.product((-1, 0, 1), repeat=3)
              if all(periodic[a] or s[a] == 0 for a in range(3))]
    h2 = h * h
    rows = []
    for i in range(n):
        if typ[i] == W.OUTER_WALL:
            rows.append(np.zeros(0, np.int64))
            continue
        hit = np.zeros(n, bool)
        raw = pos[i][None, :] - pos
        for s in shifts:
            d = raw - np.asarray(s, float) * np.asarray(L, float)
            r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            hit |= r2 < h2
        hit[i] = False
        rows.append(np.nonzero(hit)[0])
    return rows


CASES = [
    ("periodic", (7.0, 6.0, 8.0), (1, 1, 1), 900, 0),
    ("walls", (6.0, 7.5, 5.0), (0, 0, 0), 700, 1),
    ("hybrid_xy", (6.0, 6.0, 9.0), (1, 1, 0), 800, 2),
    ("hybrid_z", (5.0, 9.0, 4.6), (0, 0, 1), 600, 3),
    ("exact_h_pairs", (6.0, 6.0, 6.0), (1, 1, 1), 500, 4),
]


@pytest.mark.parametrize("name,L,per,n,seed", CASES)
def test_neighbors_match_brute_force(oracle_lib, name, L, per, n, seed):
    p, parts, _ = W.random_box(n, L, per, h=1.5, seed=seed,
                               exact_pairs=60 if name == "exact_h_pairs" else 0,
                               wall=(name == "walls"))
    if name == "walls":
        # also make a few outer walls: they own no neighbour row
        parts["type"][::13] = W.OUTER_WALL
    p["kBT"] = 0.0
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    rp, cols = o.read_neighbors()
    ref = brute_force_neighbors(parts["pos"], parts["type"], L, per, 1.5)
    for i in range(n):
        assert np.array_equal(cols[rp[i]:rp[i + 1]], ref[i]), i
    if name == "exact_h_pairs":
        # pairs planted at exactly r = h are not neighbours (strict <)
        for k in range(60):
            a, b = 2 * k, 2 * k + 1
            assert b not in cols[rp[a]:rp[a + 1]]


def test_lattice_has_18_neighbours(oracle_lib):
    p, parts, _ = W.reverse_poiseuille(n_side=(6, 6, 6), kBT=0.0)
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    rp, _ = o.read_neighbors()
    assert np.all(np.diff(rp) == 18)


def test_symmetric_neighbor_relation(oracle_lib):
    p, parts, _ = W.random_box(1000, (8.0, 8.0, 8.0), (1, 0, 1), seed=9)
    p["kBT"] = 0.0
    o = oracle_lib.Oracle(p, parts)
    o.compute_forces()
    rp, cols = o.read_neighbors()
    pairs = set()
    for i in range(1000):
        for j in cols[rp[i]:rp[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)
