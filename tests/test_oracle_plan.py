"""Pins of oracle.plan: ring membership, the triangle-inequality prefilter and
the lattice filter, against direct enumeration (Sec. 2 rings, Sec. 3 triplets)."""
import itertools

import numpy as np
import pytest

from oracle import brute, plan


def test_half_open_ring_boundaries():
    # (3,4) has |g| = 5 exactly: it belongs to [5, 6) and not to [4, 5)
    rc = plan.ring_of_cell(32, [4.0, 5.0, 6.0])
    assert rc[4, 3] == 1 and rc[0, 5] == 1 and rc[0, 4] == 0
    assert rc[0, 0] == -1


@pytest.mark.parametrize("n,edges", [(16, [1.0, 1.9, 2.6, 3.4, 4.6, 5.3]),
                                     (32, [1.2, 2.0, 3.3, 5.1, 7.0, 10.5])])
def test_prefilter_is_necessary_and_lattice_filter_exact(n, edges):
    nb = len(edges) - 1
    every = [t for t in itertools.combinations_with_replacement(range(nb), 3)]
    counts = brute.triangle_counts(n, edges, every, cyclic=False)
    pre = set(plan.prefilter_triplets(edges))
    for t, c in zip(every, counts):
        if c > 0:
            assert t in pre, t          # a closed triangle obeys lo_k < hi_i + hi_j
    trips, cnt = plan.plan_triplets(n, edges)
    want = [t for t, c in zip(every, counts) if c > 0]
    assert [tuple(x) for x in trips.tolist()] == want
    assert cnt.tolist() == [int(c) for c in counts if c > 0]


def test_c1_shapes():
    # 128 x 128, 8 log rings 2 .. 42: 120 combinations, 79 pass the prefilter,
    # 75 contain closed lattice triangles
    e = plan.log_edges(2.0, 42.0, 8)
    assert len(list(itertools.combinations_with_replacement(range(8), 3))) == 120
    assert len(plan.prefilter_triplets(e)) == 79
    trips, _ = plan.plan_triplets(128, e)
    assert len(trips) == 75
