"""Pins of oracle.brute against triangles counted by hand (Sec. 2, the
weighted-average-over-closed-triangles reading of Eq. 12)."""
import numpy as np

from oracle import brute, plan

# rings on an 8 x 8 grid: a0 = {|g|^2 = 1} (4 axis cells), a1 = {|g|^2 = 2} (4 diagonals),
# a2 = {|g|^2 = 4} ((+-2, 0), (0, +-2))
EDGES = [1.0, 1.2, 1.5, 2.1]


def test_ring_cells_by_hand():
    cells = plan.ring_cells(8, EDGES)
    as_set = [set(map(tuple, c.tolist())) for c in cells]
    assert as_set[0] == {(1, 0), (-1, 0), (0, 1), (0, -1)}
    assert as_set[1] == {(1, 1), (1, -1), (-1, 1), (-1, -1)}
    assert as_set[2] == {(2, 0), (-2, 0), (0, 2), (0, -2)}


def test_hand_counted_triangles():
    trips = [(0, 0, 0), (0, 0, 1), (0, 1, 1), (1, 1, 1), (0, 0, 2), (1, 1, 2), (0, 1, 2)]
    # (0,0,1): g1 perpendicular to g2 -> 4 * 2 ordered pairs; (0,0,2): g2 = g1 -> 4;
    # (1,1,2): two diagonals summing to an axis vector of length 2: g2 = g1 reflected
    # about the axis -> 4 * 2; (0,1,2): unit axis + diagonal = length-2 axis vector
    # never holds -> 0; three unit vectors or three diagonals never close -> 0.
    # (0,1,1): an axis vector plus a diagonal is never a diagonal -> 0.
    want = [0, 8, 0, 0, 4, 8, 0]
    got = brute.triangle_counts(8, EDGES, trips, cyclic=False)
    assert got.tolist() == want
    got_c = brute.triangle_counts(8, EDGES, trips, cyclic=True)
    assert got_c.tolist() == want   # max |g| = 2 < 8/3: no wrap-around


def test_weighted_sum_by_hand():
    # X = 1 everywhere except X(1,0) = X(-1,0) = 2: triplet (0,0,2) has the four
    # triangles (g, g, -2g) for the axis units g; the two along u carry 2*2 = 4.
    n = 8
    X = np.ones((n, n), complex)
    X[0, 1] = 2.0
    X[0, n - 1] = 2.0
    s = brute.triangle_sums(X, n, EDGES, [(0, 0, 2)], cyclic=False)
    assert np.isclose(s[0], 2 * 4 + 2 * 1)


def test_wraparound_differs_from_planar():
    # n = 8: (2,0) + (3,0) + (3,0) = (8,0) = 0 mod 8 closes only cyclically
    edges = [1.9, 2.1, 3.0, 3.5]
    trips = [(0, 2, 2)]
    cyc = brute.triangle_counts(8, edges, trips, cyclic=True)
    pla = brute.triangle_counts(8, edges, trips, cyclic=False)
    assert cyc[0] > pla[0] > 0
