"""Oracle: direct enumeration of closed grid triangles (tiny grids only).

TEST INFRASTRUCTURE ONLY (see the package header).

Source: Gill et al. 2024, Sec. 2, the paragraph after Eq. (12): the estimator
considers all closed triangles U_g1 + U_g2 + U_g3 = 0 with one vertex in each of
the three rings and returns their weighted average.  Here the numerator and
denominator of Eq. (12) are written out as those triangle sums:

    S_t = sum_{g1 in a_i} sum_{g2 in a_j} [g3 = -(g1 + g2) in a_k] X(g1) X(g2) X(g3)
    N_t = the same with Y

``cyclic=True`` closes triangles modulo n (what a periodic DFT sums);
``cyclic=False`` requires the planar closure g1 + g2 + g3 = 0 with g3 on the grid.
Cost is O(|a_i| |a_j|) per triplet: use n <= 32.

Parity: this module is the independent pin of ``estimator``; it is itself
checked against hand-countable cases in tests/test_oracle_brute.py.
"""
import numpy as np

from .plan import ring_of_cell, ring_cells


def triangle_sums(X, n, edges, trips, cyclic=True):
    """Sum of X(g1) X(g2) X(g3) over closed triangles, per triplet (complex)."""
    rc = ring_of_cell(n, edges)
    cells = ring_cells(n, edges)
    out = np.zeros(len(trips), np.complex128)
    for t, (i, j, k) in enumerate(trips):
        g1 = cells[i][:, None, :]
        g2 = cells[j][None, :, :]
        g3 = -(g1 + g2)
        if cyclic:
            g3w = ((g3 + n // 2) % n) - n // 2
            inside = np.ones(g3.shape[:2], bool)
        else:
            g3w = g3
            inside = np.all((g3 >= -(n // 2)) & (g3 < n - n // 2), axis=2)
        ix = np.where(inside, g3w[..., 0] % n, 0)
        iy = np.where(inside, g3w[..., 1] % n, 0)
        ok = inside & (rc[iy, ix] == k)
        if not ok.any():
            continue
        a = X[cells[i][:, 1] % n, cells[i][:, 0] % n][:, None]
        b = X[cells[j][:, 1] % n, cells[j][:, 0] % n][None, :]
        c = X[iy, ix]
        out[t] = np.sum(np.where(ok, a * b * c, 0))
    return out


def triangle_counts(n, edges, trips, cyclic=True):
    """Number of closed lattice triangles per triplet (integers)."""
    one = np.ones((n, n), np.complex128)
    return np.rint(triangle_sums(one, n, edges, trips, cyclic).real).astype(np.int64)
