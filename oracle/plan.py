"""Oracle: annular rings and the ring-triplet list (FP64 / exact integers).

TEST INFRASTRUCTURE ONLY (see the package header).

Sources (Gill et al. 2024):
* Sec. 2, the paragraph introducing Eq. (10): the uv plane is divided into
  annular rings a_m with mean radii U_m, and ell_m = 2 pi U_m.
* Sec. 3, the ring scheme paragraph: B-hat is evaluated for all triplets of rings,
  each estimate being the average over all closed triangles with one vertex in
  each ring.
* Sec. 2, below Eq. (3): ell_1 >= ell_2 >= ell_3, mu = (l1^2 + l2^2 - l3^2)/(2 l1 l2),
  t = l2 / l1 (Sec. 2 after Eq. 12 gives the same mu in terms of side lengths).

Readings where the paper is silent:
* ring membership is half-open, lo <= |g| < hi, decided with the exact integer
  |g|^2 compared against the FP64 squares of the edges;
* a triplet (i <= j <= k) exists when its rings contain at least one closed
  lattice triangle (counted modulo n, which is what a periodic FFT counts);
  the cheap prefilter lo_k < hi_i + hi_j is the triangle inequality;
* the "mean radius" of a ring is the unweighted mean of |g| over its lattice
  cells (used only for labels).

Pins: tests/test_oracle_plan.py (brute-force counts on tiny grids, the
triangle-inequality prefilter, label ranges, the paper's 22-ring scheme).
"""
import numpy as np


def signed_index(n):
    """Grid index i -> signed frequency g (DC at 0, i >= n/2 maps to i - n)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < n // 2, i, i - n)


def cell_r2(n):
    """Exact integer gx^2 + gy^2 on the [row = gy][col = gx] grid."""
    g = signed_index(n)
    return g[:, None] ** 2 + g[None, :] ** 2


def ring_of_cell(n, edges):
    """Bin id of every grid cell, or -1 when the cell is in no ring."""
    edges = np.asarray(edges, dtype=np.float64)
    r2 = cell_r2(n).astype(np.float64)  # exact: r2 < 2**53
    out = np.full((n, n), -1, dtype=np.int64)
    for m in range(len(edges) - 1):
        lo2, hi2 = edges[m] * edges[m], edges[m + 1] * edges[m + 1]
        out[(r2 >= lo2) & (r2 < hi2)] = m
    return out


def ring_masks(n, edges):
    rc = ring_of_cell(n, edges)
    return np.stack([rc == m for m in range(len(edges) - 1)])


def ring_cells(n, edges):
    """Signed (gx, gy) coordinates of every lattice cell of every ring."""
    rc = ring_of_cell(n, edges)
    g = signed_index(n)
    out = []
    for m in range(len(edges) - 1):
        iy, ix = np.nonzero(rc == m)
        out.append(np.stack([g[ix], g[iy]], axis=1))
    return out


def mean_radius(n, edges):
    """Unweighted mean |g| over each ring's lattice cells (NaN for empty rings)."""
    res = []
    for c in ring_cells(n, edges):
        res.append(np.sqrt((c.astype(np.float64) ** 2).sum(1)).mean() if len(c) else np.nan)
    return np.array(res)


def prefilter_triplets(edges):
    """All i <= j <= k whose rings can close a triangle: lo_k < hi_i + hi_j."""
    e = np.asarray(edges, dtype=np.float64)
    nb = len(e) - 1
    return [(i, j, k) for i in range(nb) for j in range(i, nb) for k in range(j, nb)
            if e[k] < e[i + 1] + e[j + 1]]


def unit_counts(n, edges, trips, chunk=1 << 16):
    """Number of closed lattice triangles (mod n) per triplet, exact integers.

    Computed as sum_theta I_i I_j I_k / n^2 with unit-valued ring fields I_m
    (Eq. 11 with W = 1), by numpy FFT in FP64, then rounded; the rounding step
    asserts that the FP64 value is within 1e-3 of an integer.
    """
    from .estimator import triple_sums
    masks = ring_masks(n, edges)
    F = np.stack([np.fft.fft2(m.astype(np.float64)).real for m in masks])
    c = triple_sums(F, trips, chunk=chunk)
    r = np.rint(c)
    assert np.all(np.abs(c - r) < 1e-3), "unit counts are not integral"
    return r.astype(np.int64)


def plan_triplets(n, edges):
    """Triplets with at least one closed lattice triangle, and their counts."""
    cand = prefilter_triplets(edges)
    if not cand:
        return np.zeros((0, 3), np.int64), np.zeros(0, np.int64)
    cnt = unit_counts(n, edges, cand)
    keep = cnt >= 1
    return np.array(cand, dtype=np.int64)[keep], cnt[keep]


def labels(n, edges, trips, du=1.0):
    """(ell1, ell2, ell3, mu, t) per triplet from the rings' mean radii.

    Triplets are stored i <= j <= k, so ell1 = ell_k >= ell2 = ell_j >= ell3 = ell_i
    with ell = 2 pi du U_m (Sec. 2, ell = 2 pi U).
    """
    ell = 2.0 * np.pi * du * mean_radius(n, edges)
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    l3, l2, l1 = ell[trips[:, 0]], ell[trips[:, 1]], ell[trips[:, 2]]
    mu = (l1 ** 2 + l2 ** 2 - l3 ** 2) / (2.0 * l1 * l2)
    t = l2 / l1
    return np.stack([l1, l2, l3, mu, t], axis=1)


def log_edges(lo, hi, nb):
    """nb logarithmically spaced rings between radii lo and hi (grid units)."""
    return lo * (hi / lo) ** (np.arange(nb + 1, dtype=np.float64) / nb)


def paper_ring_edges():
    """The 22-ring scheme of Sec. 3: one ring 1-5, nine rings 5-50, five 50-100,
    five 100-200 and two 200-250 (grid units), equal widths within each group."""
    e = [1.0, 5.0]
    for lo, hi, k in ((5.0, 50.0, 9), (50.0, 100.0, 5), (100.0, 200.0, 5), (200.0, 250.0, 2)):
        e += list(lo + (hi - lo) * np.arange(1, k + 1) / k)
    return np.array(e)
