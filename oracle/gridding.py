"""Oracle: gridding of visibilities onto the uv grid, Eq. (9), in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Source: Gill et al. 2024, Sec. 2, Eq. (9): V_g = sum_i w~(U_g - U_i) V(U_i) with each
visibility assigned to the nearest grid point, N_g the number of contributing
visibilities, and Sec. 3: grid spacing dU_g = sqrt(ln 2) / (pi theta_0).

Readings of the paper where it is silent or ambiguous:
* nearest cell = round-half-to-even of u / dU_g in FP64 (numpy.rint), a rule that
  is symmetric under U -> -U;
* every visibility also contributes conj(V) at -g, because the sky is real and
  V(-U) = conj V(U) (Eq. 4), so the gridded plane is Hermitian by construction;
* a visibility is kept only if both g and -g lie on the grid, i.e. every
  component satisfies |g| < n/2; the rest are counted as dropped;
* GAUSS7: w~(U_g - U_i) = exp(-pi^2 theta_0^2 |U_g - U_i|^2) (the Gaussian aperture of
  Eq. A6 without its pi theta_0^2 prefactor) on the 7 x 7 cells around the nearest
  one; N_g = sum of those weights.

Pins: tests/test_oracle_gridding.py (hand-placed visibilities, Hermitian
symmetry, count conservation, the kernel's value at one cell offset).
"""
import numpy as np

NEAREST, GAUSS7 = 0, 1


def grid_visibilities(n, du, uv, vis, vis_w=None, kernel=NEAREST, theta0=None):
    """Return (grid complex128 [n][n], wsum float64 [n][n], dropped count)."""
    uv = np.asarray(uv, dtype=np.float64).reshape(-1, 2)
    vis = np.asarray(vis).astype(np.complex128).reshape(-1)
    w = np.ones(len(vis)) if vis_w is None else np.asarray(vis_w, dtype=np.float64)
    gx = np.rint(uv[:, 0] / du).astype(np.int64)
    gy = np.rint(uv[:, 1] / du).astype(np.int64)
    half = n // 2
    keep = (np.abs(gx) < half) & (np.abs(gy) < half)
    grid = np.zeros((n, n), np.complex128)
    wsum = np.zeros((n, n), np.float64)
    if kernel == NEAREST:
        offs = [(0, 0)]
    elif kernel == GAUSS7:
        offs = [(dx, dy) for dy in range(-3, 4) for dx in range(-3, 4)]
    else:
        raise ValueError("unknown gridding kernel")
    for dx, dy in offs:
        cx, cy = gx + dx, gy + dy
        ok = keep & (np.abs(cx) < half) & (np.abs(cy) < half)
        if kernel == NEAREST:
            kw = np.ones(len(vis))
        else:
            ddx = cx * du - uv[:, 0]
            ddy = cy * du - uv[:, 1]
            kw = np.exp(-np.pi ** 2 * theta0 ** 2 * (ddx ** 2 + ddy ** 2))
        c = (kw * w)[ok]
        v = vis[ok]
        np.add.at(grid, (cy[ok] % n, cx[ok] % n), c * v)
        np.add.at(grid, ((-cy[ok]) % n, (-cx[ok]) % n), c * np.conj(v))
        np.add.at(wsum, (cy[ok] % n, cx[ok] % n), c)
        np.add.at(wsum, ((-cy[ok]) % n, (-cx[ok]) % n), c)
    return grid, wsum, int((~keep).sum())
