"""Pins of oracle.gridding (Eq. 9) with hand-placed visibilities."""
import numpy as np

from oracle import gridding, theory


def test_nearest_cell_and_hermitian_completion():
    n, du = 16, 1.0
    uv = np.array([[2.4, -1.2], [2.6, 0.4], [-0.5, 0.5], [9.0, 0.0], [1.5, 2.5]])
    vis = np.array([1 + 2j, 3 - 1j, 5 + 0j, 7 + 7j, 1j])
    g, w, dropped = gridding.grid_visibilities(n, du, uv, vis)
    assert dropped == 1                      # |u| = 9 >= n/2
    assert g[-1 % n, 2] == 1 + 2j            # (2.4, -1.2) -> (2, -1)
    assert g[1, -2 % n] == 1 - 2j            # its mirror carries conj(V)
    assert g[0, 3] == 3 - 1j and g[0, -3 % n] == 3 + 1j
    # round half to even: (-0.5, 0.5) -> (0, 0); V and conj(V) land on the same cell
    assert g[0, 0] == 10 and w[0, 0] == 2
    # (1.5, 2.5) -> (2, 2)
    assert g[2, 2] == 1j and g[-2 % n, -2 % n] == -1j
    assert w.sum() == 2 * (len(uv) - dropped)
    assert np.allclose(g, np.conj(g[np.ix_((-np.arange(n)) % n, (-np.arange(n)) % n)]))


def test_gauss7_kernel_weights():
    n = 32
    th0 = theory.theta0()
    du = theory.grid_spacing(th0)
    uv = np.array([[3 * du, -2 * du]])       # exactly on cell (3, -2)
    g, w, _ = gridding.grid_visibilities(n, du, uv, np.array([1.0]), kernel=gridding.GAUSS7, theta0=th0)
    # at this spacing exp(-pi^2 theta0^2 du^2 |dg|^2) = 2^-|dg|^2
    assert np.isclose(w[-2 % n, 3], 1.0)
    assert np.isclose(w[-2 % n, 4], 0.5)
    assert np.isclose(w[-1 % n, 4], 0.25)
    assert np.isclose(w[-2 % n, 6], 2.0 ** -9)
    assert w[-2 % n, 7] == 0                 # outside the 7 x 7 footprint
