"""Pin of the empty-triplet rule of the oracle (Eq. 12 when no closed triangle carries
weight): B_t is NaN exactly where the weighted triangle set of a triplet is empty, decided
by N_t < w_min^3 / 2, and the rule agrees with direct triangle enumeration."""
import numpy as np

from oracle import brute, estimator, plan


def _sparse_weights(n, edges):
    """Weights that leave only some cells of rings 0 and 1 weighted: ring 0 keeps the
    cells on the v axis (gx = 0), ring 1 those on the u axis (gy = 0); every other ring
    keeps unit-ish weights.  Symmetric, non-negative."""
    g = plan.signed_index(n)
    gx, gy = np.meshgrid(g, g)
    rc = plan.ring_of_cell(n, edges)
    rng = np.random.default_rng(11)
    W = estimator.hermitian_part(rng.uniform(0.5, 1.5, (n, n)).astype(complex)).real
    W[(rc == 0) & (gx != 0)] = 0.0
    W[(rc == 1) & (gy != 0)] = 0.0
    return W


def test_empty_weighted_triplets_are_nan_and_match_brute_force():
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    W = _sparse_weights(n, edges)
    trips, counts = plan.plan_triplets(n, edges)
    assert np.all(counts >= 1)                  # every plan triplet has lattice triangles
    rng = np.random.default_rng(3)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    out = estimator.estimate(V, W, edges, 1.0, wmode=estimator.GIVEN, trips=trips)
    Y = estimator.hermitian_part(W.astype(complex))
    X = estimator.hermitian_part(W * V)
    N_b = brute.triangle_sums(Y, n, edges, trips, cyclic=False).real
    S_b = brute.triangle_sums(X, n, edges, trips, cyclic=False).real
    wmin = out["wmin"]
    assert 0.5 <= wmin <= 1.5
    empty = N_b == 0.0                           # brute force: no weighted triangle at all
    # (0, 1, 1): the ring-0 cell (0, +-1) and ring-1 cells (+-2, 0) close only with
    # ring-1 cells (-+2, -+1), which carry no weight: empty despite its lattice triangles
    t011 = [q for q, t in enumerate(trips.tolist()) if t == [0, 1, 1]][0]
    assert empty[t011]
    assert empty.any() and (~empty).any()
    assert np.all(N_b[~empty] >= wmin ** 3 * (1 - 1e-12))
    assert np.array_equal(np.isnan(out["B"]), empty)
    assert np.allclose(out["B"][~empty], S_b[~empty] / N_b[~empty], rtol=1e-9)
    # the FFT route's N_t of an empty triplet is rounding noise, far below the threshold
    assert np.all(np.abs(out["N"][empty]) < 1e-9 * wmin ** 3)


def test_unit_weights_never_empty():
    n, edges = 32, [1.2, 2.0, 3.3, 5.1, 7.0, 10.5]
    trips, _ = plan.plan_triplets(n, edges)
    rng = np.random.default_rng(4)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    out = estimator.estimate(V, None, edges, 1.0, trips=trips)
    assert out["wmin"] == 1.0
    assert np.all(np.isfinite(out["B"]))


def test_subset_route_applies_the_same_rule():
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    W = _sparse_weights(n, edges)
    trips, _ = plan.plan_triplets(n, edges)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    full = estimator.estimate(V, W, edges, 1.0, wmode=estimator.GIVEN, trips=trips)
    sub = estimator.estimate_subset(V, W, edges, 1.0, trips, wmode=estimator.GIVEN)
    assert full["wmin"] == sub["wmin"]
    assert np.array_equal(np.isnan(full["B"]), np.isnan(sub["B"]))
    ok = ~np.isnan(full["B"])
    assert np.allclose(full["B"][ok], sub["B"][ok], rtol=1e-9)
