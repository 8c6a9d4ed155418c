"""Pins of oracle.estimator (Eqs. 10-12) against direct triangle enumeration,
exact integer counts, symmetries and a Parseval special case."""
import numpy as np
import pytest

from oracle import brute, estimator, plan

UNIT, INV, GIVEN = estimator.UNIT, estimator.INV_COUNT, estimator.GIVEN


def _random_case(n, seed, hermitian=False):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if hermitian:
        V = estimator.hermitian_part(V)
    Wraw = rng.uniform(0.2, 2.0, (n, n))
    W = 0.5 * (Wraw + estimator.mirror(Wraw))     # weights are symmetric
    return V, W


CASES = [
    (8, [1.0, 1.6, 2.3]),
    (16, [1.0, 2.0, 3.1, 4.2, 5.3]),
    (32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]),
]


@pytest.mark.parametrize("n,edges", CASES)
def test_fft_equals_brute_force_planar(n, edges):
    # edges[-1] <= n/3: cyclic and planar closure coincide
    V, W = _random_case(n, n)
    trips = plan.prefilter_triplets(edges)
    out = estimator.estimate(V, W, edges, 1.0, wmode=GIVEN, trips=trips)
    X = estimator.hermitian_part(W * V)
    Y = estimator.hermitian_part(W.astype(complex))
    S_b = brute.triangle_sums(X, n, edges, trips, cyclic=False)
    N_b = brute.triangle_sums(Y, n, edges, trips, cyclic=False)
    scale = np.abs(X).max() ** 3 * max(1, len(trips))
    assert np.allclose(out["S"], S_b.real, rtol=1e-10, atol=1e-12 * scale)
    assert np.allclose(out["N"], N_b.real, rtol=1e-10, atol=1e-12 * scale)
    # the imaginary part of the triangle sum of a Hermitian field vanishes
    assert np.all(np.abs(S_b.imag) <= 1e-10 * np.abs(X).max() ** 3 * 1e3)


@pytest.mark.parametrize("n,edges", [(8, [1.0, 2.2, 3.9]), (16, [2.0, 4.5, 7.9])])
def test_fft_equals_brute_force_cyclic(n, edges):
    # rings beyond n/3: the FFT closes triangles modulo n
    V, W = _random_case(n, 100 + n)
    trips = plan.prefilter_triplets(edges)
    out = estimator.estimate(V, W, edges, 1.0, wmode=GIVEN, trips=trips)
    X = estimator.hermitian_part(W * V)
    S_c = brute.triangle_sums(X, n, edges, trips, cyclic=True)
    S_p = brute.triangle_sums(X, n, edges, trips, cyclic=False)
    assert np.allclose(out["S"], S_c.real, rtol=1e-10, atol=1e-9)
    assert not np.allclose(out["S"], S_p.real, rtol=1e-6)


@pytest.mark.parametrize("n,edges", CASES)
def test_unit_counts_are_brute_force_integers(n, edges):
    trips = plan.prefilter_triplets(edges)
    c_fft = plan.unit_counts(n, edges, trips)
    c_b = brute.triangle_counts(n, edges, trips, cyclic=False)
    assert c_fft.tolist() == c_b.tolist()
    out = estimator.estimate(np.ones((n, n)), None, edges, 1.0, wmode=UNIT, trips=trips)
    assert np.allclose(out["N"], c_b, atol=1e-8)


def test_weight_modes():
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    rng = np.random.default_rng(5)
    cnt = rng.integers(0, 4, (n, n)).astype(float)
    cnt = np.maximum(cnt, estimator.mirror(cnt))
    W = estimator.effective_weights(n, cnt, INV)
    assert np.all(W[cnt == 0] == 0) and np.allclose(W[cnt > 0], 1 / cnt[cnt > 0])
    V, _ = _random_case(n, 7)
    a = estimator.estimate(V, cnt, edges, 1.0, wmode=INV)
    b = estimator.estimate(V, W, edges, 1.0, wmode=GIVEN)
    assert np.allclose(a["B"], b["B"], equal_nan=True)


def _B(V, W, edges, n):
    trips, _ = plan.plan_triplets(n, edges)    # triplets with closed lattice triangles
    return estimator.estimate(V, W, edges, 1.0, wmode=GIVEN, trips=trips)["B"]


def test_invariants():
    n, edges = 32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]
    V, W = _random_case(n, 11, hermitian=True)
    B0 = _B(V, W, edges, n)
    g = plan.signed_index(n)
    # 90-degree rotation of the uv plane: (gx, gy) -> (-gy, gx); rings are invariant
    rot = lambda A: A[np.ix_(g % n, (-g) % n)].T
    assert np.allclose(_B(rot(V), rot(W), edges, n), B0, rtol=1e-9, atol=0)
    # reflection gx -> -gx
    ref = lambda A: A[:, (-np.arange(n)) % n]
    assert np.allclose(_B(ref(V), ref(W), edges, n), B0, rtol=1e-9)
    # integer sky shift: V(g) exp(-2 pi i g.s / n) leaves every closed triangle unchanged
    s = (5, -3)
    ph = np.exp(-2j * np.pi * (g[None, :] * s[0] + g[:, None] * s[1]) / n)
    assert np.allclose(_B(V * ph, W, edges, n), B0, rtol=1e-9)
    # V -> c V scales B by c^3, W -> c W leaves B unchanged
    assert np.allclose(_B(1.7 * V, W, edges, n), 1.7 ** 3 * B0, rtol=1e-9)
    assert np.allclose(_B(V, 3.0 * W, edges, n), B0, rtol=1e-9)


def test_permutation_symmetry():
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    V, W = _random_case(n, 3, hermitian=True)
    masks = plan.ring_masks(n, edges)
    D = estimator.ring_fields(estimator.hermitian_part(W * V), masks)
    trips = plan.prefilter_triplets(edges)
    ref = estimator.triple_sums(D, trips)
    for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)):
        pt = [tuple(t[p] for p in perm) for t in trips]
        # triple_sums indexes pair (i, j) then k: permuting the roles must not matter
        pt = [tuple(sorted(t[:2])) + (t[2],) for t in pt]
        assert np.allclose(estimator.triple_sums(D, pt), ref, rtol=1e-10, atol=1e-9)


def test_parseval_with_dc_ring():
    # A ring holding only g = 0 with X(0) = Y(0) = 1: S_{0,i,i} = sum_{a_i} |X|^2,
    # N_{0,i,i} = sum_{a_i} Y^2, and S_{0,i,j} = 0 for disjoint rings i != j.
    n = 16
    edges = [0.0, 0.5, 2.0, 3.5, 5.0]
    V, W = _random_case(n, 21)
    V[0, 0] = 1.0
    W[0, 0] = 1.0
    trips = [(0, 1, 1), (0, 2, 2), (0, 3, 3), (0, 1, 2), (0, 2, 3)]
    out = estimator.estimate(V, W, edges, 1.0, wmode=GIVEN, trips=trips)
    X = estimator.hermitian_part(W * V)
    Y = estimator.hermitian_part(W.astype(complex)).real
    masks = plan.ring_masks(n, edges)
    for q, (i, j, k) in enumerate(trips):
        if j == k:
            assert np.isclose(out["S"][q], np.sum(np.abs(X[masks[j]]) ** 2), rtol=1e-10)
            assert np.isclose(out["N"][q], np.sum(Y[masks[j]] ** 2), rtol=1e-10)
        else:
            assert abs(out["S"][q]) < 1e-9 and abs(out["N"][q]) < 1e-9


def test_noise_scale_metric_is_zero_for_exact_values():
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    V, W = _random_case(n, 2, hermitian=True)
    ref = estimator.estimate(V, W, edges, 2.5, wmode=GIVEN, with_scales=True)
    assert np.all(estimator.relative_error(ref["B"], ref, 2.5) == 0)
    e = estimator.relative_error(ref["B"] * (1 + 1e-6), ref, 2.5)
    assert np.all(e <= 1.0000001e-6)


def test_subset_estimate_matches_full():
    n, edges = 32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]
    V, W = _random_case(n, 31, hermitian=True)
    trips, _ = plan.plan_triplets(n, edges)
    full = estimator.estimate(V, W, edges, 2.0, wmode=GIVEN, trips=trips, with_scales=True)
    sub = trips[::3]
    part = estimator.estimate_subset(V, W, edges, 2.0, sub, wmode=GIVEN)
    for key in ("S", "N", "B", "rhoS", "rhoN"):
        assert np.allclose(part[key], full[key][::3], rtol=1e-10, atol=1e-12), key


@pytest.mark.parametrize("n,edges", CASES)
def test_complex_input_equals_brute_force(n, edges):
    """General complex input (no Hermitian symmetrisation): the complex triangle sum of
    X = W V by direct enumeration, for the FFT route of estimate_complex."""
    V, W = _random_case(n, 300 + n)
    trips = plan.prefilter_triplets(edges)
    out = estimator.estimate_complex(V, W, edges, 1.0, wmode=GIVEN, trips=trips)
    X = W * V
    S_b = brute.triangle_sums(X, n, edges, trips, cyclic=False)
    scale = np.abs(X).max() ** 3 * max(1, len(trips))
    assert np.allclose(out["S"], S_b, rtol=1e-10, atol=1e-12 * scale)
    assert np.any(np.abs(S_b.imag) > 1e-3 * np.abs(S_b.real).max())   # genuinely complex


def test_complex_input_reduces_to_the_hermitian_estimator():
    n, edges = 32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]
    V, W = _random_case(n, 77, hermitian=True)
    trips = plan.prefilter_triplets(edges)
    c = estimator.estimate_complex(V, W, edges, 0.3, wmode=GIVEN, trips=trips)
    r = estimator.estimate(V, W, edges, 0.3, wmode=GIVEN, trips=trips)
    ok = ~np.isnan(r["B"])
    assert np.allclose(c["B"].real[ok], r["B"][ok], rtol=1e-9, atol=1e-12 * np.abs(r["B"][ok]).max())
    assert np.all(np.abs(c["B"].imag[ok]) <= 1e-9 * np.abs(r["B"][ok]).max())
    # scaling by a complex constant multiplies B by its cube
    z = 0.7 - 1.3j
    c2 = estimator.estimate_complex(z * V, W, edges, 0.3, wmode=GIVEN, trips=trips)
    assert np.allclose(c2["B"][ok], z ** 3 * c["B"][ok], rtol=1e-9)


def test_half_plane_input_gives_the_full_plane_estimate():
    """Grids and weights supplied on a half plane only (one cell of every (g, -g) pair, the
    other zero): their Hermitian parts are half the full ones on every ring cell, S_t and N_t
    scale by 1/8 and B_t is unchanged."""
    n, edges = 32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]
    V, W = _random_case(n, 5, hermitian=True)
    g = plan.signed_index(n)
    gx, gy = np.meshgrid(g, g)
    half = (gy > 0) | ((gy == 0) & (gx > 0))
    trips = plan.prefilter_triplets(edges)
    full = estimator.estimate(V, W, edges, 1.0, wmode=GIVEN, trips=trips)
    hp = estimator.estimate(np.where(half, V, 0), np.where(half, W, 0), edges, 1.0, wmode=GIVEN, trips=trips)
    ok = ~np.isnan(full["B"])
    assert np.allclose(hp["N"], full["N"] / 8, rtol=1e-10, atol=1e-12 * np.abs(full["N"]).max())
    assert np.allclose(hp["B"][ok], full["B"][ok], rtol=1e-9, atol=1e-12 * np.abs(full["B"][ok]).max())
