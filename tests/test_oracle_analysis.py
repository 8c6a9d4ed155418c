"""Pins of oracle.analysis: the (ell1, mu, t) re-binning, ensemble statistics and deviation
metrics of Secs. 3-4, against the paper's printed bin layout, hand-placed labels, brute-force
enumeration of every closed triangle of a bin, and closed forms of small ensembles."""
import json
import os

import numpy as np

import synth
from oracle import analysis, brute, estimator, plan, theory

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_equilateral_bin_is_the_papers():
    nmu = nt = GOLD["mu_t_bins"]["value"]
    l1e = [10.0, 100.0]
    lab = np.array([[50.0, 50.0, 50.0, 0.5, 1.0]])           # an equilateral triplet
    b = analysis.bin_index(lab, l1e, nmu, nt)[0]
    cen = analysis.bin_centres(l1e, nmu, nt)[b]
    assert np.isclose(cen[1], GOLD["equilateral_bin_centre"]["mu"])
    assert np.isclose(cen[2], GOLD["equilateral_bin_centre"]["t"])
    assert b == 0 * nt + (nt - 1)                             # first mu bin, last t bin


def test_bin_index_hand_cases():
    l1e = [10.0, 20.0, 40.0]
    lab = np.array([
        [10.0, 9.0, 2.0, 0.99, 0.9],     # ell1 on the lower edge: first ell1 bin; mu bin 4, t bin 4
        [20.0, 15.0, 8.0, 0.70, 0.75],   # second ell1 bin; mu 0.70 -> bin 2; t 0.75 -> bin 2
        [39.9, 39.9, 1.0, 1.02, 1.0],    # mu above 1 clamps into the last bin
        [30.0, 14.0, 13.0, 0.55, 0.47],  # t below 0.5 clamps into the first bin
        [40.0, 30.0, 20.0, 0.6, 0.75],   # ell1 on the upper edge: outside
        [5.0, 5.0, 5.0, 0.5, 1.0],       # below the ell1 range: outside
    ])
    got = analysis.bin_index(lab, l1e, 5, 5)
    assert got.tolist() == [(0 * 5 + 4) * 5 + 4, (1 * 5 + 2) * 5 + 2, (1 * 5 + 4) * 5 + 4, (1 * 5 + 0) * 5 + 0, -1, -1]


def test_rebinned_value_is_the_average_over_every_triangle_of_the_bin():
    """Bin value = weighted average of X1 X2 X3 / A over all closed triangles whose triplet
    falls in the bin, each triangle weighted by Y1 Y2 Y3 (enumerated one by one)."""
    n, edges = 32, [1.5, 2.7, 4.1, 6.0, 8.2, 10.6]
    rng = np.random.default_rng(8)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    W = synth.symmetrize(rng.uniform(0.2, 2.0, (n, n)))
    trips, _ = plan.plan_triplets(n, edges)
    norm = 0.7
    est = estimator.estimate(V, W, edges, norm, wmode=estimator.GIVEN, trips=trips)
    lab = plan.labels(n, edges, trips)
    l1e = plan.log_edges(2 * np.pi * 3.0, 2 * np.pi * 11.0, 3)
    bins = analysis.bin_index(lab, l1e, 5, 5)
    nb = 3 * 25
    Bbin, Nbin = analysis.rebin(est["B"], est["N"], bins, nb)
    # every closed triangle, enumerated per triplet, pooled by bin
    X = estimator.hermitian_part(W * V)
    Y = estimator.hermitian_part(W.astype(complex))
    num = np.zeros(nb, complex)
    den = np.zeros(nb, complex)
    for q, t in enumerate(trips.tolist()):
        if bins[q] < 0:
            continue
        num[bins[q]] += brute.triangle_sums(X, n, edges, [t], cyclic=False)[0]
        den[bins[q]] += brute.triangle_sums(Y, n, edges, [t], cyclic=False)[0]
    used = den.real > 0
    assert used.sum() >= 5 and np.all(np.isnan(Bbin[~used]))
    assert np.allclose(Bbin[used], num.real[used] / (norm * den.real[used]), rtol=1e-9)
    assert np.allclose(Nbin[used], den.real[used], rtol=1e-9)


def test_empty_triplets_are_left_out():
    B = np.array([1.0, np.nan, 3.0])
    N = np.array([1.0, 1e-20, 3.0])
    Bbin, Nbin = analysis.rebin(B, N, np.array([0, 0, 0]), 2)
    assert np.isclose(Bbin[0], (1.0 + 9.0) / 4.0) and np.isclose(Nbin[0], 4.0)
    assert np.isnan(Bbin[1]) and Nbin[1] == 0.0


def test_ensemble_closed_forms():
    X = np.array([[1.0, 5.0, 2.0], [3.0, 5.0, -2.0]])
    mean, sigma = analysis.ensemble(X)
    assert np.allclose(mean, [2.0, 5.0, 0.0])
    assert np.allclose(sigma, [1.0, 0.0, 2.0])          # population sigma: |a - b| / 2
    dB, ds = analysis.deviations(mean, sigma, np.array([4.0, 4.0, 1.0]))
    assert np.allclose(dB, [0.5, 0.25, 1.0])
    assert np.allclose(ds[[0, 2]], [2.0, 0.5]) and np.isinf(ds[1])


def test_binned_local_quadratic_model():
    """128 x 128 grids of the local quadratic model (f = 1, C ~ l^-2, sigma_phi = 0.05), 8 log
    rings, unit weights: over 192 realisations the binned ensemble mean agrees with the
    binned [B_Ana]_d within its standard error, and a 0.8x prediction is rejected."""
    n, R = 128, 192
    e = plan.log_edges(2.0, 42.0, 8)
    C = synth.powerlaw_spectrum(n, 0.05)
    trips, _ = plan.plan_triplets(n, e)
    lab = plan.labels(n, e, trips)
    l1e = plan.log_edges(2 * np.pi * 2.0, 2 * np.pi * 42.0, 4)
    bins = analysis.bin_index(lab, l1e, 5, 5)
    nb = 4 * 25
    rng = np.random.default_rng(synth.seed_for(0, 500))
    Bb = []
    for r in range(R):
        V = synth.nongaussian_grid(C, 1.0, rng)
        est = estimator.estimate(V, None, e, float(n * n), trips=trips)
        Bb.append(analysis.rebin(est["B"], est["N"], bins, nb)[0])
    Bb = np.array(Bb)
    used = ~np.isnan(Bb[0])
    mean, sigma = analysis.ensemble(Bb[:, used])
    est = estimator.estimate(np.ones((n, n)), None, e, 1.0, trips=trips)
    bd = theory.b_ana_discrete(n, e, trips, C, 1.0)
    model, _ = analysis.rebin(bd, est["N"], bins, nb)
    model = model[used]
    z = np.abs(mean - model) / (sigma / np.sqrt(R))
    print("binned z: max %.2f median %.2f over %d bins" % (z.max(), np.median(z), used.sum()))
    assert used.sum() >= 8
    assert np.max(z) <= 4.0 and np.median(z) <= 1.2
    z08 = np.abs(mean - 0.8 * model) / (sigma / np.sqrt(R))
    assert np.max(z08) > 5.0
