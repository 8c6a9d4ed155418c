"""Pins of the oracle against numbers printed in the paper and the closed-form
bispectrum of the local quadratic model (Eq. 14, derived in App. B)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import estimator, plan, theory

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _close(name, x):
    g = GOLD[name]
    assert abs(x - g["value"]) <= g["tol"], (name, x, g)


def test_printed_constants():
    _close("theta_F_deg", theory.mwa_fwhm_deg())
    _close("dU_g", theory.grid_spacing())
    _close("off_closure_factor", theory.off_closure_factor())
    _close("ell_at_U250", 2 * np.pi * 250)
    _close("ell_at_U100", 2 * np.pi * 100)
    # the normalisation A = pi theta_0^2 / 3 with theta_0 = 0.6 theta_F
    assert np.isclose(theory.norm_A(), np.pi * (0.6 * np.deg2rad(24.68)) ** 2 / 3)


def test_paper_ring_scheme():
    e = theory_edges = plan.paper_ring_edges()
    _close("ring_count", len(e) - 1)
    assert e[0] == 1 and e[1] == 5 and e[10] == 50 and e[15] == 100 and e[20] == 200 and e[22] == 250
    ell = 2 * np.pi * theory.grid_spacing() * plan.mean_radius(1024, theory_edges)
    _close("smallest_ring_ell", ell[0])
    _close("third_ring_ell", ell[2])


def test_equilateral_special_case():
    c = np.array([0.3, 1.7, 2.0])
    assert np.allclose(theory.b_ana(c, c, c, 0.17), GOLD["equilateral_factor"]["value"] * 0.17 * c ** 2)


def test_labels_in_allowed_region():
    n = 1024
    e = plan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)
    trips = np.array(plan.prefilter_triplets(e))
    lab = plan.labels(n, e, trips)
    l1, l2, l3, mu, t = lab.T
    assert np.all(l1 >= l2) and np.all(l2 >= l3)
    tri = l3 >= l1 - l2          # the mean radii themselves close a triangle
    lo, hi = GOLD["mu_t_range"]["lo"], GOLD["mu_t_range"]["hi"]
    assert tri.sum() > 0.5 * len(trips)   # near-degenerate triplets need not close on mean radii
    assert np.all((mu[tri] >= lo - 1e-12) & (mu[tri] <= hi + 1e-12))
    assert np.all((t >= lo - 1e-12) | (mu > 1))   # t >= 0.5 wherever a triangle exists
    assert np.all(2 * mu[tri] * t[tri] >= 1 - 1e-12)
    eq = (trips[:, 0] == trips[:, 1]) & (trips[:, 1] == trips[:, 2])
    assert np.allclose(mu[eq], 0.5) and np.allclose(t[eq], 1.0)


def _ensemble(f, R, seed):
    n = 128
    e = plan.log_edges(2.0, 42.0, 8)
    trips, _ = plan.plan_triplets(n, e)
    C = synth.powerlaw_spectrum(n, 0.05)
    rng = np.random.default_rng(seed)
    B = np.array([estimator.estimate(synth.nongaussian_grid(C, f, rng), None, e, float(n * n),
                                     wmode=estimator.UNIT, trips=trips)["B"] for _ in range(R)])
    return n, e, trips, C, B


def test_closed_form_local_quadratic():
    """E[B-hat] = [B_Ana]_d (Eq. 14 averaged over each triplet's lattice triangles),
    with the synthetic normalisation A = Omega = n^2 in pixel units (Eqs. 1-3)."""
    R = 512
    n, e, trips, C, B = _ensemble(1.0, R, synth.seed_for(0, 0))
    pred = theory.b_ana_discrete(n, e, trips, C, 1.0)
    se = B.std(0, ddof=1) / np.sqrt(R)
    z = (B.mean(0) - pred) / se
    assert np.median(np.abs(z)) <= 1.0, np.median(np.abs(z))
    assert np.abs(z).max() <= 4.5, np.abs(z).max()
    # the same data rejects a prediction with a wrong factor or sign
    for wrong in (0.8 * pred, -pred):
        assert np.median(np.abs((B.mean(0) - wrong) / se)) > 1.5


def test_zero_mean_gaussian():
    """Odd moments of a Gaussian field vanish (App. B), so E[B-hat] = 0 for f = 0."""
    R = 384
    _, _, _, _, B = _ensemble(0.0, R, synth.seed_for(0, 5000))
    z = B.mean(0) / (B.std(0, ddof=1) / np.sqrt(R))
    assert np.median(np.abs(z)) <= 1.0
    assert np.abs(z).max() <= 4.5


def test_validation_spectrum_values():
    """Sec. 3's C_l = (l / l0)^-1 exp(-l^2 / (pi l0)^2) with l0 = 1000: C(l0) = exp(-1 / pi^2),
    C(2 l0) = exp(-4 / pi^2) / 2, and the ratio of two small-l values is the power law's
    times the Gaussian's."""
    assert np.isclose(theory.cl_model(1000.0), np.exp(-1.0 / np.pi ** 2), rtol=1e-14)
    assert np.isclose(theory.cl_model(2000.0), 0.5 * np.exp(-4.0 / np.pi ** 2), rtol=1e-14)
    r = theory.cl_model(10.0) / theory.cl_model(20.0)
    assert np.isclose(r, 2.0 * np.exp((400.0 - 100.0) / (np.pi * 1000.0) ** 2), rtol=1e-14)
