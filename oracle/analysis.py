"""Oracle: (ell1, mu, t) re-binning, ensemble statistics and deviation metrics (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Sources (Gill et al. 2024):
* Sec. 3, the paragraph after the ring scheme: the triplet estimates do not fall on a
  regular grid of (ell1, mu, t), so ell1 is divided into bins of equal logarithmic width,
  mu and t into bins of equal linear width, and the estimates in each bin are averaged,
  weighted by their number of triangles; 500 realisations give the ensemble mean B and
  the variance sigma^2 = <B-hat^2> - B^2.
* Sec. 4 (Fig. 3): the range 0.5 <= mu, t <= 1 is cut into 5 x 5 linear bins; the
  equilateral shape sits in the bin (mu, t) = (0.55, 0.95).
* Sec. 4 (Figs. 4, 5): Delta_B = |B - [B_Ana]_d| / [B_Ana]_d and
  Delta_sigma = |B - [B_Ana]_d| / sigma.

Readings where the paper is silent or ambiguous:
* the weight of a triplet is its N_t, the weighted triangle count of Eq. (12)'s
  denominator (for unit weights exactly the number of triangles).  The bin value
  sum N_t B_t / sum N_t is then Eq. (12) applied to the union of the bin's triangles;
* a triplet's (ell1, mu, t) are its plan labels (from the rings' mean radii); ell1 bins
  are half-open [lo, hi) between given edges and triplets outside them are not binned;
  mu and t take nmu and nt equal bins of [0.5, 1], half-open except the last one;
  labels below 0.5 or above 1 (mean radii of wide rings need not close a triangle)
  are clamped into the end bins;
* empty triplets (B_t NaN) are left out of every bin; a bin without triplets is NaN;
* sigma^2 is the ensemble variance as defined in Sec. 3 (mean of squares minus the
  squared mean over the R realisations, no Bessel correction);
* Delta_B divides by [B_Ana]_d, as the Sec. 4 text states (the Fig. 4 caption writes B).

Pins: tests/test_oracle_analysis.py (the paper's equilateral bin centre, hand-placed
labels, brute-force enumeration of every closed triangle of a bin, closed-form
statistics of small ensembles, the local quadratic model's binned prediction).
"""
import numpy as np


def bin_index(labels, l1_edges, nmu=5, nt=5):
    """Bin of every triplet: l1_bin * nmu * nt + mu_bin * nt + t_bin, or -1 when ell1
    lies outside the ell1 edges.  labels: [ntrip][5] (ell1, ell2, ell3, mu, t)."""
    labels = np.asarray(labels, dtype=np.float64).reshape(-1, 5)
    l1e = np.asarray(l1_edges, dtype=np.float64)
    out = np.full(len(labels), -1, dtype=np.int64)
    for q, (l1, _, _, mu, t) in enumerate(labels):
        lb = -1
        for b in range(len(l1e) - 1):
            if l1e[b] <= l1 < l1e[b + 1]:
                lb = b
                break
        if lb < 0:
            continue
        # inner edges 0.5 + 0.5 m / nbins (FP64); the bin is the number of them at or below
        mb = sum(1 for m in range(1, nmu) if mu >= 0.5 + 0.5 * m / nmu)
        tb = sum(1 for m in range(1, nt) if t >= 0.5 + 0.5 * m / nt)
        out[q] = (lb * nmu + mb) * nt + tb
    return out


def bin_centres(l1_edges, nmu=5, nt=5):
    """(ell1, mu, t) at the centre of every bin, in bin_index order (ell1: geometric mean)."""
    l1e = np.asarray(l1_edges, dtype=np.float64)
    cen = []
    for b in range(len(l1e) - 1):
        for m in range(nmu):
            for k in range(nt):
                cen.append((np.sqrt(l1e[b] * l1e[b + 1]), 0.5 + 0.5 * (m + 0.5) / nmu, 0.5 + 0.5 * (k + 0.5) / nt))
    return np.array(cen)


def rebin(B, N, bins, nbins):
    """Triangle-weighted bin averages: Bbin = sum N_t B_t / sum N_t and Nbin = sum N_t
    over the bin's non-empty triplets (NaN / 0 for a bin without any)."""
    B = np.asarray(B, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    num = np.zeros(nbins)
    den = np.zeros(nbins)
    for t in range(len(B)):
        b = bins[t]
        if b < 0 or np.isnan(B[t]):
            continue
        num[b] += N[t] * B[t]
        den[b] += N[t]
    with np.errstate(invalid="ignore", divide="ignore"):
        Bbin = np.where(den != 0, num / np.where(den != 0, den, 1.0), np.nan)
    return Bbin, den


def ensemble(X):
    """Ensemble mean and sigma (Sec. 3: sigma^2 = <X^2> - <X>^2) over axis 0."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    var = (X * X).mean(axis=0) - mean * mean
    return mean, np.sqrt(np.maximum(var, 0.0))


def deviations(mean, sigma, model):
    """Delta_B = |B - model| / model and Delta_sigma = |B - model| / sigma (Sec. 4)."""
    d = np.abs(np.asarray(mean) - np.asarray(model))
    with np.errstate(invalid="ignore", divide="ignore"):
        return d / np.asarray(model), d / np.asarray(sigma)
