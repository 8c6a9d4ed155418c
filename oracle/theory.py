"""Oracle: closed forms and constants from the paper (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

* Eq. (5): MWA tile beam A(theta) = sinc^2(pi d theta_x / lambda) sinc^2(pi d theta_y / lambda),
  d = 4 m, nu = 154.25 MHz; the paper quotes FWHM theta_F = 24.68 deg.
* Eq. (6): Gaussian approximation with theta_0 = 0.6 theta_F.
* Eq. (12): A = pi theta_0^2 / 3.
* Sec. 3: grid spacing dU_g = sqrt(ln 2) / (pi theta_0), and the off-closure factor
  exp(-pi^2 theta_0^2 dU^2 / 3) at dU^2 = dU_g^2 / 2 (the paper quotes 0.89).
* Sec. 3: validation spectrum C_l = (l / l_0)^-1 exp(-l^2 / (pi l_0)^2), l_0 = 1000.
* Eq. (14): first-order bispectrum of the local quadratic model, Eq. (13):
  B_Ana = 2 f (C1 C2 + C2 C3 + C3 C1) with f = f_NG / sigma_T.
* Sec. 4 (discussion of Fig. 2): [B_Ana]_d, the same prediction averaged over exactly
  the lattice triangles that enter each ring triplet.  Here that average is
  weighted like Eq. (12)'s denominator (by Y1 Y2 Y3) and evaluated with FFTs of
  C-weighted ring shells: sum_theta (J_i J_j I_k + I_i J_j J_k + J_i I_j J_k) / sum_theta I_i I_j I_k
  with J_m the field of Y C on ring m and I_m the field of Y on ring m.

Pins: tests/test_oracle_theory.py (numbers printed in the paper, and the
equilateral special case 6 f C^2 quoted in Sec. 4).
"""
import numpy as np

C_LIGHT = 299792458.0
THETA_F_DEG = 24.68          # Sec. 2, FWHM of the Eq. (5) beam as quoted
NU_HZ = 154.25e6             # Sec. 2 / Sec. 3 observing frequency
DISH_M = 4.0                 # Sec. 2, MWA tile size d
ELL0 = 1000.0                # Sec. 3, validation spectrum
F_NG = 0.17                  # Sec. 3


def theta0(theta_f_deg=THETA_F_DEG):
    return 0.6 * np.deg2rad(theta_f_deg)


def grid_spacing(th0=None):
    th0 = theta0() if th0 is None else th0
    return np.sqrt(np.log(2.0)) / (np.pi * th0)


def norm_A(th0=None):
    th0 = theta0() if th0 is None else th0
    return np.pi * th0 ** 2 / 3.0


def off_closure_factor(th0=None):
    th0 = theta0() if th0 is None else th0
    du = grid_spacing(th0)
    return np.exp(-np.pi ** 2 * th0 ** 2 * (du ** 2 / 2.0) / 3.0)


def mwa_beam(theta_x, theta_y, d=DISH_M, nu=NU_HZ):
    lam = C_LIGHT / nu
    def s2(t):
        x = np.pi * d * np.asarray(t, dtype=np.float64) / lam
        return np.where(x == 0, 1.0, (np.sin(x) / np.where(x == 0, 1, x)) ** 2)
    return s2(theta_x) * s2(theta_y)


def mwa_fwhm_deg(d=DISH_M, nu=NU_HZ):
    """Full width at half maximum of Eq. (5) along one axis, by bisection."""
    lo, hi = 1e-6, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mwa_beam(mid, 0.0, d, nu) > 0.5:
            lo = mid
        else:
            hi = mid
    return np.rad2deg(2.0 * 0.5 * (lo + hi))


def cl_model(ell, ell0=ELL0):
    ell = np.asarray(ell, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(ell > 0, (ell / ell0) ** -1.0 * np.exp(-ell ** 2 / (np.pi * ell0) ** 2), 0.0)


def b_ana(c1, c2, c3, f):
    return 2.0 * f * (c1 * c2 + c2 * c3 + c3 * c1)


def b_ana_discrete(n, edges, trips, C, f, Y=None, chunk=1 << 16):
    """[B_Ana]_d per triplet: Eq. (14) averaged over the triplet's closed lattice
    triangles with weight Y1 Y2 Y3 (Y = 1 when not given); NaN for a triplet without any
    weighted triangle (the empty-triplet rule of the estimator)."""
    from .plan import ring_masks
    from .estimator import min_weight
    masks = ring_masks(n, edges)
    Y = np.ones((n, n)) if Y is None else np.asarray(Y, dtype=np.float64)
    I = np.stack([np.fft.fft2(np.where(m, Y, 0.0)).real for m in masks])
    J = np.stack([np.fft.fft2(np.where(m, Y * C, 0.0)).real for m in masks])
    nb = len(masks)
    I = I.reshape(nb, -1)
    J = J.reshape(nb, -1)
    trips = [tuple(int(x) for x in t) for t in trips]
    num = np.zeros(len(trips))
    den = np.zeros(len(trips))
    for s in range(0, n * n, chunk):
        Ic, Jc = I[:, s:s + chunk], J[:, s:s + chunk]
        for q, (i, j, k) in enumerate(trips):
            num[q] += np.dot(Jc[i] * Jc[j], Ic[k]) + np.dot(Ic[i] * Jc[j], Jc[k]) + np.dot(Jc[i] * Ic[j], Jc[k])
            den[q] += np.dot(Ic[i] * Ic[j], Ic[k])
    wmin = min_weight(Y, masks)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(den < 0.5 * wmin ** 3, np.nan, 2.0 * f * num / den)
