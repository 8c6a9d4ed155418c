"""Pins of the Eq. (4) visibility oracle (oracle/simulate.py) against things fixed
independently of it: a point source's closed form, numpy's inverse FFT on baselines that
fall on the sky grid's reciprocal lattice, Hermitian symmetry of a real sky, and the beam
widths the paper prints (Sec. 2: FWHM 24.68 deg for a 4 m tile at 154.25 MHz)."""
import numpy as np

from oracle import simulate as osim
from oracle import theory


def test_point_source_closed_form():
    """One bright pixel s at (a0, b0): V(U) = q dtheta^2 A(theta0) s exp(2 pi i U . theta0)."""
    n, dth, q = 32, 0.01, 1.7
    a0, b0, s = 21, 9, 3.25
    sky = np.zeros((n, n))
    sky[b0, a0] = s
    th = osim.pixel_angles(n, dth)
    rng = np.random.default_rng(1)
    uv = rng.uniform(-40, 40, (50, 2))
    for kind, par in ((osim.BEAM_NONE, 0.0), (osim.BEAM_MWA, 8.2), (osim.BEAM_GAUSS, 0.07)):
        V = osim.visibilities(sky, dth, uv, kind, par, q=q)
        A0 = osim.beam(kind, th[a0], th[b0], par)
        want = q * dth ** 2 * A0 * s * np.exp(2j * np.pi * (uv[:, 0] * th[a0] + uv[:, 1] * th[b0]))
        assert np.allclose(V, want, rtol=1e-12, atol=0)


def test_reciprocal_lattice_baselines_match_inverse_fft():
    """At U = (j, k) / (N dtheta) the sum is a 2-D DFT: numpy's ifft2 of the pixel values
    (times N^2 and the phase of the centred origin)."""
    n, dth = 16, 0.02
    rng = np.random.default_rng(2)
    sky = rng.standard_normal((n, n))
    js = np.array([(j, k) for j in range(-n // 2, n // 2) for k in range(-n // 2, n // 2)])
    uv = js / (n * dth)
    V = osim.visibilities(sky, dth, uv)
    F = np.fft.ifft2(sky) * n * n          # sum_ab sky exp(+2 pi i (k b + j a) / n)
    want = dth ** 2 * F[js[:, 1] % n, js[:, 0] % n] * np.exp(-1j * np.pi * (js[:, 0] + js[:, 1]))
    assert np.allclose(V, want, rtol=1e-11, atol=1e-13)


def test_real_sky_is_hermitian_and_periodic():
    n, dth = 32, 0.015
    rng = np.random.default_rng(3)
    sky = rng.standard_normal((n, n))
    uv = rng.uniform(-30, 30, (40, 2))
    V = osim.visibilities(sky, dth, uv, osim.BEAM_MWA, 6.0)
    Vm = osim.visibilities(sky, dth, -uv, osim.BEAM_MWA, 6.0)
    assert np.allclose(Vm, np.conj(V), rtol=1e-12, atol=1e-14)
    Vp = osim.visibilities(sky, dth, uv + np.array([1.0 / dth, -2.0 / dth]), osim.BEAM_MWA, 6.0)
    assert np.allclose(Vp, V, rtol=1e-9, atol=1e-12)


def test_beam_widths_printed_in_the_paper():
    """Eq. (5) with d = 4 m at 154.25 MHz is at half power 24.68 / 2 deg off axis (the FWHM
    the paper quotes, to its printed precision); Eq. (6) is e^-1 at theta_0."""
    d_lam = theory.DISH_M * theory.NU_HZ / theory.C_LIGHT
    half = np.deg2rad(theory.THETA_F_DEG / 2)
    assert abs(osim.beam(osim.BEAM_MWA, half, 0.0, d_lam) - 0.5) < 2e-3
    assert abs(osim.beam(osim.BEAM_MWA, 0.0, half, d_lam) - 0.5) < 2e-3
    th0 = theory.theta0()
    assert np.isclose(osim.beam(osim.BEAM_GAUSS, th0, 0.0, th0), np.exp(-1.0), rtol=1e-14)
    assert osim.beam(osim.BEAM_MWA, 0.0, 0.0, d_lam) == 1.0
