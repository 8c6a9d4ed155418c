"""Oracle: visibilities of a flat-sky brightness field, Eq. (4), by direct summation
(FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Source: Gill et al. 2024, Sec. 2, Eq. (4): V(U) = Q int d^2 theta A(theta) dT(theta)
exp(i 2 pi U . theta) with the primary beam A of Eq. (5) (MWA tile, sinc^2 per axis) or
its Gaussian approximation Eq. (6); Sec. 3: the sky is simulated on a flat 2-D grid,
multiplied by A and transformed to the baselines by a DFT.

Readings of the paper where it is silent or ambiguous:
* the integral over a grid of N x N pixels of side dtheta is the pixel sum times
  dtheta^2; pixel (a, b) (a: column / theta_x, b: row / theta_y) sits at
  ((a - N/2) dtheta, (b - N/2) dtheta), so the beam centre is pixel (N/2, N/2);
* Eq. (5) is parametrised by the tile side in wavelengths, d / lambda; Eq. (6) by theta_0.

The sum is evaluated exactly as written, one baseline chunk at a time:
V = q dtheta^2 sum_b exp(2 pi i v theta_b) sum_a exp(2 pi i u theta_a) A_ab sky_ab
(the exponential factorises over the two axes; no other reordering).

Pins: tests/test_oracle_simulate.py (a point source against its closed form; on-grid
baselines against numpy's inverse FFT; Hermitian symmetry; the beam's half-power width
against the FWHM the paper prints; the Gaussian beam's value at theta_0).
"""
import numpy as np

BEAM_NONE, BEAM_MWA, BEAM_GAUSS = 0, 1, 2


def pixel_angles(nsky, dtheta):
    """Angle of every pixel index along one axis: (a - N/2) dtheta."""
    return (np.arange(nsky) - nsky // 2) * float(dtheta)


def beam(kind, theta_x, theta_y, param):
    """A(theta) of Eq. (5) (param = d / lambda) or Eq. (6) (param = theta_0), or 1."""
    tx = np.asarray(theta_x, dtype=np.float64)
    ty = np.asarray(theta_y, dtype=np.float64)
    if kind == BEAM_NONE:
        return np.ones(np.broadcast(tx, ty).shape)
    if kind == BEAM_MWA:
        return np.sinc(param * tx) ** 2 * np.sinc(param * ty) ** 2   # np.sinc(x) = sin(pi x) / (pi x)
    if kind == BEAM_GAUSS:
        return np.exp(-(tx ** 2 + ty ** 2) / param ** 2)
    raise ValueError("unknown beam")


def visibilities(sky, dtheta, uv, beam_kind=BEAM_NONE, beam_param=0.0, q=1.0, chunk=1024):
    """V(U) for every baseline (complex128 [nvis]); sky real [N][N] (row = theta_y)."""
    sky = np.asarray(sky, dtype=np.float64)
    n = sky.shape[0]
    th = pixel_angles(n, dtheta)
    A = beam(beam_kind, th[None, :], th[:, None], beam_param)      # [b][a]
    f = q * dtheta ** 2 * A * sky
    uv = np.asarray(uv, dtype=np.float64).reshape(-1, 2)
    out = np.empty(len(uv), np.complex128)
    for s in range(0, len(uv), chunk):
        u = uv[s:s + chunk, 0:1]
        v = uv[s:s + chunk, 1:2]
        Ex = np.exp(2j * np.pi * u * th[None, :])                   # [c][a]
        Ey = np.exp(2j * np.pi * v * th[None, :])                   # [c][b]
        inner = Ex @ f.T                                            # [c][b] = sum_a Ex f[b, a]
        out[s:s + chunk] = np.sum(Ey * inner, axis=1)
    return out
