"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only draws inputs: sky fields, sampling masks, noise and visibility
streams.  It holds none of the estimator's arithmetic (no ring masks, no ring
fields, no triangle sums), so the oracle and the GPU path stay independent.

Recipes (stand-ins for the paper's simulated MWA data, which is not public):
* Gaussian random field on an n x n periodic pixel grid: white N(0,1) pixels,
  forward FFT, times sqrt(C(g)), inverse FFT.  Then E|phi_hat(g)|^2 = n^2 C(g).
* local quadratic non-Gaussianity (Sec. 3, Eq. 13): delta = phi + f (phi^2 - sigma^2),
  with sigma^2 the ensemble variance of phi; gridded visibilities V = fft2(delta).
* spectra: the paper's validation C_l = (l / l_0)^-1 exp(-l^2 / (pi l_0)^2), l_0 = 1000,
  with l = 2 pi |g| du; or a pure power law C proportional to l^-2.
* baseline-density mask: N_g ~ Poisson(lam0 exp(-|g| / U0)) drawn on one half plane and
  mirrored (N_-g = N_g); thermal noise: Hermitian complex Gaussian of per-cell
  variance E|S_g|^2 / snr^2; the gridded sum is V_g = N_g (S_g + n_g).
* visibility streams for gridding: baselines with density proportional to
  exp(-|U| / U0) inside |U| < rmax, complex-normal values.
"""
import numpy as np

SEED_BASE = 20241202


def seed_for(config_index, realisation):
    return SEED_BASE + 1000 * int(config_index) + int(realisation)


def signed_freq(n):
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def radius_grid(n):
    g = signed_freq(n).astype(np.float64)
    return np.sqrt(g[:, None] ** 2 + g[None, :] ** 2)


def paper_spectrum(n, du=1.0, ell0=1000.0):
    ell = 2.0 * np.pi * du * radius_grid(n)
    with np.errstate(divide="ignore"):
        c = np.where(ell > 0, (ell0 / np.where(ell > 0, ell, 1.0)) * np.exp(-ell ** 2 / (np.pi * ell0) ** 2), 0.0)
    return c


def powerlaw_spectrum(n, sigma, du=1.0):
    """C proportional to l^-2 (C(0) = 0), scaled so the pixel rms is sigma."""
    ell = 2.0 * np.pi * du * radius_grid(n)
    with np.errstate(divide="ignore"):
        c = np.where(ell > 0, 1.0 / np.where(ell > 0, ell, 1.0) ** 2, 0.0)
    var = c.sum() / n ** 2
    return c * (sigma ** 2 / var)


def field_variance(C):
    n = C.shape[0]
    return C.sum() / n ** 2


def gaussian_field(C, rng):
    n = C.shape[0]
    white = rng.standard_normal((n, n))
    return np.fft.ifft2(np.fft.fft2(white) * np.sqrt(C)).real


def local_quadratic(phi, f, sigma2):
    return phi + f * (phi * phi - sigma2)


def hermitian_noise(var, rng):
    """Hermitian complex Gaussian noise with E|n_g|^2 = var[g]."""
    n = var.shape[0]
    white = rng.standard_normal((n, n))
    return np.fft.fft2(white) * np.sqrt(var / n ** 2)


def symmetrize(A):
    """Make A(-g) = A(g): the cell with the smaller linear index keeps its draw."""
    n = A.shape[0]
    neg = (-np.arange(n)) % n
    L = np.arange(n)[:, None] * n + np.arange(n)[None, :]
    Lm = neg[:, None] * n + neg[None, :]
    return np.where(L <= Lm, A, A[neg[:, None], neg[None, :]])


def poisson_counts(n, lam0, U0, rng):
    r = radius_grid(n)
    return symmetrize(rng.poisson(lam0 * np.exp(-r / U0)).astype(np.float64))


def nongaussian_grid(C, f, rng):
    """Visibilities V = fft2(phi + f (phi^2 - sigma^2)) for one realisation."""
    sigma2 = field_variance(C)
    phi = gaussian_field(C, rng)
    return np.fft.fft2(local_quadratic(phi, f, sigma2))


def mwa_like(n, seed, du=1.0, f_ng=0.17, lam0=4.0, U0=None, snr=5.0, counts=None):
    """One MWA-shaped channel: signal with the paper's C_l and f = f_NG / sigma_T,
    Poisson baseline counts, thermal noise at amplitude SNR ``snr`` per cell.
    Returns (V complex128 [n][n] = N_g (S + noise), counts float64 [n][n])."""
    rng = np.random.default_rng(seed)
    U0 = n / 8.0 if U0 is None else U0
    C = paper_spectrum(n, du)
    sigma = np.sqrt(field_variance(C))
    S = nongaussian_grid(C, f_ng / sigma, rng)
    if counts is None:
        counts = poisson_counts(n, lam0, U0, rng)
    noise = hermitian_noise(n ** 2 * C / snr ** 2, rng)
    V = counts * (S + noise)
    return V, counts


def visibility_stream(nvis, rmax, U0, du, seed, batch=1):
    """(uv float64 [nvis][2] in wavelengths, vis complex64 [batch][nvis])."""
    rng = np.random.default_rng(seed)
    # radius density proportional to r exp(-r / U0) on [0, rmax): rejection from a gamma(2)
    r = np.empty(0)
    while len(r) < nvis:
        c = rng.gamma(2.0, U0, size=2 * nvis)
        r = np.concatenate([r, c[c < rmax]])
    r = r[:nvis]
    phi = rng.uniform(0.0, 2.0 * np.pi, nvis)
    uv = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1) * du
    vis = (rng.standard_normal((batch, nvis)) + 1j * rng.standard_normal((batch, nvis))).astype(np.complex64)
    return uv, vis


def mwa_visibilities(n, nvis, rmax, seed, batch=1, du=1.0, f_ng=0.17, U0=None, snr=5.0):
    """Visibilities of an MWA-shaped channel on one shared baseline set: ``batch``
    independent sky realisations (the paper's C_l, local quadratic with f = f_NG/sigma_T)
    sampled at the cell nearest to each baseline, plus thermal noise per visibility
    at amplitude SNR ``snr``.  Baselines: density proportional to exp(-|U|/U0) inside
    |U| < rmax, U0 = n/8 by default.  Returns (uv float64 [nvis][2], vis complex64
    [batch][nvis])."""
    U0 = n / 8.0 if U0 is None else U0
    uv, _ = visibility_stream(nvis, rmax, U0, du, seed, batch=1)
    rng = np.random.default_rng(seed + 7919)
    C = paper_spectrum(n, du)
    sigma = np.sqrt(field_variance(C))
    gx = np.rint(uv[:, 0] / du).astype(np.int64) % n
    gy = np.rint(uv[:, 1] / du).astype(np.int64) % n
    amp = np.sqrt(n ** 2 * C[gy, gx]) / snr
    vis = np.empty((batch, nvis), np.complex64)
    for b in range(batch):
        S = nongaussian_grid(C, f_ng / sigma, rng)
        noise = (rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)) * (amp / np.sqrt(2.0))
        vis[b] = (S[gy, gx] + noise).astype(np.complex64)
    return uv, vis


def mwa_visibilities_device(n, nvis, rmax, seed, batch=1, du=1.0, f_ng=0.17, U0=None, snr=5.0,
                            device="cuda"):
    """The recipe of ``mwa_visibilities`` drawn with torch on a device (for workloads too
    large to draw on the host in reasonable time): baselines with radius density
    proportional to r exp(-r / U0) on [0, rmax) (a gamma(2) radius, the sum of two
    exponentials, redrawn where it falls outside) and uniform angle; per realisation a
    Gaussian sky with the paper's C_l, the local quadratic term with f = f_NG / sigma_T,
    sampled at each baseline's nearest cell, plus complex thermal noise at amplitude SNR
    ``snr``.  Seeded by a torch generator on the device; the draws differ from the numpy
    recipe's.  Returns (uv float64 [nvis][2], vis complex64 [batch][nvis]) on the device."""
    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    U0 = n / 8.0 if U0 is None else U0
    f64 = torch.float64
    r = torch.empty(nvis, dtype=f64, device=dev)
    todo = torch.arange(nvis, device=dev)
    while todo.numel():
        e = torch.empty((2, todo.numel()), dtype=f64, device=dev).exponential_(1.0, generator=g)
        c = U0 * (e[0] + e[1])
        ok = c < rmax
        r[todo[ok]] = c[ok]
        todo = todo[~ok]
    phi = torch.rand(nvis, dtype=f64, device=dev, generator=g) * (2.0 * np.pi)
    uv = torch.stack([r * torch.cos(phi), r * torch.sin(phi)], dim=1) * du
    del r, phi, todo
    C = torch.from_numpy(paper_spectrum(n, du)).to(dev)
    var = C.sum() / n ** 2
    f = f_ng / float(torch.sqrt(var))
    gx = torch.remainder(torch.round(uv[:, 0] / du).long(), n)
    gy = torch.remainder(torch.round(uv[:, 1] / du).long(), n)
    lin = gy * n + gx
    amp = (torch.sqrt(n ** 2 * C.reshape(-1)[lin]) / snr / np.sqrt(2.0)).float()
    sq = torch.sqrt(C)
    vis = torch.empty((batch, nvis), dtype=torch.complex64, device=dev)
    for b in range(batch):
        white = torch.randn((n, n), dtype=f64, device=dev, generator=g)
        phi_s = torch.fft.ifft2(torch.fft.fft2(white) * sq).real
        S = torch.fft.fft2(phi_s + f * (phi_s * phi_s - var)).reshape(-1)
        noise = torch.randn((2, nvis), dtype=torch.float32, device=dev, generator=g) * amp
        vis[b] = S[lin].to(torch.complex64) + torch.complex(noise[0], noise[1])
        del white, phi_s, S, noise
    return uv.contiguous(), vis
