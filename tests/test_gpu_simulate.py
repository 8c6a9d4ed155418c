"""GPU parity of the Eq. (4) front-end (abs_simulate: a type-2 non-uniform FFT) against the
direct-summation oracle, and of the whole chain simulate -> abs_grid -> abs_estimate
against the oracle's chain.  Gate: every |V - V*| <= 1e-5 of the rms of V* (the kernel's
own error is about 1e-7 of sum |f|, the FP32 transforms about 1e-6 of the rms)."""
import numpy as np
import pytest

from oracle import estimator as oest
from oracle import gridding as ogrid
from oracle import plan as oplan
from oracle import simulate as osim
from oracle import theory

pytestmark = pytest.mark.gpu
VTOL = 1e-5


def _run(sky, dth, uv, beam, par, q=1.0):
    import torch
    import paper_2412_02246_amd as A
    s = torch.from_numpy(np.ascontiguousarray(sky, dtype=np.float32)).cuda()
    u = torch.from_numpy(np.ascontiguousarray(uv, dtype=np.float64)).cuda()
    V = A.simulate(s, dth, u, beam=beam, beam_param=par, q=q)
    torch.cuda.synchronize()
    return V.cpu().numpy().astype(np.complex128)


def _check(V, ref, label):
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.abs(V - ref) / rms
    print("%s: max |V - V*| / rms %.3g, median %.3g, nvis %d" % (label, err.max(), np.median(err), len(V)), flush=True)
    assert err.max() <= VTOL, (label, err.max())


@pytest.mark.parametrize("nsky", [16, 64, 256])
@pytest.mark.parametrize("beam", [0, 1, 2])
def test_simulate_matches_direct_sum(nsky, beam):
    rng = np.random.default_rng(100 * nsky + beam)
    dth = 0.004
    par = {0: 0.0, 1: 1.0 / (0.4 * nsky * dth), 2: 0.2 * nsky * dth}[beam]
    sky = rng.standard_normal((2, nsky, nsky)).astype(np.float32).astype(np.float64)
    # baselines over the whole period 1/dtheta and a little beyond (the sum is periodic)
    uv = rng.uniform(-0.6 / dth, 0.6 / dth, (1500, 2))
    uv[:8] = [[0, 0], [0.5 / dth, 0], [-0.5 / dth, 0.25 / dth], [1.0 / (nsky * dth), 0],
              [3.0 / (nsky * dth), -5.0 / (nsky * dth)], [1e-3, -1e-3], [0.4999 / dth, 0.4999 / dth], [7.3, -2.1]]
    V = _run(sky, dth, uv, beam, par, q=2.5)
    for b in range(2):
        ref = osim.visibilities(sky[b], dth, uv, beam, par, q=2.5)
        _check(V[b], ref, "nsky %d beam %d [%d]" % (nsky, beam, b))


def test_point_source_sky():
    """One bright pixel: |V| is constant over all baselines (sharpest test of the kernel's
    deconvolution at the edge of the sky)."""
    nsky, dth = 128, 0.003
    sky = np.zeros((1, nsky, nsky))
    sky[0, 3, nsky - 2] = 5.0
    rng = np.random.default_rng(7)
    uv = rng.uniform(-0.5 / dth, 0.5 / dth, (2000, 2))
    V = _run(sky, dth, uv, 0, 0.0)
    ref = osim.visibilities(sky[0], dth, uv)
    _check(V[0], ref, "point source")


def test_paper_sky_mwa_beam():
    """The paper's simulation geometry (Sec. 3): a 4096^2 sky of 0.029 deg pixels (117 deg
    across) through the MWA tile beam of Eq. (5), baselines within U = 250 wavelengths;
    200 baselines against the direct sum."""
    nsky, dth = 4096, np.deg2rad(0.029)
    d_lam = theory.DISH_M * theory.NU_HZ / theory.C_LIGHT
    rng = np.random.default_rng(11)
    sky = rng.standard_normal((1, nsky, nsky)).astype(np.float32).astype(np.float64)
    r = 250.0 * np.sqrt(rng.uniform(0, 1, 200))
    ph = rng.uniform(0, 2 * np.pi, 200)
    uv = np.stack([r * np.cos(ph), r * np.sin(ph)], axis=1)
    V = _run(sky, dth, uv, 1, d_lam)
    ref = osim.visibilities(sky[0], dth, uv, osim.BEAM_MWA, d_lam, chunk=50)
    _check(V[0], ref, "4096^2 MWA beam")


def test_chain_simulate_grid_estimate():
    """Sky -> visibilities (Eq. 4, Gaussian beam) -> nearest-cell gridding (Eq. 9) -> the
    estimator (Eqs. 10-12) on the GPU, against the same chain in the oracle.  A relative
    visibility error delta moves each triple product by at most about 3 delta, so the gate
    on e_t is 3 VTOL plus the estimator's own FP32 gate."""
    import torch
    import paper_2412_02246_amd as A
    n, nsky, dth = 128, 256, 1.0 / 256
    rng = np.random.default_rng(21)
    # a smooth sky: white noise low-passed in Fourier space
    k = np.fft.fftfreq(nsky)
    lp = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2 * 0.08 ** 2))
    sky = np.fft.ifft2(np.fft.fft2(rng.standard_normal((nsky, nsky))) * lp).real
    sky = sky.astype(np.float32).astype(np.float64)
    e = oplan.log_edges(3.0, 40.0, 10)
    nvis = 20000
    rad = e[-1] * np.sqrt(rng.uniform(0, 1, nvis))
    ph = rng.uniform(0, 2 * np.pi, nvis)
    uv = np.stack([rad * np.cos(ph), rad * np.sin(ph)], axis=1)
    Vg = _run(sky[None], dth, uv, 2, 0.3)[0]
    p = A.Plan(n, e, wmode=A.W_INV_COUNT).bind()
    uv_d = torch.from_numpy(uv).cuda()
    g, w, _ = p.grid(uv_d, torch.from_numpy(Vg.astype(np.complex64)).cuda())
    B, N = p.estimate(g, w)
    torch.cuda.synchronize()
    Vo = osim.visibilities(sky, dth, uv, osim.BEAM_GAUSS, 0.3)
    _check(Vg, Vo, "chain visibilities")
    go, wo, _ = ogrid.grid_visibilities(n, 1.0, uv, Vo)
    ref = oest.estimate(go, wo, e, p.norm, wmode=oest.INV_COUNT, trips=p.triplets, with_scales=True)
    Bg = B[0].cpu().numpy()
    keep = ~np.isnan(ref["B"])
    assert np.array_equal(np.isnan(Bg), ~keep)
    et = oest.relative_error(Bg, ref, p.norm)[keep]
    print("chain: max e_t %.3g median %.3g over %d triplets" % (et.max(), np.median(et), keep.sum()), flush=True)
    assert et.max() <= 3 * VTOL + 1e-5
