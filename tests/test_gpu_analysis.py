"""GPU parity of the steps after the estimator (Secs. 3-4): the (ell1, mu, t) bin table,
triangle-weighted re-binning, ensemble mean / sigma, the model's discretely sampled
prediction [B_Ana]_d and Delta_B / Delta_sigma, each against the FP64 oracle, on the
128^2 / 8-ring local quadratic workload (unit weights) and on a weighted 256^2 plan."""
import numpy as np
import pytest

import synth
from oracle import analysis as oan
from oracle import estimator as oest
from oracle import plan as oplan
from oracle import theory

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def test_c1_rebinned_ensemble_against_the_model():
    """64 realisations of the local quadratic model (f = 1, C ~ l^-2, sigma_phi = 0.05) on
    128^2 with 8 log rings: GPU estimate -> GPU rebin -> GPU ensemble and GPU [B_Ana]_d,
    each step compared with the oracle applied to the same inputs."""
    torch = _torch()
    import paper_2412_02246_amd as A
    n, R = 128, 64
    e = oplan.log_edges(2.0, 42.0, 8)
    C = synth.powerlaw_spectrum(n, 0.05)
    rng = np.random.default_rng(synth.seed_for(0, 700))
    grids = np.stack([synth.nongaussian_grid(C, 1.0, rng) for _ in range(R)])
    p = A.Plan(n, e, norm=float(n * n), max_batch=R).bind()
    B, N = p.estimate(torch.from_numpy(grids).to(torch.complex128).cuda())
    # the bin table equals the oracle's, from the oracle's labels
    l1e = oplan.log_edges(2 * np.pi * 2.0, 2 * np.pi * 42.0, 4)
    bins, nbins = p.rebin_table(l1e)
    lab = oplan.labels(n, e, p.triplets)
    assert np.array_equal(bins, oan.bin_index(lab, l1e, 5, 5))
    bins_d = torch.from_numpy(bins).cuda()
    Bb, Nb = p.rebin(B, N, bins_d, nbins)
    Bh, Nh = B.cpu().numpy(), N.cpu().numpy()
    Bbh, Nbh = Bb.cpu().numpy(), Nb.cpu().numpy()
    # re-binning arithmetic: the oracle on the same (GPU) estimates, to FP64 rounding
    for r in (0, R - 1):
        ob, on = oan.rebin(Bh[r], Nh[r], bins, nbins)
        assert np.array_equal(np.isnan(ob), np.isnan(Bbh[r]))
        ok = ~np.isnan(ob)
        assert np.allclose(Bbh[r][ok], ob[ok], rtol=1e-13, atol=0) and np.allclose(Nbh[r], on, rtol=1e-13)
    # end to end: the oracle's own estimate of realisation 0, re-binned by the oracle
    ref = oest.estimate(grids[0], None, e, float(n * n), trips=p.triplets, with_scales=True)
    ob, _ = oan.rebin(ref["B"], ref["N"], bins, nbins)
    ok = ~np.isnan(ob)
    scale = np.abs(ob[ok]).max()
    assert np.allclose(Bbh[0][ok], ob[ok], rtol=1e-5, atol=1e-5 * scale)
    used = ~np.isnan(Bbh[0])
    # model prediction per triplet, then binned with the same weights
    c_d = torch.from_numpy(C.astype(np.float32)).cuda()
    bd = p.model_discrete(c_d, 1.0)
    bd_ref = theory.b_ana_discrete(n, e, p.triplets, C.astype(np.float32).astype(np.float64), 1.0)
    bdh = bd.cpu().numpy()
    print("model: max rel diff %.3g" % np.max(np.abs(bdh / bd_ref - 1)), flush=True)
    assert np.allclose(bdh, bd_ref, rtol=1e-9)
    model_b, _ = p.rebin(bd.unsqueeze(0).contiguous(), N[:1].contiguous(), bins_d, nbins)
    model_b = model_b[0]
    # ensemble statistics over the used bins against the oracle's on the same values
    X = Bb[:, torch.from_numpy(used).cuda()].contiguous()
    mod = model_b[torch.from_numpy(used).cuda()].contiguous()
    mean, sigma, dB, dS = A.ensemble(X, mod)
    om, osg = oan.ensemble(X.cpu().numpy())
    odB, odS = oan.deviations(om, osg, mod.cpu().numpy())
    assert np.allclose(mean.cpu().numpy(), om, rtol=1e-12)
    assert np.allclose(sigma.cpu().numpy(), osg, rtol=1e-9)
    assert np.allclose(dB.cpu().numpy(), odB, rtol=1e-8) and np.allclose(dS.cpu().numpy(), odS, rtol=1e-8)
    z = dS.cpu().numpy() * np.sqrt(R)        # |mean - model| in standard errors
    print("binned ensemble: %d bins, max Delta_B %.3f, max z %.2f" % (used.sum(), dB.max().item(), z.max()),
          flush=True)
    assert z.max() <= 4.5


def test_model_prediction_with_counts_weights():
    """[B_Ana]_d with INV_COUNT weights (Poisson baseline counts) on 256^2 / 12 rings, and
    the paper's C_l: the weighted triangle average of the model against the oracle's."""
    torch = _torch()
    import paper_2412_02246_amd as A
    n = 256
    e = oplan.log_edges(3.0, 80.0, 12)
    rng = np.random.default_rng(31)
    counts = synth.poisson_counts(n, 4.0, n / 8, rng)
    C = synth.paper_spectrum(n, 1.0)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT).bind()
    c32 = C.astype(np.float32)
    bd = p.model_discrete(torch.from_numpy(c32).cuda(), 0.3,
                          w=torch.from_numpy(counts.astype(np.float32)).cuda()).cpu().numpy()
    Y = oest.effective_weights(n, counts, oest.INV_COUNT)
    bd_ref = theory.b_ana_discrete(n, e, p.triplets, c32.astype(np.float64), 0.3, Y=Y)
    assert np.array_equal(np.isnan(bd), np.isnan(bd_ref))
    ok = ~np.isnan(bd_ref)
    print("weighted model: max rel diff %.3g over %d triplets" % (np.max(np.abs(bd[ok] / bd_ref[ok] - 1)), ok.sum()))
    assert np.allclose(bd[ok], bd_ref[ok], rtol=1e-7)
