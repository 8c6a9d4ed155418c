"""GPU parity at full size: 4096 x 4096 MWA-shaped grid, 32 log rings over
4 x (46 <= l < 1320), INV_COUNT weights, in FP32 and in the two precision forms.
The oracle computes a sample of the triplets one by one: every plan triplet whose
three rings lie in a fixed subset of 9 rings, each compared element by element."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import plan as oplan

pytestmark = pytest.mark.gpu

N = 4096
EDGES = oplan.log_edges(4 * 46 / (2 * np.pi), 4 * 1320 / (2 * np.pi), 32)
SUBSET = {0, 4, 8, 12, 16, 20, 24, 28, 31}
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}


@pytest.fixture(scope="module")
def c3():
    import paper_2412_02246_amd as A
    V, counts = synth.mwa_like(N, synth.seed_for(2, 0), U0=N / 8)
    V = V.astype(np.complex64)
    host = A.Plan(N, EDGES)          # the triplet list only (host, exact)
    idx = np.array([q for q, t in enumerate(host.triplets) if set(t.tolist()) <= SUBSET])
    print("C3 sample: %d of %d triplets" % (len(idx), host.ntrip), flush=True)
    ref = oest.estimate_subset(V, counts, EDGES, host.norm, host.triplets[idx], wmode=oest.INV_COUNT)
    return V, counts, idx, ref, host.triplets


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_c3_full_size(c3, prec):
    import torch
    import paper_2412_02246_amd as A
    V, counts, idx, ref, trips = c3
    P = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    p = A.Plan(N, EDGES, wmode=A.W_INV_COUNT, precision=P).bind()
    assert np.array_equal(p.triplets, trips)
    B, Nn = p.estimate(torch.from_numpy(V).cuda(), torch.from_numpy(counts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    B = B[0].cpu().numpy()[idx]
    Nn = Nn[0].cpu().numpy()[idx]
    assert np.array_equal(np.isnan(B), np.isnan(ref["B"]))   # empty weighted triplets
    ok = ~np.isnan(ref["B"])
    e = oest.relative_error(B, ref, p.norm)[ok]
    en = oest.count_error(Nn, ref)
    print("C3 %s: e_t median %.3g max %.3g, e_N max %.3g over %d sampled triplets"
          % (prec, np.median(e), e.max(), en.max(), len(idx)), flush=True)
    assert np.all(np.isfinite(B[ok]))
    assert e.max() <= TOL[prec]
    assert en.max() <= 1e-5


# 8192 x 8192, 64 log rings over 8 x (46 <= l < 1320): the large-ensemble shapes.  The
# oracle's sample is every plan triplet within 4 rings spread over the range.
N5 = 8192
EDGES5 = oplan.log_edges(8 * 46 / (2 * np.pi), 8 * 1320 / (2 * np.pi), 64)
SUBSET5 = {0, 21, 42, 63}


@pytest.fixture(scope="module")
def c5():
    import paper_2412_02246_amd as A
    V, counts = synth.mwa_like(N5, synth.seed_for(4, 0), U0=N5 / 8)
    V = V.astype(np.complex64)
    host = A.Plan(N5, EDGES5)
    idx = np.array([q for q, t in enumerate(host.triplets) if set(t.tolist()) <= SUBSET5])
    print("C5 sample: %d of %d triplets" % (len(idx), host.ntrip), flush=True)
    ref = oest.estimate_subset(V, counts, EDGES5, host.norm, host.triplets[idx], wmode=oest.INV_COUNT)
    return V, counts, idx, ref, host.triplets


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_c5_full_size(c5, prec):
    import torch
    import paper_2412_02246_amd as A
    V, counts, idx, ref, trips = c5
    P = {"fp32": A.FP32, "bf16x3": A.BF16X3}[prec]
    p = A.Plan(N5, EDGES5, wmode=A.W_INV_COUNT, precision=P)
    p.compile(workers=8)   # the code parts in worker processes
    p.bind()
    assert np.array_equal(p.triplets, trips)
    B, Nn = p.estimate(torch.from_numpy(V).cuda(), torch.from_numpy(counts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    B = B[0].cpu().numpy()[idx]
    Nn = Nn[0].cpu().numpy()[idx]
    assert np.array_equal(np.isnan(B), np.isnan(ref["B"]))   # empty weighted triplets
    ok = ~np.isnan(ref["B"])
    e = oest.relative_error(B, ref, p.norm)[ok]
    en = oest.count_error(Nn, ref)
    print("C5 %s: e_t median %.3g max %.3g, e_N max %.3g over %d sampled triplets"
          % (prec, np.median(e), e.max(), en.max(), len(idx)), flush=True)
    assert np.all(np.isfinite(B[ok]))
    assert e.max() <= TOL[prec]
    assert en.max() <= 1e-5


# The large-ensemble use of the 8192^2 / 64-ring shapes: many realisations of one channel
# (shared weights: the counts N_t computed once), estimated in FP32 and in BF16x3 on the
# same GPU.  The split form must not move the ensemble statistics: over R realisations the
# difference of the two sample means of every triplet stays below 1% of that triplet's
# standard error, and the sample variances agree to 0.1%.
R5 = 16
BATCH5 = 4


def _c5_realisations(counts, seed):
    """R5 Hermitian grids on the GPU: a real Gaussian sky with C(l) ~ l^-2 inside the rings,
    its FFT weighted by the counts (the gridded sum over baselines)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    k = torch.fft.fftfreq(N5, d=1.0 / N5, device="cuda", dtype=torch.float64)
    r = torch.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    amp = torch.where(r > 0, 1.0 / torch.clamp(r, min=1.0), torch.zeros_like(r))
    w = torch.from_numpy(counts).cuda().to(torch.float64)
    out = []
    for _ in range(R5):
        sky = torch.randn((N5, N5), generator=g, device="cuda", dtype=torch.float64)
        V = torch.fft.fft2(sky) * amp * w
        out.append(V.to(torch.complex64))
    return out


def test_c5_ensemble_fp32_vs_bf16x3(c5):
    import torch
    import paper_2412_02246_amd as A
    _, counts, _, _, trips = c5
    grids = _c5_realisations(counts, synth.seed_for(4, 1))
    wt = torch.from_numpy(counts.astype(np.float32)).cuda()
    res = {}
    for prec, P in (("fp32", A.FP32), ("bf16x3", A.BF16X3)):
        p = A.Plan(N5, EDGES5, wmode=A.W_INV_COUNT, precision=P, max_batch=BATCH5)
        p.compile(workers=8)
        p.bind()
        assert np.array_equal(p.triplets, trips)
        n_given = p.counts(wt)
        Bs = []
        for b0 in range(0, R5, BATCH5):
            B, _ = p.estimate(torch.stack(grids[b0:b0 + BATCH5]), wt, n_given=n_given)
            Bs.append(B.cpu().numpy())
        torch.cuda.synchronize()
        res[prec] = np.concatenate(Bs)
        p.close()
    f, h = res["fp32"], res["bf16x3"]
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(h))
    mean_f, mean_h = f.mean(0), h.mean(0)
    sd_f = f.std(0, ddof=1)
    var_h = h.var(0, ddof=1)
    z = np.abs(mean_h - mean_f) / (sd_f / np.sqrt(R5))
    dv = np.abs(var_h / sd_f ** 2 - 1)
    print("C5 ensemble (%d realisations, %d triplets): max |mean diff| / s.e. %.3g, "
          "max |var ratio - 1| %.3g" % (R5, f.shape[1], z.max(), dv.max()), flush=True)
    assert z.max() <= 1e-2
    assert dv.max() <= 1e-3


# The two power-of-two sizes between the small grids and 4096^2 that the serving mix uses
# (512^2 and 2048^2, 16 and 24 log rings with radii scaled by n/1024), against the oracle on
# every plan triplet within a subset of rings: each size has its own FFT kernel shapes
# (column workgroup width, transforms per workgroup).
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,nb,subset", [(512, 16, {0, 5, 10, 15}), (2048, 24, {0, 8, 16, 23})])
def test_mid_sizes(n, nb, subset, prec):
    import torch
    import paper_2412_02246_amd as A
    s = n / 1024.0
    edges = oplan.log_edges(s * 46 / (2 * np.pi), s * 1320 / (2 * np.pi), nb)
    V, counts = synth.mwa_like(n, synth.seed_for(3, n), U0=n / 8)
    V = V.astype(np.complex64)
    P = {"fp32": A.FP32, "bf16x3": A.BF16X3}[prec]
    p = A.Plan(n, edges, wmode=A.W_INV_COUNT, precision=P).bind()
    idx = np.array([q for q, t in enumerate(p.triplets) if set(t.tolist()) <= subset])
    ref = oest.estimate_subset(V, counts, edges, p.norm, p.triplets[idx], wmode=oest.INV_COUNT)
    B, Nn = p.estimate(torch.from_numpy(V).cuda(), torch.from_numpy(counts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    B = B[0].cpu().numpy()[idx]
    Nn = Nn[0].cpu().numpy()[idx]
    assert np.array_equal(np.isnan(B), np.isnan(ref["B"]))   # empty weighted triplets
    ok = ~np.isnan(ref["B"])
    e = oest.relative_error(B, ref, p.norm)[ok]
    en = oest.count_error(Nn, ref)
    print("n%d/%d %s: e_t median %.3g max %.3g, e_N max %.3g over %d of %d triplets"
          % (n, nb, prec, np.median(e), e.max(), en.max(), len(idx), p.ntrip), flush=True)
    assert len(idx) > 0
    assert np.all(np.isfinite(B[ok]))
    assert e.max() <= TOL[prec]
    assert en.max() <= 1e-5
