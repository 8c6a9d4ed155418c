"""GPU parity of multi-frequency plans (the estimator with the three fields of a triplet
taken at three channels) against the FP64 oracle on every channel triplet: all weight
modes, per-grid and shared weights, forced resolution levels, both split-precision forms,
cached counts; and identical channels against the single-frequency plan."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import plan as oplan

pytestmark = pytest.mark.gpu
TOL = 1e-5
PREC_TOL = 1e-4


def _check(B, N, ref, norm, tol=TOL, label=""):
    empty = np.isnan(ref["B"])
    assert np.array_equal(np.isnan(B), empty), (label, int(np.isnan(B).sum()), int(empty.sum()))
    keep = ~empty
    e = oest.relative_error(B, ref, norm)[keep]
    en = oest.count_error(N, ref)
    print("%s max e_t %.3g median %.3g max e_N %.3g ntrip %d (%d empty)"
          % (label, e.max(), np.median(e), en.max(), len(B), int(empty.sum())), flush=True)
    assert e.max() <= tol, (label, e.max())
    assert en.max() <= tol, (label, en.max())


def _weights(rng, n, wmode, k=None):
    shape = (n, n) if k is None else (k, n, n)
    if wmode == 1:
        w = rng.integers(0, 4, shape).astype(np.float64)
    elif wmode == 2:
        w = rng.uniform(0.1, 2.0, shape)
    else:
        return None
    return synth.symmetrize(w) if k is None else np.stack([synth.symmetrize(x) for x in w])


CASES = [(64, 2, 0), (128, 3, 0), (256, 2, 1)]   # (n, channels, force every level)


@pytest.mark.parametrize("n,C,every", CASES)
@pytest.mark.parametrize("wmode", [0, 1, 2])
def test_multifreq_matches_oracle(n, C, every, wmode):
    import torch
    import paper_2412_02246_amd as A
    e = oplan.log_edges(2.0, n / 3.2, {64: 6, 128: 8, 256: 10}[n])
    rng = np.random.default_rng(30 * n + wmode)
    batch = 2
    V = rng.standard_normal((batch, C, n, n)) + 1j * rng.standard_normal((batch, C, n, n))
    w = _weights(rng, n, wmode, batch * C)   # per-grid, per-channel weights
    flags = A.EVERY_LEVEL if every else 0
    p = A.Plan(n, e, norm=1.0, wmode=wmode, max_batch=batch, nchan=C, flags=flags, levels=4 if every else 1).bind()
    print("n %d C %d levels %s ntrip %d" % (n, C, [(l["m"], l["ring0"], l["nbins"], l["ntrip"]) for l in p.levels],
                                            p.ntrip), flush=True)
    g = torch.from_numpy(V.reshape(batch * C, n, n)).to(torch.complex64).cuda()
    wt = None if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
    B, N = p.estimate(g, wt, w_batched=w is not None)
    torch.cuda.synchronize()
    B, N = B.cpu().numpy(), N.cpu().numpy()
    for b in range(batch):
        wb = None if w is None else w.reshape(batch, C, n, n)[b]
        ref = oest.estimate_multifreq(V[b], wb, e, 1.0, wmode=wmode, trips=p.triplets)
        _check(B[b], N[b], ref, 1.0, label="n%d C%d w%d [%d]" % (n, C, wmode, b))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_multifreq_precision_forms_and_cached_counts(prec):
    import torch
    import paper_2412_02246_amd as A
    n, C = 256, 3
    e = oplan.log_edges(4.0, 80.0, 12)
    P = {"bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    grids, counts = zip(*[synth.mwa_like(n, synth.seed_for(3, 60 + c)) for c in range(C)])
    w = counts[0]                       # one baseline set for every channel
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, nchan=C, precision=P, flags=A.EVERY_LEVEL).bind()
    g = torch.from_numpy(np.stack(grids)).to(torch.complex64).cuda()
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    B, N = p.estimate(g, wt)
    Nc = p.counts(wt)
    B2, _ = p.estimate(g, wt, n_given=Nc)
    torch.cuda.synchronize()
    # the same partials summed in the same order: bit for bit (NaN where a triplet is empty)
    assert torch.equal(Nc, N[0])
    assert np.array_equal(B2.cpu().numpy(), B.cpu().numpy(), equal_nan=True)
    ref = oest.estimate_multifreq(np.stack(grids), w, e, p.norm, wmode=oest.INV_COUNT, trips=p.triplets)
    _check(B[0].cpu().numpy(), N[0].cpu().numpy(), ref, p.norm, tol=PREC_TOL, label="mf %s" % prec)


def test_identical_channels_match_the_single_frequency_plan():
    import torch
    import paper_2412_02246_amd as A
    n, C = 128, 3
    e = oplan.log_edges(2.0, 40.0, 8)
    V, counts = synth.mwa_like(n, synth.seed_for(3, 77))
    one = A.Plan(n, e, wmode=A.W_INV_COUNT).bind()
    mf = A.Plan(n, e, wmode=A.W_INV_COUNT, nchan=C).bind()
    wt = torch.from_numpy(counts.astype(np.float32)).cuda()
    g1 = torch.from_numpy(V[None]).to(torch.complex64).cuda()
    B1, _ = one.estimate(g1, wt)
    Bm, _ = mf.estimate(g1.repeat(C, 1, 1).contiguous(), wt)
    torch.cuda.synchronize()
    B1, Bm = B1[0].cpu().numpy(), Bm[0].cpu().numpy()
    ref = oest.estimate(V, counts, e, one.norm, wmode=oest.INV_COUNT, trips=one.triplets, with_scales=True)
    idx = {tuple(int(x) for x in t): q for q, t in enumerate(one.triplets)}
    nb = len(e) - 1
    ts = np.array([idx[tuple(sorted(int(x) % nb for x in s))] for s in mf.triplets])
    keep = ~np.isnan(B1[ts])
    rho = ref["rhoS"][ts] / (one.norm * np.abs(ref["N"][ts]))
    d = np.abs(Bm - B1[ts])[keep] / np.maximum(np.abs(B1[ts]), rho)[keep]
    print("identical channels: max |B_mf - B_1| / scale %.3g over %d channel triplets" % (d.max(), len(ts)), flush=True)
    assert np.array_equal(np.isnan(Bm), np.isnan(B1[ts]))
    assert d.max() <= 2 * TOL
