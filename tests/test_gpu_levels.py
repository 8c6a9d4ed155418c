"""GPU parity of resolution levels: plans whose triplets run on m x m grids (m = n/2 down
to n/8, each triplet i <= j <= k on the smallest level with h_i + h_j + h_k < m and
2 h_k < m, h a ring's largest |g_x|) against the FP64 oracle on every triplet, in every
weight mode and
precision form, for wrapped (cyclic) plans, with cached counts and for the complex
estimator; and against the same plan evaluated at n alone.  Gates as in the other parity
tests: e_t <= 1e-5 for FP32, 1e-4 for the split-precision forms."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import plan as oplan

pytestmark = pytest.mark.gpu
TOL = 1e-5
PREC_TOL = 1e-4


def _torch():
    import torch
    return torch


def _A():
    import paper_2412_02246_amd as A
    return A


def _check(B, N, ref, norm, tol=TOL, label=""):
    empty = np.isnan(ref["B"])
    assert np.array_equal(np.isnan(B), empty), (label, int(np.isnan(B).sum()), int(empty.sum()))
    keep = ~empty
    e = oest.relative_error(B, ref, norm)[keep]
    en = oest.count_error(N, ref)
    print("%s max e_t %.3g  median %.3g  max e_N %.3g  ntrip %d (%d empty)"
          % (label, e.max(), np.median(e), en.max(), len(B), int(empty.sum())), flush=True)
    assert np.all(np.isfinite(B[keep]))
    assert e.max() <= tol, (label, e.max(), int(np.argmax(e)))
    assert en.max() <= tol, (label, en.max())
    return e


def _weights(rng, n, wmode):
    if wmode == 1:
        return synth.symmetrize(rng.integers(0, 4, (n, n)).astype(np.float64))
    if wmode == 2:
        return synth.symmetrize(rng.uniform(0.1, 2.0, (n, n)))
    return None


def _levels_of(p):
    return [(lv["m"], lv["ring0"], lv["nbins"], lv["ntrip"]) for lv in p.levels]


CASES = {
    # 256^2, 16 rings to n/3: levels 256, 128, 64, 32
    "256x16": (256, oplan.log_edges(3.0, 85.0, 16), 8, 0),
    # 512^2, 24 rings: levels 512, 256, 128
    "512x24": (512, oplan.log_edges(4.0, 170.0, 24), 4, 0),
    # 128^2 with rings past n/3 (cyclic closure at n for the outer triplets)
    "wrap128": (128, oplan.log_edges(2.0, 60.0, 12), 8, 1),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("wmode", [0, 1, 2])
def test_every_level_matches_oracle(case, wmode):
    A = _A()
    torch = _torch()
    n, e, ratio, wrap = CASES[case]
    flags = A.EVERY_LEVEL | (A.ALLOW_WRAP if wrap else 0)
    rng = np.random.default_rng(7000 + 10 * n + wmode)
    V = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    w = _weights(rng, n, wmode)
    p = A.Plan(n, e, norm=1.0, wmode=wmode, max_batch=2, flags=flags, levels=ratio)
    assert len(p.levels) >= 3, _levels_of(p)
    print("%s: levels %s" % (case, _levels_of(p)), flush=True)
    p.bind()
    g = torch.from_numpy(V).to(torch.complex64).cuda()
    wt = None if w is None else torch.from_numpy(w.astype(np.float32)).cuda()
    B, N = p.estimate(g, wt)
    torch.cuda.synchronize()
    B, N = B.cpu().numpy(), N.cpu().numpy()
    for b in range(2):
        ref = oest.estimate(V[b], w, e, 1.0, wmode=wmode, trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, 1.0, label="%s w%d [%d]" % (case, wmode, b))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_levels_precision_forms(prec):
    A = _A()
    torch = _torch()
    n, e, _, _ = CASES["512x24"]
    P = {"bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    V, counts = synth.mwa_like(n, synth.seed_for(1, 31))
    # each form's default bound on n / m (2 for the BF16 split, 4 for the FP16 split)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, precision=P, flags=A.EVERY_LEVEL)
    assert len(p.levels) == {"bf16x3": 2, "fp16x3": 3}[prec], _levels_of(p)
    p.bind()
    B, N = p.estimate(torch.from_numpy(V).to(torch.complex64).cuda(),
                      torch.from_numpy(counts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref = oest.estimate(V, counts, e, p.norm, wmode=oest.INV_COUNT, trips=p.triplets, with_scales=True)
    _check(B[0].cpu().numpy(), N[0].cpu().numpy(), ref, p.norm, tol=PREC_TOL, label="512x24 %s" % prec)


def test_levels_cached_counts_and_complex_input():
    """abs_counts of a levelled plan gives the N_t its estimate reports (bit for bit: the
    same partials summed in the same order), an estimate with those cached counts the same
    B, and the complex estimator matches the oracle's complex B."""
    A = _A()
    torch = _torch()
    n, e, ratio, _ = CASES["256x16"]
    rng = np.random.default_rng(4321)
    V = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    w = _weights(rng, n, 2).astype(np.float32).astype(np.float64)   # the weights the GPU reads
    p = A.Plan(n, e, norm=1.0, wmode=A.W_GIVEN, max_batch=2, flags=A.EVERY_LEVEL, levels=ratio).bind()
    g = torch.from_numpy(V).to(torch.complex64).cuda()
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    B, N = p.estimate(g, wt)
    Nc = p.counts(wt)
    B2, N2 = p.estimate(g, wt, n_given=Nc)
    Bc, Nx = p.estimate_complex(g, wt)
    torch.cuda.synchronize()
    assert torch.equal(Nc, N[0]) and torch.equal(Nc, N[1])
    assert np.array_equal(B2.cpu().numpy(), B.cpu().numpy(), equal_nan=True) and torch.equal(N2, N)
    for b in range(2):
        ref = oest.estimate_complex(V[b], w, e, 1.0, wmode=oest.GIVEN, trips=p.triplets)
        Bb = Bc[b].cpu().numpy()
        empty = np.isnan(ref["B"].real)
        assert np.array_equal(np.isnan(Bb.real), empty)
        k = ~empty
        rho = ref["rhoS"][k] / np.abs(ref["N"][k])
        err = np.abs(Bb[k] - ref["B"][k]) / np.maximum(np.abs(ref["B"][k]), rho)
        print("complex [%d] max e_t %.3g" % (b, err.max()), flush=True)
        assert err.max() <= TOL
        # the weight path is FP64 throughout: N_t to ~1e-9 of its random-error scale
        assert np.all(oest.count_error(Nx[b].cpu().numpy(), ref) <= 1e-9)


def test_mwa_1024_levels_against_single_level_and_oracle():
    """The 1024^2 / 20-ring MWA-shaped channel with the levels the cost model picks for
    batches of 16 (1024 for rings 15-19, 512 for the rest), on two realisations with
    per-grid counts: every triplet against the oracle, and against the same plan with every
    triplet at 1024."""
    A = _A()
    torch = _torch()
    n = 1024
    e = oplan.log_edges(46.0 / (2 * np.pi), 1320.0 / (2 * np.pi), 20)
    grids, ws = zip(*[synth.mwa_like(n, synth.seed_for(1, 40 + r)) for r in range(2)])
    g = torch.from_numpy(np.stack(grids)).to(torch.complex64).cuda()
    wt = torch.from_numpy(np.stack(ws).astype(np.float32)).cuda()
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=16)
    assert _levels_of(p) == [(1024, 15, 5, 9), (512, 0, 20, 681)], _levels_of(p)
    q = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=16, levels=1)
    assert len(q.levels) == 1
    p.bind()
    q.bind()
    B, N = p.estimate(g, wt, w_batched=True)
    B1, N1 = q.estimate(g, wt, w_batched=True)
    torch.cuda.synchronize()
    B, N, B1, N1 = (x.cpu().numpy() for x in (B, N, B1, N1))
    for b in range(2):
        ref = oest.estimate(grids[b], ws[b], e, p.norm, wmode=oest.INV_COUNT, trips=p.triplets, with_scales=True)
        e_lv = _check(B[b], N[b], ref, p.norm, label="mwa1024 levels [%d]" % b)
        e_one = _check(B1[b], N1[b], ref, p.norm, label="mwa1024 single [%d]" % b)
        # the level at 512 sums over a quarter of the pixels: its rounding error is larger
        # but within the same gate
        lv = np.isin(np.arange(p.ntrip), p.levels[1]["tmap"])[~np.isnan(ref["B"])]
        print("  level 512 max e_t %.3g (single level %.3g)" % (e_lv[lv].max(), e_one[lv].max()), flush=True)
