"""GPU parity of the general complex-input estimator (abs_estimate_complex, through the C ABI)
against the FP64 oracle's estimate_complex: complex B_t on every triplet, e_t = |B - B*| /
max(|B*|, rho_t) <= 1e-5 in FP32 and <= 1e-4 in the precision forms, the same empty triplets,
and N_t as for the Hermitian estimator.  Hermitian input must give Im B = 0 (to rounding) and
Re B equal to abs_estimate's B."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import plan as oplan

pytestmark = pytest.mark.gpu
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}


def _prec(A, name):
    return {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[name]


def _run(plan, grids, w=None, w_batched=False, n_given=None):
    import torch
    g = torch.from_numpy(np.ascontiguousarray(grids)).to(torch.complex64).cuda()
    wt = None if w is None else torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    B, N = plan.estimate_complex(g, wt, w_batched=w_batched, n_given=n_given)
    torch.cuda.synchronize()
    return B.cpu().numpy(), N.cpu().numpy()


def _check(B, N, ref, norm, tol, label):
    empty = np.isnan(ref["B"].real)
    assert np.array_equal(np.isnan(B.real), empty), label
    assert np.array_equal(np.isnan(B.imag), empty), label
    keep = ~empty
    e = oest.relative_error(B, ref, norm)[keep]
    en = oest.count_error(N, ref)
    print("%s max e_t %.3g  median %.3g  max e_N %.3g  ntrip %d (%d empty)  |Im|/|B| median %.3g"
          % (label, e.max(), np.median(e), en.max(), len(B), int(empty.sum()),
             np.median(np.abs(ref["B"].imag[keep]) / np.abs(ref["B"][keep]))), flush=True)
    assert np.all(np.isfinite(B[keep]))
    assert e.max() <= tol, (label, e.max(), int(np.argmax(e)))
    assert en.max() <= 1e-5, (label, en.max())


SMALL = [
    (16, [1.0, 2.0, 3.1, 4.2, 5.3]),
    (64, [1.0, 1.1, 2.3, 2.9, 3.0, 6.2, 9.9, 13.0, 21.0]),
    (256, list(oplan.log_edges(3.0, 80.0, 13))),
]


@pytest.mark.parametrize("n,edges", SMALL)
@pytest.mark.parametrize("wmode", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_small_grids_complex(n, edges, wmode, prec):
    import paper_2412_02246_amd as A
    rng = np.random.default_rng(7000 + 100 * n + 10 * wmode)
    V = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))     # not Hermitian
    if wmode == 1:
        w = synth.symmetrize(rng.integers(0, 4, (n, n)).astype(np.float64))
    elif wmode == 2:
        w = synth.symmetrize(rng.uniform(0.1, 2.0, (n, n)))
    else:
        w = None
    p = A.Plan(n, edges, norm=1.0, wmode=wmode, max_batch=2, precision=_prec(A, prec)).bind()
    B, N = _run(p, V.astype(np.complex64), w)
    for b in range(2):
        ref = oest.estimate_complex(V[b].astype(np.complex64), w, edges, 1.0, wmode=wmode, trips=p.triplets)
        _check(B[b], N[b], ref, 1.0, TOL[prec], "complex n%d w%d %s [%d]" % (n, wmode, prec, b))
    p.close()


def test_per_grid_weights_and_given_counts():
    """w_batched (a weight set per grid) and n_given (counts supplied by abs_counts)."""
    import torch
    import paper_2412_02246_amd as A
    n, edges = 64, [1.0, 2.3, 3.0, 6.2, 9.9, 13.0, 21.0]
    rng = np.random.default_rng(31)
    V = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    w = np.stack([synth.symmetrize(rng.uniform(0.2, 2.0, (n, n))) for _ in range(3)])
    p = A.Plan(n, edges, norm=2.5, wmode=A.W_GIVEN, max_batch=3).bind()
    B, N = _run(p, V, w, w_batched=True)
    for b in range(3):
        ref = oest.estimate_complex(V[b].astype(np.complex64), w[b], edges, 2.5, wmode=2, trips=p.triplets)
        _check(B[b], N[b], ref, 2.5, TOL["fp32"], "complex w_batched [%d]" % b)
    w0 = torch.from_numpy(w[0].astype(np.float32)).cuda()
    N0 = p.counts(w0)
    B2, N2 = _run(p, V, w[0], n_given=N0)
    for b in range(3):
        ref = oest.estimate_complex(V[b].astype(np.complex64), w[0], edges, 2.5, wmode=2, trips=p.triplets)
        _check(B2[b], N2[b], ref, 2.5, TOL["fp32"], "complex n_given [%d]" % b)
    p.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_hermitian_input_matches_the_real_estimator(prec):
    import paper_2412_02246_amd as A
    n = 256
    edges = list(oplan.log_edges(3.0, 80.0, 12))
    V, counts = synth.mwa_like(n, synth.seed_for(2, 40), U0=n / 8)
    p = A.Plan(n, edges, wmode=A.W_INV_COUNT, max_batch=1, precision=_prec(A, prec)).bind()
    import torch
    g = torch.from_numpy(V.astype(np.complex64)).cuda()[None]
    w = torch.from_numpy(counts.astype(np.float32)).cuda()
    Bc, Nc = p.estimate_complex(g, w)
    Br, Nr = p.estimate(g, w)
    torch.cuda.synchronize()
    Bc, Br = Bc[0].cpu().numpy(), Br[0].cpu().numpy()
    ref = oest.estimate(V.astype(np.complex64), counts, edges, p.norm, wmode=oest.INV_COUNT, trips=p.triplets,
                        with_scales=True)
    keep = ~np.isnan(ref["B"])
    assert np.array_equal(np.isnan(Bc.real), ~keep)
    scale = np.maximum(np.abs(ref["B"]), ref["rhoS"] / (p.norm * np.abs(ref["N"])))[keep]
    e_im = np.abs(Bc.imag[keep]) / scale
    e_re = np.abs(Bc.real[keep] - Br[keep]) / scale
    print("hermitian %s: max |Im B|/scale %.3g, max |Re B - B_real|/scale %.3g" % (prec, e_im.max(), e_re.max()),
          flush=True)
    assert e_im.max() <= TOL[prec] and e_re.max() <= 2 * TOL[prec]
    assert torch.equal(Nc, Nr)
    p.close()


def test_mwa_1024_complex_channel():
    """A 1024^2 MWA-shaped channel whose gridded visibilities carry a non-Hermitian part
    (per-cell noise added before any symmetrisation), 24 log rings, INV_COUNT weights,
    every triplet against the oracle, in FP32 and BF16x3."""
    import torch
    import paper_2412_02246_amd as A
    n = 1024
    edges = list(oplan.log_edges(46.0 / (2 * np.pi), 1320.0 / (2 * np.pi), 24))
    V, counts = synth.mwa_like(n, synth.seed_for(3, 7), U0=n / 8)
    rng = np.random.default_rng(99)
    amp = 0.3 * np.sqrt(np.mean(np.abs(V[counts > 0]) ** 2))
    V = V + counts * (counts > 0) * amp * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    V = V.astype(np.complex64)
    ref = None
    for prec in ("fp32", "bf16x3"):
        p = A.Plan(n, edges, wmode=A.W_INV_COUNT, max_batch=1, precision=_prec(A, prec))
        p.compile(workers=8)
        p.bind()
        if ref is None:
            ref = oest.estimate_complex(V, counts, edges, p.norm, wmode=oest.INV_COUNT, trips=p.triplets)
        B, N = p.estimate_complex(torch.from_numpy(V).cuda()[None], torch.from_numpy(counts.astype(np.float32)).cuda())
        torch.cuda.synchronize()
        _check(B[0].cpu().numpy(), N[0].cpu().numpy(), ref, p.norm, TOL[prec], "mwa1024 complex %s" % prec)
        p.close()


def test_half_plane_grids():
    """A channel supplied on a half plane (one cell of every (g, -g) pair, zero elsewhere, with
    its counts likewise) gives the full-plane B_t in the Hermitian estimator (INV_COUNT
    weights; N_t is 1/8 of the full-plane count).  The complex estimator takes the grid as it
    is, and no closed triangle lies inside a half plane, so its S_t is zero to rounding."""
    import torch
    import paper_2412_02246_amd as A
    n = 256
    edges = list(oplan.log_edges(3.0, 80.0, 12))
    V, counts = synth.mwa_like(n, synth.seed_for(2, 41), U0=n / 8)
    g = oplan.signed_index(n)
    gx, gy = np.meshgrid(g, g)
    half = (gy > 0) | ((gy == 0) & (gx > 0))
    Vh, ch = np.where(half, V, 0).astype(np.complex64), np.where(half, counts, 0)
    p = A.Plan(n, edges, wmode=A.W_INV_COUNT, max_batch=1).bind()
    ref = oest.estimate(V.astype(np.complex64), counts, edges, p.norm, wmode=oest.INV_COUNT, trips=p.triplets,
                        with_scales=True)
    gt = torch.from_numpy(Vh).cuda()[None]
    wt = torch.from_numpy(ch.astype(np.float32)).cuda()
    B, N = p.estimate(gt, wt)
    Bc, _ = p.estimate_complex(gt, wt)
    torch.cuda.synchronize()
    B, N, Bc = B[0].cpu().numpy(), N[0].cpu().numpy(), Bc[0].cpu().numpy()
    keep = ~np.isnan(ref["B"])
    assert np.array_equal(np.isnan(B), ~keep)
    e = oest.relative_error(B, ref, p.norm)[keep]
    en = oest.count_error(N, dict(ref, N=ref["N"] / 8, rhoN=ref["rhoN"] / 8))
    refc = oest.estimate_complex(Vh, ch, edges, p.norm, wmode=oest.INV_COUNT, trips=p.triplets)
    assert np.all(np.abs(refc["S"]) <= 1e-9 * refc["rhoS"])
    okc = ~np.isnan(refc["B"].real)
    ec = oest.relative_error(Bc, refc, p.norm)[okc]
    print("half plane: max e_t %.3g, max e_N (vs N/8) %.3g; complex |B|/rho max %.3g" % (e.max(), en.max(), ec.max()),
          flush=True)
    assert e.max() <= 1e-5 and en.max() <= 1e-5 and ec.max() <= 1e-5
    p.close()
