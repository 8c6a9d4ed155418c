"""GPU parity: libabs.so (through the C ABI) against the FP64 oracle, element by
element, on seeded inputs.  Gate for the FP32 path: the noise-scale-normalised error
e_t = |B - B*| / max(|B*|, rho_t) <= 1e-5 on every triplet (rho_t: FP64 random-error
scale of the triangle sum), and the same normalisation for N_t."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import gridding as ogrid
from oracle import plan as oplan

pytestmark = pytest.mark.gpu
TOL = 1e-5
PREC_TOL = 1e-4     # precision forms (split BF16 / FP16 products)


def _torch():
    import torch
    return torch


def _A():
    import paper_2412_02246_amd as A
    return A


def _run(plan, grids, w=None, w_batched=False, dtype=None, n_given=None):
    torch = _torch()
    dt = dtype or torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(grids)).to(dt).cuda()
    wt = None if w is None else torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda()
    B, N = plan.estimate(g, wt, w_batched=w_batched, n_given=n_given)
    torch.cuda.synchronize()
    return B.cpu().numpy(), N.cpu().numpy()


def _check(B, N, ref, norm, tol=TOL, label=""):
    # A triplet whose rings close triangles only through zero-weight cells has an empty
    # weighted set: N_t is rounding noise of an exact zero and B_t is NaN (N_t below
    # w_min^3 / 2, since any weighted triangle adds at least w_min^3).  The GPU must mark
    # exactly the oracle's empty triplets; B is compared on the others.
    empty = np.isnan(ref["B"])
    assert np.array_equal(np.isnan(B), empty), (label, int(np.isnan(B).sum()), int(empty.sum()))
    assert np.all(np.abs(N[empty]) <= 1e-9 * np.maximum(ref["rhoN"][empty], ref["wmin"] ** 3)), label
    keep = ~empty
    e = oest.relative_error(B, ref, norm)[keep]
    en = oest.count_error(N, ref)
    print("%s max e_t %.3g  median %.3g  max e_N %.3g  ntrip %d (%d empty)"
          % (label, e.max(), np.median(e), en.max(), len(B), int(empty.sum())), flush=True)
    assert np.all(np.isfinite(B[keep]))
    assert e.max() <= tol, (label, e.max(), int(np.argmax(e)))
    assert en.max() <= tol, (label, en.max())


def test_c1_complex128_unit_weights():
    """128 x 128 complex128 grids, 8 log rings (2 .. 42), unit weights, 2 realisations."""
    A = _A()
    n, e = 128, oplan.log_edges(2.0, 42.0, 8)
    C = synth.powerlaw_spectrum(n, 0.05)
    rng = np.random.default_rng(synth.seed_for(0, 0))
    grids = np.stack([synth.nongaussian_grid(C, 1.0, rng) for _ in range(2)])
    p = A.Plan(n, e, norm=float(n * n), max_batch=2).bind()
    B, N = _run(p, grids, dtype=_torch().complex128)
    for b in range(2):
        ref = oest.estimate(grids[b], None, e, float(n * n), trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, float(n * n), label="C1[%d]" % b)
    # unit counts are integers
    assert np.allclose(N[0], np.rint(N[0]), atol=1e-6 * N[0].max())


SMALL = [
    (16, [1.0, 2.0, 3.1, 4.2, 5.3], 0),
    (32, [1.2, 2.0, 3.3, 5.1, 7.0, 10.5], 0),
    (64, [1.0, 1.1, 2.3, 2.9, 3.0, 6.2, 9.9, 13.0, 21.0], 0),
    (32, [1.5, 4.0, 7.0, 11.5, 15.0], 1),      # ALLOW_WRAP: cyclic closure
    (256, list(oplan.log_edges(3.0, 80.0, 13)), 0),
]


@pytest.mark.parametrize("n,edges,flags", SMALL)
@pytest.mark.parametrize("wmode", [0, 1, 2])
def test_small_grids_all_weight_modes(n, edges, flags, wmode):
    A = _A()
    rng = np.random.default_rng(1000 * n + 10 * wmode + flags)
    V = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))   # not Hermitian
    if wmode == 1:
        w = synth.symmetrize(rng.integers(0, 4, (n, n)).astype(np.float64))
    elif wmode == 2:
        w = synth.symmetrize(rng.uniform(0.1, 2.0, (n, n)))
    else:
        w = None
    p = A.Plan(n, edges, norm=1.0, wmode=wmode, max_batch=3, flags=flags).bind()
    B, N = _run(p, V, w)
    for b in range(3):
        ref = oest.estimate(V[b], w, edges, 1.0, wmode=wmode, trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, 1.0, label="n%d w%d f%d [%d]" % (n, wmode, flags, b))


def test_parseval_dc_ring():
    A = _A()
    n, edges = 16, [0.0, 0.5, 2.0, 3.5, 5.0]
    rng = np.random.default_rng(3)
    V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    V[0, 0] = 1.0
    p = A.Plan(n, edges, norm=1.0, flags=A.ALLOW_DC).bind()
    B, N = _run(p, V[None])
    ref = oest.estimate(V, None, edges, 1.0, trips=p.triplets, with_scales=True)
    _check(B[0], N[0], ref, 1.0, label="dc")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_empty_weighted_triplets(prec):
    """Hand-built weights (ring 0 weighted only on the v axis, ring 1 only on the u axis)
    leave plan triplets such as (0, 1, 1) without any weighted triangle: B_t must be NaN on
    exactly the oracle's empty triplets, in every precision form, and N_t is still reported."""
    A = _A()
    n, edges = 16, [1.0, 2.0, 3.1, 4.2, 5.3]
    g = oplan.signed_index(n)
    gx, gy = np.meshgrid(g, g)
    rc = oplan.ring_of_cell(n, edges)
    rng = np.random.default_rng(11)
    w = synth.symmetrize(rng.uniform(0.5, 1.5, (n, n)))
    w[(rc == 0) & (gx != 0)] = 0.0
    w[(rc == 1) & (gy != 0)] = 0.0
    V = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    P = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    p = A.Plan(n, edges, norm=1.0, wmode=A.W_GIVEN, max_batch=2, precision=P).bind()
    B, N = _run(p, V, w)
    for b in range(2):
        ref = oest.estimate(V[b], w, edges, 1.0, wmode=2, trips=p.triplets, with_scales=True)
        assert np.isnan(ref["B"]).sum() >= 1
        _check(B[b], N[b], ref, 1.0, tol=TOL if prec == "fp32" else PREC_TOL,
               label="empty %s [%d]" % (prec, b))


def _mwa_inputs(n, batch, cfg, seed0=0):
    grids, counts = [], None
    for r in range(batch):
        V, counts = synth.mwa_like(n, synth.seed_for(cfg, seed0 + r), counts=counts)
        grids.append(V)
    return np.stack(grids), counts


def test_c2_mwa_shared_weights_batch():
    """1024 x 1024 complex64, 20 log rings over 46 <= l < 1320, Poisson baseline mask,
    thermal noise at SNR 5, INV_COUNT weights shared by a batch of 3 realisations."""
    A = _A()
    n = 1024
    e = oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)
    grids, counts = _mwa_inputs(n, 3, 1)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=3).bind()
    B, N = _run(p, grids.astype(np.complex64), counts)
    for b in range(3):
        ref = oest.estimate(grids[b].astype(np.complex64), counts, e, p.norm, wmode=1,
                            trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, p.norm, label="C2[%d]" % b)
    # cached denominators give the same B bit for bit
    torch = _torch()
    Ng = p.counts(torch.from_numpy(counts.astype(np.float32)).cuda())
    B2, N2 = _run(p, grids.astype(np.complex64), counts, n_given=Ng)
    assert np.array_equal(B2, B) and np.array_equal(N2, N)


def test_c2_per_grid_weights_and_batch_independence():
    A = _A()
    n = 1024
    e = oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)
    rng = np.random.default_rng(77)
    grids, ws = [], []
    for r in range(2):
        V, c = synth.mwa_like(n, synth.seed_for(1, 100 + r))
        grids.append(V.astype(np.complex64))
        ws.append(c)
    grids, ws = np.stack(grids), np.stack(ws)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=2).bind()
    B, N = _run(p, grids, ws, w_batched=True)
    for b in range(2):
        ref = oest.estimate(grids[b], ws[b], e, p.norm, wmode=1, trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, p.norm, label="C2w[%d]" % b)
    # each result is the same alone and in the batch, bit for bit
    B1, N1 = _run(p, grids[1:2], ws[1:2], w_batched=True)
    assert np.array_equal(B1[0], B[1]) and np.array_equal(N1[0], N[1])
    assert not np.array_equal(B[0], B[1])
    del rng


def test_gridding_matches_oracle_and_is_deterministic():
    A = _A()
    torch = _torch()
    n = 256
    e = oplan.log_edges(3.0, 80.0, 12)
    p = A.Plan(n, e, max_batch=2, wmode=A.W_INV_COUNT).bind()
    uv, vis = synth.visibility_stream(200000, 80.0, 32.0, 1.0, seed=5, batch=2)
    uv[:7] = [[0.5, 0.5], [-0.5, 1.5], [300.0, 0.0], [127.6, 3.0], [-127.4, 0.0], [2.5, -2.5], [0, 0]]
    uvt = torch.from_numpy(uv).cuda()
    vt = torch.from_numpy(vis).cuda()
    g1, w1, d1 = p.grid(uvt, vt)
    g2, w2, d2 = p.grid(uvt, vt)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(w1, w2)
    for b in range(2):
        go, wo, dro = ogrid.grid_visibilities(n, 1.0, uv, vis[b])
        gg = g1[b].cpu().numpy()
        scale = np.abs(vis[b]).max()
        assert np.allclose(gg, go, rtol=2 ** -22, atol=2 ** -24 * scale)
        assert np.array_equal(w1.cpu().numpy(), wo.astype(np.float32))
        assert int(d1.item()) == dro
    # Gaussian kernel with per-visibility weights
    vw = np.random.default_rng(9).uniform(0.5, 1.5, len(uv)).astype(np.float32)
    g3, w3, _ = p.grid(uvt, vt, vis_w=torch.from_numpy(vw).cuda(), kernel=A.GAUSS7)
    go, wo, _ = ogrid.grid_visibilities(n, 1.0, uv, vis[0], vis_w=vw.astype(np.float64),
                                        kernel=ogrid.GAUSS7, theta0=p_theta0(p))
    assert np.allclose(g3[0].cpu().numpy(), go, rtol=1e-5, atol=1e-6 * np.abs(go).max())
    assert np.allclose(w3.cpu().numpy(), wo, rtol=1e-5, atol=1e-6 * wo.max())


@pytest.mark.parametrize("batch", [3, 18])
def test_gridding_batches(batch):
    """Odd batches (8-byte record loads) and batches over 16 (two gather passes), with
    per-visibility weights on the nearest-cell kernel."""
    A = _A()
    torch = _torch()
    n = 128
    p = A.Plan(n, oplan.log_edges(3.0, 40.0, 6), max_batch=batch, wmode=A.W_INV_COUNT).bind()
    uv, vis = synth.visibility_stream(40000, 40.0, 16.0, 1.0, seed=11 + batch, batch=batch)
    vw = np.random.default_rng(batch).uniform(0.5, 1.5, len(uv)).astype(np.float32)
    uvt, vt = torch.from_numpy(uv).cuda(), torch.from_numpy(vis).cuda()
    for w in (None, vw):
        g, ws, d = p.grid(uvt, vt, vis_w=None if w is None else torch.from_numpy(w).cuda())
        torch.cuda.synchronize()
        for b in range(batch):
            go, wo, dro = ogrid.grid_visibilities(n, 1.0, uv, vis[b],
                                                  vis_w=None if w is None else w.astype(np.float64))
            scale = np.abs(vis).max() * (1.0 if w is None else 1.5)
            assert np.allclose(g[b].cpu().numpy(), go, rtol=2 ** -22, atol=2 ** -23 * scale), (b, w is None)
            assert int(d.item()) == dro
        if w is None:
            assert np.array_equal(ws.cpu().numpy(), wo.astype(np.float32))
        else:
            assert np.allclose(ws.cpu().numpy(), wo, rtol=2 ** -22, atol=2 ** -22)


def p_theta0(p):
    return 0.6 * np.deg2rad(24.68)


def test_argument_errors():
    A = _A()
    torch = _torch()
    p = A.Plan(64, [2.0, 4.0, 8.0], max_batch=1)
    g = torch.zeros((1, 64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(A.AbsError) as ei:
        p._work = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
        p.device = g.device
        p.estimate(g)
    assert ei.value.status == 3               # not bound
    p.bind()
    with pytest.raises(A.AbsError) as ei:
        p.estimate(torch.zeros((2, 64, 64), dtype=torch.complex64, device="cuda"))
    assert ei.value.status == 1               # batch > max_batch
    q = A.Plan(64, [2.0, 4.0, 8.0], wmode=A.W_INV_COUNT).bind()
    with pytest.raises(A.AbsError):
        q.estimate(g)                         # weights required


# ---- precision form: BF16 / FP16 hi+lo split products on MFMA, FP32 accumulation ----


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_precision_form_c2(prec):
    """1024 x 1024 MWA-shaped grids, 20 rings, INV_COUNT weights shared by 2 grids:
    e_t <= 1e-4 on every triplet (FP64 weights, FP32 FFTs, split-precision contraction)."""
    A = _A()
    n = 1024
    e = oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)
    grids, counts = _mwa_inputs(n, 2, 1, seed0=200)
    P = {"bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=2, precision=P).bind()
    B, N = _run(p, grids.astype(np.complex64), counts)
    for b in range(2):
        ref = oest.estimate(grids[b].astype(np.complex64), counts, e, p.norm, wmode=1,
                            trips=p.triplets, with_scales=True)
        err = oest.relative_error(B[b], ref, p.norm)
        rel = np.abs(B[b] / ref["B"] - 1)
        print("%s C2[%d]: e_t median %.3g p99 %.3g max %.3g | raw rel median %.3g p99 %.3g"
              % (prec, b, np.median(err), np.quantile(err, 0.99), err.max(), np.median(rel),
                 np.quantile(rel, 0.99)), flush=True)
        _check(B[b], N[b], ref, p.norm, tol=PREC_TOL, label="%s C2[%d]" % (prec, b))


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,edges,flags", [SMALL[0], SMALL[1], SMALL[2], SMALL[4], SMALL[3]])
def test_precision_form_small(prec, n, edges, flags):
    """Small plans against the oracle; n = 16 has two 128-pixel chunks per block, fewer
    than the loads the kernel keeps in flight, so it also runs the phases past the block
    end (which stage zeros)."""
    A = _A()
    rng = np.random.default_rng(7 * n + flags)
    # a large dynamic range between rings exercises the per-ring FP16 scaling
    V = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))) * 1e3
    w = synth.symmetrize(rng.uniform(0.1, 2.0, (n, n)))
    P = {"bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    p = A.Plan(n, edges, norm=1.0, wmode=A.W_GIVEN, max_batch=2, flags=flags, precision=P).bind()
    B, N = _run(p, V, w)
    for b in range(2):
        ref = oest.estimate(V[b], w, edges, 1.0, wmode=2, trips=p.triplets, with_scales=True)
        _check(B[b], N[b], ref, 1.0, tol=PREC_TOL, label="%s n%d[%d]" % (prec, n, b))
