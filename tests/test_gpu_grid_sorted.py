"""GPU parity of gridding on a baseline set sorted once (abs_grid_sort, abs_grid_permute,
abs_grid_sorted), Eq. (9) with the nearest cell and unit weights: against the FP64
oracle element by element, bit for bit against abs_grid on the same visibilities, with
the slot order checked against its definition, and at the 8192^2 / 8-realisation shape
the throughput runs time (sampled cells against the oracle, every cell against abs_grid)."""
import numpy as np
import pytest

import synth
from oracle import gridding as ogrid
from oracle import plan as oplan

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _A():
    import paper_2412_02246_amd as A
    return A


def _slot_keys(n, uv, du=1.0):
    """The documented slot order's key of each baseline: 2 lc for a visibility nearest to
    the representative cell of pair lc, 2 lc + 1 for one nearest to its mirror, -1 when
    dropped.  Representatives: rows 0 .. n/2, in rows 0 and n/2 columns 0 .. n/2."""
    gx = np.rint(uv[:, 0] / du).astype(np.int64)
    gy = np.rint(uv[:, 1] / du).astype(np.int64)
    half = n // 2
    keep = (np.abs(gx) < half) & (np.abs(gy) < half)
    iy, ix = gy % n, gx % n
    rep = (iy <= half) & ~(((iy == 0) | (iy == half)) & (ix > half))
    my, mx = (-gy) % n, (-gx) % n
    key = np.where(rep, 2 * (iy * n + ix), 2 * (my * n + mx) + 1)
    return np.where(keep, key, -1)


def _check_set(bset, n, uv):
    kept = bset.kept
    perm = bset.perm.cpu().numpy()
    keys = _slot_keys(n, uv)
    assert kept == int((keys >= 0).sum())
    assert np.all(perm[kept:] == -1)
    # the kept baselines, each exactly once, in non-decreasing key order
    assert np.array_equal(np.sort(perm[:kept]), np.flatnonzero(keys >= 0))
    assert np.all(np.diff(keys[perm[:kept]]) >= 0)


@pytest.mark.parametrize("batch", [1, 2, 3, 18])
def test_sorted_matches_oracle_and_abs_grid(batch):
    A = _A()
    torch = _torch()
    n = 256
    p = A.Plan(n, oplan.log_edges(3.0, 80.0, 12), max_batch=batch, wmode=A.W_INV_COUNT).bind()
    uv, vis = synth.visibility_stream(150000, 80.0, 32.0, 1.0, seed=40 + batch, batch=batch)
    # hand-placed: half-integer ties, off-grid, the DC cell, the rows and columns -n/2, the
    # representative rows 0 and n/2 on both sides of column n/2
    uv[:10] = [[0.5, 0.5], [-0.5, 1.5], [300.0, 0.0], [127.6, 3.0], [-127.4, 0.0], [2.5, -2.5],
               [0.0, 0.0], [-128.0, 5.0], [100.0, 0.0], [-100.0, 0.0]]
    uvt, vt = torch.from_numpy(uv).cuda(), torch.from_numpy(vis).cuda()
    bset = p.grid_sort(uvt)
    _check_set(bset, n, uv)
    vs = bset.permute(vt)
    g, ws = p.grid_sorted(bset, vs, wsum=True)
    g0, w0, d0 = p.grid(uvt, vt)
    torch.cuda.synchronize()
    assert torch.equal(g, g0), "sorted and unsorted gridding differ"
    assert torch.equal(ws, w0) and torch.equal(bset.wsum, w0)
    assert bset.kept + int(d0.item()) == len(uv)
    for b in range(batch):
        go, wo, dro = ogrid.grid_visibilities(n, 1.0, uv, vis[b])
        scale = np.abs(vis[b]).max()
        assert np.allclose(g[b].cpu().numpy(), go, rtol=2 ** -22, atol=2 ** -24 * scale), b
        assert np.array_equal(ws.cpu().numpy(), wo.astype(np.float32))
        assert bset.kept == len(uv) - dro


@pytest.mark.parametrize("tiny", [False, True])
def test_sorted_is_independent_of_the_order_in_a_cell_and_of_padding(tiny):
    """Every cell's run reversed, a second sort, slots padded past the kept count, and a
    plane cut short (only its slots are gridded).  With `tiny`, every 53rd visibility is
    scaled by 1e-12, so that the cells holding one sum values whose magnitudes span more
    than an FP64 sum keeps exactly (the fixed-point form)."""
    A = _A()
    torch = _torch()
    n = 128
    p = A.Plan(n, oplan.log_edges(3.0, 40.0, 6), max_batch=4, wmode=A.W_INV_COUNT).bind()
    # few distinct baselines, many visibilities each: long runs in every cell
    rng = np.random.default_rng(77)
    cells = rng.integers(-20, 21, (40, 2)).astype(np.float64)
    uv = cells[rng.integers(0, 40, 30000)] + rng.uniform(-0.45, 0.45, (30000, 2))
    vis = (rng.standard_normal((4, 30000)) + 1j * rng.standard_normal((4, 30000))).astype(np.complex64)
    if tiny:
        vis[:, ::53] *= np.float32(1e-12)
    uvt, vt = torch.from_numpy(uv).cuda(), torch.from_numpy(vis).cuda()
    s1, s2 = p.grid_sort(uvt), p.grid_sort(uvt)
    _check_set(s2, n, uv)
    vs = s1.permute(vt)
    g1 = p.grid_sorted(s1, vs)
    # the same slots with every key's run reversed
    keys = _slot_keys(n, uv)[s1.perm[:s1.kept].cpu().numpy()]
    rev = np.lexsort((-np.arange(s1.kept), keys))
    grev = p.grid_sorted(s1, vs[torch.from_numpy(rev).cuda()].contiguous())
    g2 = p.grid_sorted(s2, s2.permute(vt))
    gpad = p.grid_sorted(s1, s1.permute(vt, ld=len(uv)))
    cut = s1.kept // 3
    gcut, wcut = p.grid_sorted(s1, s1.permute(vt, ld=cut), wsum=True)
    g0, _, _ = p.grid(uvt, vt)
    torch.cuda.synchronize()
    assert not np.array_equal(rev, np.arange(s1.kept))
    assert torch.equal(g1, grev) and torch.equal(g1, g2) and torch.equal(g1, gpad) and torch.equal(g1, g0)
    sel = s1.perm[:cut].cpu().numpy()
    for b in range(4):
        go, wo, _ = ogrid.grid_visibilities(n, 1.0, uv, vis[b])
        assert np.allclose(g1[b].cpu().numpy(), go, rtol=2 ** -22, atol=2 ** -22 * np.abs(vis[b]).max())
        go, wo, _ = ogrid.grid_visibilities(n, 1.0, uv[sel], vis[b][sel])
        assert np.allclose(gcut[b].cpu().numpy(), go, rtol=2 ** -22, atol=2 ** -22 * np.abs(vis[b]).max())
    assert np.array_equal(wcut.cpu().numpy(), wo.astype(np.float32))


def test_sorted_empty_and_all_dropped():
    A = _A()
    torch = _torch()
    n = 64
    p = A.Plan(n, oplan.log_edges(2.0, 20.0, 4), max_batch=2).bind()
    for uv in (np.zeros((0, 2)), np.array([[40.0, 0.0], [0.0, -32.0], [1e9, 1.0]])):
        uvt = torch.from_numpy(uv).cuda()
        bset = p.grid_sort(uvt)
        assert bset.kept == 0
        vt = torch.ones((2, len(uv)), dtype=torch.complex64, device="cuda")
        g, ws = p.grid_sorted(bset, bset.permute(vt, ld=len(uv)), wsum=True)
        torch.cuda.synchronize()
        assert not g.abs().any() and not ws.any() and not bset.wsum.any()
        if len(uv):
            assert np.all(bset.perm.cpu().numpy() == -1)


def test_sorted_argument_checks():
    A = _A()
    torch = _torch()
    p = A.Plan(64, oplan.log_edges(2.0, 20.0, 4), max_batch=2).bind()
    uvt = torch.zeros((10, 2), dtype=torch.float64, device="cuda")
    bset = p.grid_sort(uvt)
    with pytest.raises(A.AbsError):
        p.grid_sorted(bset, torch.zeros((3, 10), dtype=torch.complex64, device="cuda"))   # batch > max_batch
    with pytest.raises(A.AbsError):
        bset.permute(torch.zeros((1, 10), dtype=torch.complex64, device="cuda"), ld=11)   # ld > nvis
    q = A.Plan(128, oplan.log_edges(2.0, 20.0, 4)).bind()
    with pytest.raises(ValueError):
        q.grid_sorted(bset, torch.zeros((1, 10), dtype=torch.complex64, device="cuda"))


def test_sorted_full_size_8192():
    """8192^2 grid, 8192^2 MWA-shaped baselines, 16 realisations (the throughput workload's
    launch: 8 lanes a pair, 512-thread blocks): every cell bit for bit against abs_grid, and
    64 cells (dense short baselines, the band edges, both sides of the half plane) against
    the oracle over the visibilities that reach them."""
    A = _A()
    torch = _torch()
    n, batch = 8192, 16
    e = oplan.log_edges(8 * 46 / (2 * np.pi), 8 * 1320 / (2 * np.pi), 64)
    # gridding uses only the plan's n, du and max_batch: a few rings keep its bind cheap
    p = A.Plan(n, e[:5], wmode=A.W_INV_COUNT, max_batch=batch, levels=1).bind()
    uv_d, vis_d = synth.mwa_visibilities_device(n, n * n, e[-1], synth.seed_for(5, 0), batch=batch)
    print("full size: inputs drawn", flush=True)
    bset = p.grid_sort(uv_d)
    vs = bset.permute(vis_d)
    g = p.grid_sorted(bset, vs)
    torch.cuda.synchronize()
    del vs
    print("full size: sorted grid done, kept %d of %d" % (bset.kept, n * n), flush=True)
    g0, w0, d0 = p.grid(uv_d, vis_d)
    torch.cuda.synchronize()
    assert torch.equal(g, g0), "sorted and unsorted gridding differ at 8192^2"
    assert torch.equal(bset.wsum, w0) and bset.kept + int(d0.item()) == n * n
    del g0
    p._work = None
    torch.cuda.empty_cache()
    rng = np.random.default_rng(8192)
    cy = np.concatenate([rng.integers(-40, 41, 24), rng.integers(-3000, 3001, 32), [0, 0, 4095, -4095, 1, -1, 7, 2000]])
    cx = np.concatenate([rng.integers(-40, 41, 24), rng.integers(-3000, 3001, 32), [0, 4095, 0, 3, -4095, 4095, -7, -2000]])
    uv = uv_d.cpu().numpy()
    gx, gy = np.rint(uv[:, 0]), np.rint(uv[:, 1])
    want = set(zip(cy.tolist(), cx.tolist())) | set(zip((-cy).tolist(), (-cx).tolist()))
    # visibilities within one cell of a sampled cell or its mirror (a superset: the oracle
    # places them)
    codes = np.array([a * 65536 + b for a, b in want], np.float64)
    near = np.zeros(len(uv), bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.isin((gy + dy) * 65536 + (gx + dx), codes)
    sel = np.flatnonzero(near)
    print("full size: %d visibilities reach the %d sampled cells" % (len(sel), len(cy)), flush=True)
    vsel = vis_d[:, torch.from_numpy(sel).cuda()].cpu().numpy()
    gs = g[:, torch.from_numpy(cy % n).cuda(), torch.from_numpy(cx % n).cuda()].cpu().numpy()
    for b in range(batch):
        go, wo, _ = ogrid.grid_visibilities(n, 1.0, uv[sel], vsel[b])
        ref = go[cy % n, cx % n]
        scale = np.abs(vsel[b]).max()
        assert np.allclose(gs[b], ref, rtol=2 ** -22, atol=2 ** -24 * scale), b
        if b == 0:
            assert np.array_equal(bset.wsum.cpu().numpy()[cy % n, cx % n], wo[cy % n, cx % n].astype(np.float32))


def test_sorted_multifrequency_channels():
    """A multi-frequency plan grids C channel grids per multi-frequency grid: 2 grids of 3
    channels sharing one baseline set, bit for bit the general call's grids, and the
    estimate from them equal to the estimate from the general call's grids."""
    A = _A()
    torch = _torch()
    n, C, batch = 128, 3, 2
    e = oplan.log_edges(3.0, 40.0, 6)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=batch, nchan=C).bind()
    uv, vis = synth.visibility_stream(60000, 40.0, 16.0, 1.0, seed=321, batch=batch * C)
    uvt, vt = torch.from_numpy(uv).cuda(), torch.from_numpy(vis).cuda()
    bset = p.grid_sort(uvt)
    g, ws = p.grid_sorted(bset, bset.permute(vt), wsum=True)
    g0, w0, _ = p.grid(uvt, vt)
    B, N = p.estimate(g, ws)
    B0, N0 = p.estimate(g0, w0)
    torch.cuda.synchronize()
    assert g.shape == (batch * C, n, n)
    assert torch.equal(g, g0) and torch.equal(ws, w0)
    assert np.array_equal(B.cpu().numpy(), B0.cpu().numpy(), equal_nan=True) and torch.equal(N, N0)
    for b in range(batch * C):
        go, _, _ = ogrid.grid_visibilities(n, 1.0, uv, vis[b])
        assert np.allclose(g[b].cpu().numpy(), go, rtol=2 ** -22, atol=2 ** -24 * np.abs(vis[b]).max()), b
