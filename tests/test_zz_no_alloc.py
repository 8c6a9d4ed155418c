"""abs_estimate_noalloc (the entry point for callers that cannot allocate device memory)
against abs_estimate, through the C ABI: two calls in a row on the static scratch, the
second with a smaller input, each bit for bit equal to the caller-workspace entry point;
a call that needs more than the scratch is refused before anything is launched."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import plan as oplan

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _noalloc(plan, grids, w, w_batched=False, n_given=None):
    import torch
    import paper_2412_02246_amd as A
    L = A._lib
    batch = grids.shape[0]
    B = torch.full((batch, plan.ntrip), -1.0, dtype=torch.float64, device=grids.device)
    N = torch.full((batch, plan.ntrip), -1.0, dtype=torch.float64, device=grids.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = L.lib().abs_estimate_noalloc(plan.handle, batch, L.C64, _p(grids), _p(w), int(w_batched),
                                     _p(n_given), _p(B), _p(N), st)
    return s, B, N


def test_noalloc_matches_workspace_entry_point():
    import torch
    import paper_2412_02246_amd as A
    n = 256
    e = oplan.log_edges(3.0, 80.0, 13)
    rng = np.random.default_rng(2024)
    V = (rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))).astype(np.complex64)
    w = np.stack([synth.poisson_counts(n, 4.0, n / 8, rng) for _ in range(3)]).astype(np.float32)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=3).bind()
    g = torch.from_numpy(V).cuda()
    wt = torch.from_numpy(w).cuda()
    # first call: three grids with their own weights
    s, B3, N3 = _noalloc(p, g, wt, w_batched=True)
    assert s == A._lib.OK, A._lib.status_str(s)
    Bw, Nw = p.estimate(g, wt, w_batched=True)
    torch.cuda.synchronize()
    assert torch.equal(B3, Bw) and torch.equal(N3, Nw)
    # second call, smaller: one grid with shared weights, on the scratch the first call used
    s, B1, N1 = _noalloc(p, g[2:3].contiguous(), wt[0])
    assert s == A._lib.OK, A._lib.status_str(s)
    Bs, Ns = p.estimate(g[2:3].contiguous(), wt[0])
    torch.cuda.synchronize()
    assert torch.equal(B1, Bs) and torch.equal(N1, Ns)
    assert not torch.equal(B1[0], B3[2])           # other weights, other result
    # a third plan size on the same scratch, with cached counts
    q = A.Plan(128, oplan.log_edges(2.0, 42.0, 8), wmode=A.W_INV_COUNT).bind()
    g2 = torch.from_numpy(V[0, ::2, ::2].copy()).cuda().unsqueeze(0)
    w2 = torch.from_numpy(w[0, ::2, ::2].copy()).cuda()
    Ng = q.counts(w2)
    s, Bq, Nq = _noalloc(q, g2, w2, n_given=Ng)
    assert s == A._lib.OK, A._lib.status_str(s)
    Bq2, Nq2 = q.estimate(g2, w2, n_given=Ng)
    torch.cuda.synchronize()
    assert torch.equal(Bq, Bq2) and torch.equal(Nq, Nq2)


def test_noalloc_refuses_workspaces_beyond_the_scratch():
    import torch
    import paper_2412_02246_amd as A
    n = 1024
    e = oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=4).bind()
    assert p.estimate_workspace(4, w_batched=True) > (256 << 20)
    g = torch.zeros((4, n, n), dtype=torch.complex64, device="cuda")
    w = torch.ones((4, n, n), dtype=torch.float32, device="cuda")
    s, B, _ = _noalloc(p, g, w, w_batched=True)
    torch.cuda.synchronize()
    assert s == A._lib.ERR_SCRATCH
    assert bool((B == -1.0).all())                 # nothing was launched
