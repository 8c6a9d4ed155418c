"""GPU tests of the estimate's second stream: when a call computes weight fields, they run
on the plan's own stream beside the data fields (forked from the call's stream, joined
back before the normalisation).  The results must be bit for bit those of the same call
with the weight fields run after the data fields on the call's stream (which is what a
column-pass timing hook selects), work queued on the call's stream after it must see the
whole result, and back-to-back calls on one stream must each get their own weights."""
import ctypes

import numpy as np
import pytest

from oracle import estimator as oest
from oracle import plan as oplan

pytestmark = pytest.mark.gpu

N_GRID = 256
EDGES = oplan.log_edges(3.0, 85.0, 16)   # every level: 256, 128, 64 and 32


def _weights(rng, n):
    w = rng.uniform(0.1, 2.0, (n, n))
    # real and symmetric under g -> -g (indices modulo n)
    return 0.5 * (w + np.roll(np.flip(w, (0, 1)), 1, (0, 1)))


class _Events:
    """Two raw HIP events for a timing hook (the runtime torch has loaded)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.ev = []
        for _ in range(2):
            e = ctypes.c_void_p()
            assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
            self.ev.append(e)

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)


def test_forked_weights_equal_serial_and_oracle():
    import torch

    import paper_2412_02246_amd as A
    from paper_2412_02246_amd import _lib as L
    rng = np.random.default_rng(515)
    V = rng.standard_normal((2, N_GRID, N_GRID)) + 1j * rng.standard_normal((2, N_GRID, N_GRID))
    w = _weights(rng, N_GRID).astype(np.float32).astype(np.float64)
    p = A.Plan(N_GRID, EDGES, norm=1.0, wmode=A.W_GIVEN, max_batch=2, flags=A.EVERY_LEVEL, levels=8).bind()
    assert len(p.levels) >= 2
    g = torch.from_numpy(V).to(torch.complex64).cuda()
    wt = torch.from_numpy(w.astype(np.float32)).cuda()
    # forked: on a side stream, the result consumed by work queued on that stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B1, N1 = p.estimate(g, wt, stream=s)
        N1x = N1 * 2.0
        B1c, N1c = B1.clone(), N1.clone()
    s.synchronize()
    # serial: a column-pass hook set
    ev = _Events()
    try:
        L.check(L.lib().abs_profile(p.handle, L.STAGE_COLPASS, ev.ev[0], ev.ev[1]), "abs_profile")
        B2, N2 = p.estimate(g, wt)
        torch.cuda.synchronize()
        L.check(L.lib().abs_profile(p.handle, L.STAGE_COLPASS, None, None), "abs_profile")
    finally:
        ev.close()
    assert np.array_equal(B1c.cpu().numpy(), B2.cpu().numpy(), equal_nan=True)
    assert torch.equal(N1c, N2)
    assert torch.equal(N1x, N2 * 2.0)
    for b in range(2):
        ref = oest.estimate(V[b], w, EDGES, 1.0, wmode=oest.GIVEN, trips=p.triplets, with_scales=True)
        keep = ~np.isnan(ref["B"])
        e = oest.relative_error(B2[b].cpu().numpy(), ref, 1.0)[keep]
        assert e.max() <= 1e-5, e.max()
        assert oest.count_error(N2[b].cpu().numpy(), ref).max() <= 1e-5


def test_back_to_back_calls_keep_their_weights():
    """Four calls queued on one stream without synchronising, each with other weights and
    all on the same workspace: every result equals that call run alone."""
    import torch

    import paper_2412_02246_amd as A
    rng = np.random.default_rng(516)
    p = A.Plan(N_GRID, EDGES, norm=1.0, wmode=A.W_GIVEN, max_batch=1, flags=A.EVERY_LEVEL, levels=8).bind()
    gs, ws = [], []
    for _ in range(4):
        V = rng.standard_normal((N_GRID, N_GRID)) + 1j * rng.standard_normal((N_GRID, N_GRID))
        gs.append(torch.from_numpy(V).to(torch.complex64).cuda())
        ws.append(torch.from_numpy(_weights(rng, N_GRID).astype(np.float32)).cuda())
    outs = []
    for g, wt in zip(gs, ws):
        # one workspace for all four (the plan's own), outputs copied on the call's stream
        B, N = p.estimate(g, wt)
        outs.append((B.clone(), N.clone()))
    torch.cuda.synchronize()
    for (B, N), g, wt in zip(outs, gs, ws):
        B0, N0 = p.estimate(g, wt)
        torch.cuda.synchronize()
        assert np.array_equal(B.cpu().numpy(), B0.cpu().numpy(), equal_nan=True)
        assert torch.equal(N, N0)
