"""Serving form on the GPU, at the serving stream's shapes (grids of 512^2 .. 4096^2, 16 .. 32
log rings): a mixed stream of requests (realisations of two channels sharing their plan and
weights, and channels with their own) through continuous batching on several streams gives,
for every request, exactly (bit for bit) the result of that request estimated alone, and a
sample of served results (one request per grid size) matches the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest

pytestmark = pytest.mark.gpu

SIZES = (512, 1024, 2048, 4096)


def _edges(n, nb):
    s = n / 1024.0
    return tuple((46.0 * s / (2 * np.pi)) * (1320.0 / 46.0) ** (np.arange(nb + 1) / nb))


def _mix(seed=3, nreq=20):
    """(requests, host inputs): two channels (1024^2 / 20 rings and 4096^2 / 24 rings) with
    realisations, and channels of their own over the four sizes; the first 14 requests
    arrive together, the rest trickle in."""
    import torch
    from paper_2412_02246_amd.serve import Request
    rng = np.random.default_rng(seed)
    chans = {0: (1024, _edges(1024, 20)), 1: (4096, _edges(4096, 24))}
    chan_w = {c: synth.poisson_counts(n, 4.0, n / 8, rng) for c, (n, _) in chans.items()}
    reqs, host = [], []
    for k in range(nreq):
        if k % 2 == 0:
            c = (k // 2) % 2
            n, edges = chans[c]
            w, key = chan_w[c], ("chan", c)
        else:
            n = SIZES[(k // 2) % 4]
            edges = _edges(n, int(rng.integers(16, 33)))
            w, key = synth.poisson_counts(n, 4.0, n / 8, rng), None
        V = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64)
        host.append((V, w))
        reqs.append(Request(k, n, edges, torch.from_numpy(V).cuda(), torch.from_numpy(w.astype(np.float32)).cuda(),
                            key, arrival=0.0 if k < 14 else 2e-3 * (k - 13)))
    return reqs, host


def test_results_identical_alone_and_in_the_mix_and_match_the_oracle():
    import torch
    import paper_2412_02246_amd as A
    from paper_2412_02246_amd.serve import GpuExecutor, Scheduler, latency_stats, run_stream
    reqs, host = _mix()
    ex = GpuExecutor(A.W_INV_COUNT, max_batch=4, slots=3)
    ex.prepare([r.plan_key for r in reqs], workers=8)
    sched = Scheduler(ex, budget_bytes=48 << 30, max_batch=4, slots=3)
    done = run_stream(sched, reqs)
    torch.cuda.synchronize()
    assert sorted(c.rid for c in done) == list(range(len(reqs)))
    assert max(c.batch for c in done) > 1                  # channel realisations were batched
    st = latency_stats(done)
    print("serve mix: %s" % st, flush=True)
    by_rid = {c.rid: c for c in done}
    for c in done:
        r = reqs[c.rid]
        p = ex.plans[r.plan_key]
        if r.weights_key is not None:
            B1, N1 = p.estimate(r.grid.unsqueeze(0).contiguous(), r.weights,
                                n_given=ex.counts[(r.plan_key, r.weights_key)][0])
        else:
            B1, N1 = p.estimate(r.grid.unsqueeze(0).contiguous(), r.weights)
        torch.cuda.synchronize()
        assert torch.equal(B1[0], c.B), c.rid
        assert torch.equal(N1[0], c.N), c.rid
    # one served request per grid size against the oracle: every triplet at 512^2 and
    # 1024^2, the triplets within four rings spread over the range at 2048^2 and 4096^2
    checked = set()
    for r in reqs:
        if r.n in checked:
            continue
        checked.add(r.n)
        V, w = host[r.rid]
        p = ex.plans[r.plan_key]
        c = by_rid[r.rid]
        B, N = c.B.cpu().numpy(), c.N.cpu().numpy()
        if r.n <= 1024:
            idx = np.arange(p.ntrip)
            ref = oest.estimate(V, w, r.edges, p.norm, wmode=oest.INV_COUNT, trips=p.triplets, with_scales=True)
        else:
            nb = len(r.edges) - 1
            sub = {0, nb // 3, (2 * nb) // 3, nb - 1}
            idx = np.array([q for q, t in enumerate(p.triplets) if set(t.tolist()) <= sub])
            ref = oest.estimate_subset(V, w, r.edges, p.norm, p.triplets[idx], wmode=oest.INV_COUNT)
        B, N = B[idx], N[idx]
        assert np.array_equal(np.isnan(B), np.isnan(ref["B"]))
        ok = ~np.isnan(ref["B"])
        e = oest.relative_error(B, ref, p.norm)[ok]
        en = oest.count_error(N, ref)
        print("served n=%d rings=%d: max e_t %.3g, max e_N %.3g over %d triplets"
              % (r.n, len(r.edges) - 1, e.max(), en.max(), len(idx)), flush=True)
        assert len(idx) > 0 and e.max() <= 1e-5 and en.max() <= 1e-5
    assert checked == set(SIZES)
