"""Serving form on the GPU: a mixed stream of requests (grid sizes, ring sets, shared
and per-request weights) through continuous batching on several streams gives, for
every request, exactly (bit for bit) the result of that request estimated alone."""
import numpy as np
import pytest

import synth
from oracle import plan as oplan

pytestmark = pytest.mark.gpu


def _mix(seed=3, nreq=24):
    import torch
    rng = np.random.default_rng(seed)
    reqs = []
    from paper_2412_02246_amd.serve import Request
    masks = {}
    for k in range(nreq):
        n = int(rng.choice([64, 128, 256]))
        nb = int(rng.integers(5, 9))
        edges = tuple(oplan.log_edges(2.0, n / 3.2, nb))
        V = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        shared = rng.random() < 0.5
        if shared:
            if n not in masks:
                masks[n] = synth.poisson_counts(n, 4.0, n / 8, rng)
            w, key = masks[n], ("chan", n)
        else:
            w, key = synth.poisson_counts(n, 4.0, n / 8, rng), None
        reqs.append(Request(k, n, edges, torch.from_numpy(V.astype(np.complex64)).cuda(),
                            torch.from_numpy(w.astype(np.float32)).cuda(), key,
                            arrival=0.0 if k < 16 else 1e-3 * (k - 15)))
    # the first 16 arrive together (requests 5 and 11 share a plan and per-request
    # weights, so one batch holds both whatever the timing); the rest trickle in
    return reqs


def test_results_identical_alone_and_in_the_mix():
    import torch
    import paper_2412_02246_amd as A
    from paper_2412_02246_amd.serve import GpuExecutor, Scheduler, latency_stats, run_stream
    reqs = _mix()
    ex = GpuExecutor(A.W_INV_COUNT, max_batch=4, slots=3)
    ex.prepare([r.plan_key for r in reqs])
    sched = Scheduler(ex, budget_bytes=1 << 30, max_batch=4, slots=3)
    done = run_stream(sched, reqs)
    torch.cuda.synchronize()
    assert sorted(c.rid for c in done) == list(range(len(reqs)))
    assert max(c.batch for c in done) > 1                  # some requests were batched
    st = latency_stats(done)
    print("serve mix: %s" % st, flush=True)
    for c in done:
        r = reqs[c.rid]
        p = ex.plans[r.plan_key]
        B1, N1 = p.estimate(r.grid.unsqueeze(0).contiguous(), r.weights)
        torch.cuda.synchronize()
        assert torch.equal(B1[0], c.B), c.rid
        assert torch.equal(N1[0], c.N), c.rid
