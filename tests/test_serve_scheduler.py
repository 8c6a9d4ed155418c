"""The serving scheduler's policy on the CPU, with a simulated executor: continuous
batching, admission by footprint, FIFO order, rejection of requests that can never
fit, and latency accounting."""
import numpy as np

from paper_2412_02246_amd.serve import Request, Scheduler, latency_stats, run_stream


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-4):
        self.t += dt


class FakeExecutor:
    """Batches take a + b * n^2 * len(batch) seconds of simulated time; the footprint is
    proportional to n^2 per grid (shared weights are cheaper)."""

    def __init__(self, clock, slots):
        self.clock, self.jobs, self.k = clock, {}, 0
        self.launched = []
        self.free = slots

    def footprint(self, group):
        n2 = group[0].n ** 2
        per = 3 if group[0].weights_key is not None else 5
        return per * n2 * len(group)

    def launch(self, group):
        assert self.free > 0
        self.free -= 1
        dur = 1e-3 + 1e-9 * group[0].n ** 2 * len(group)
        self.k += 1
        self.jobs[self.k] = (self.clock() + dur, group)
        self.launched.append([r.rid for r in group])
        return self.k

    def done(self, h):
        return self.clock() >= self.jobs[h][0]

    def result(self, h):
        _, group = self.jobs.pop(h)
        self.free += 1
        return [(r.rid, None) for r in group]


def _requests(nreq, seed, rate):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, nreq))
    out = []
    for k in range(nreq):
        n = int(rng.choice([256, 512, 1024]))
        nb = int(rng.integers(16, 20))
        edges = tuple(np.linspace(2, n / 4, nb + 1))
        key = ("chan", n) if rng.random() < 0.5 else None
        out.append(Request(k, n, edges, None, None, key, t[k]))
    return out


def _run(nreq=300, rate=2000.0, budget=40 * 1024 ** 2, slots=3, max_batch=4, seed=1):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots)
    sched = Scheduler(ex, budget, max_batch=max_batch, slots=slots)
    done = run_stream(sched, _requests(nreq, seed, rate), clock=clock, spin=clock.advance)
    return sched, ex, done


def test_every_request_completes_once_within_budget():
    sched, ex, done = _run()
    assert sorted(c.rid for c in done) == list(range(300))
    assert sched.peak_used <= sched.budget
    assert sched.used == 0 and not sched.inflight
    # results come back in the request's own slot of its batch
    assert all(c.B == c.rid for c in done)


def test_batches_share_plan_and_weighting_and_respect_max_batch():
    sched, ex, done = _run()
    reqs = {r.rid: r for r in _requests(300, 1, 2000.0)}
    assert any(len(b) > 1 for b in ex.launched)          # batching happened
    for b in ex.launched:
        assert len(b) <= 4
        head = reqs[b[0]]
        for rid in b:
            r = reqs[rid]
            assert r.plan_key == head.plan_key
            assert r.weights_key == head.weights_key
        assert b == sorted(b)                              # FIFO inside a batch


def test_fifo_admission_heads():
    sched, ex, done = _run(rate=500.0)
    heads = [b[0] for b in ex.launched]
    assert heads == sorted(heads)                          # batch heads leave in arrival order


def test_footprint_admission_binds_under_a_small_budget():
    small = 4 * 1024 ** 2                                  # one 1024^2 batch of 1 takes 5 MiB
    sched, ex, done = _run(budget=small)
    assert sched.peak_used <= small
    reqs = {r.rid: r for r in _requests(300, 1, 2000.0)}
    # 1024^2 requests with their own weights (5 MiB) can never fit: rejected, not hung
    for rid in sched.rejected:
        assert reqs[rid].n == 1024
    assert len(done) + len(sched.rejected) == 300


def test_latency_accounting():
    sched, ex, done = _run(rate=100.0)                     # light load: no queueing
    st = latency_stats(done)
    assert st["requests"] == 300
    for c in done:
        assert c.done >= c.admitted >= c.arrival
    assert st["p50_ms"] <= st["p99_ms"]
    # at light load the latency is about the simulated execution time (+ polling step)
    assert st["p50_ms"] < 3.0
