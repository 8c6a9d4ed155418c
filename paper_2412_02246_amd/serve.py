"""Serving form: continuous batching of bispectrum estimates on one GPU.

Requests (one gridded channel or one realisation each, any supported grid size and
ring set) arrive over time.  The scheduler keeps a FIFO of pending requests and, each
time it is stepped:

* retires finished batches (their memory returns to the budget, their slot frees up);
* admits work while a slot (a HIP stream) is free: the oldest pending request opens a
  batch and takes the later pending requests that share its plan and its weighting
  (the same weights for realisations of one channel, whose triangle counts N_t are
  then computed once and reused; separate weights per grid for channels), up to
  max_batch, shrinking the batch until its device footprint fits the free budget.

Batches run concurrently on separate streams, so requests that arrive while others
are on the GPU join as soon as a slot and memory are free, and their work overlaps on
the device.  Results do not depend on how requests were batched: every kernel treats
each grid of a batch independently and reduces in a fixed order, so a result is bit
for bit the one the request gets alone.

The scheduler only talks to an executor (footprint / launch / done / result), so the
policy is exercised on the CPU with a simulated executor and on the GPU with
GpuExecutor, which drives libabs.so through Plan.
"""
import collections
import time


class Request:
    """One estimate.  grid: complex64 [n][n]; weights: float32 [n][n] (plan wmode);
    weights_key: requests with equal non-None keys share their weights (realisations of
    one channel); None means the weights belong to this request alone."""

    __slots__ = ("rid", "n", "edges", "grid", "weights", "weights_key", "arrival")

    def __init__(self, rid, n, edges, grid, weights, weights_key=None, arrival=0.0):
        self.rid, self.n, self.edges = rid, int(n), tuple(float(e) for e in edges)
        self.grid, self.weights, self.weights_key, self.arrival = grid, weights, weights_key, float(arrival)

    @property
    def plan_key(self):
        return (self.n, self.edges)


class Completion:
    __slots__ = ("rid", "B", "N", "arrival", "admitted", "done", "batch")

    def __init__(self, rid, B, N, arrival, admitted, done, batch):
        self.rid, self.B, self.N = rid, B, N
        self.arrival, self.admitted, self.done, self.batch = arrival, admitted, done, batch

    @property
    def latency(self):
        return self.done - self.arrival


class Scheduler:
    """Continuous batching with admission by device footprint (bytes)."""

    def __init__(self, executor, budget_bytes, max_batch=8, slots=4):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.slots = int(slots)
        self.pending = collections.deque()
        self.inflight = {}          # handle -> (requests, footprint, admitted time)
        self.used = 0
        self.peak_used = 0
        self.rejected = []

    def submit(self, req):
        self.pending.append(req)

    def idle(self):
        return not self.pending and not self.inflight

    def _compatible(self, head, r):
        if r.plan_key != head.plan_key:
            return False
        if head.weights_key is None:
            return r.weights_key is None
        return r.weights_key == head.weights_key

    def _admit(self, now):
        while self.pending and len(self.inflight) < self.slots:
            head = self.pending[0]
            group = [head]
            for r in list(self.pending)[1:]:
                if len(group) >= self.max_batch:
                    break
                if self._compatible(head, r):
                    group.append(r)
            # the largest prefix of the group that fits the free budget
            while group:
                fp = self.ex.footprint(group)
                if self.used + fp <= self.budget:
                    break
                group.pop()
            if not group:
                if self.ex.footprint([head]) > self.budget:
                    self.pending.popleft()         # can never fit: reject it
                    self.rejected.append(head.rid)
                    continue
                return                              # wait for memory to free up
            for r in group:
                self.pending.remove(r)
            handle = self.ex.launch(group)
            self.inflight[handle] = (group, fp, now)
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)

    def step(self, now):
        """Retire finished batches, then admit.  Returns the completions seen now."""
        out = []
        for h in [h for h in self.inflight if self.ex.done(h)]:
            group, fp, t_adm = self.inflight.pop(h)
            self.used -= fp
            for r, (B, N) in zip(group, self.ex.result(h)):
                out.append(Completion(r.rid, B, N, r.arrival, t_adm, now, len(group)))
        self._admit(now)
        return out


def run_stream(sched, requests, clock=time.perf_counter, spin=lambda: None):
    """Feed requests at their arrival times (seconds from the start) and step the
    scheduler until every request has completed.  Returns the completions."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    done, k = [], 0
    while k < len(reqs) or not sched.idle():
        now = clock() - t0
        while k < len(reqs) and reqs[k].arrival <= now:
            sched.submit(reqs[k])
            k += 1
        done.extend(sched.step(now))
        spin()
    return done


def latency_stats(done):
    import numpy as np
    lat = np.array([c.latency for c in done])
    t_first = min(c.arrival for c in done)
    t_last = max(c.done for c in done)
    return {"requests": len(done), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean()),
            "grids_per_s": len(done) / max(t_last - t_first, 1e-12),
            "mean_batch": float(np.mean([c.batch for c in done]))}


class GpuExecutor:
    """Runs batches through libabs.so plans on their own HIP streams.

    Plans (and their device tables) stay resident for the executor's lifetime, one per
    (n, edges); triangle counts for shared weights are computed once per weights_key and
    reused (abs_counts, then abs_estimate with n_given)."""

    def __init__(self, wmode, precision=0, max_batch=8, slots=4, device=0):
        import torch
        from . import _lib as L
        self.torch, self.L = torch, L
        self.wmode, self.precision, self.max_batch = wmode, precision, max_batch
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.free_streams = list(range(slots))
        self.plans = {}
        self.counts = {}             # (plan_key, weights_key) -> (N tensor, event)
        self.jobs = {}
        self._next = 0

    def plan(self, key):
        from .plan import Plan
        p = self.plans.get(key)
        if p is None:
            n, edges = key
            p = Plan(n, edges, wmode=self.wmode, precision=self.precision,
                     max_batch=self.max_batch).bind(self.device.index)
            self.plans[key] = p
        return p

    def prepare(self, keys, workers=1):
        """Create the plans for these keys, compile their kernels (in `workers` worker
        processes when > 1; start those before this process first uses the GPU), and
        bind them to the device."""
        from .jit import compile_parts
        from .plan import Plan
        keys = [k for k in dict.fromkeys(keys) if k not in self.plans]
        kw = dict(wmode=self.wmode, precision=self.precision, max_batch=self.max_batch)
        made = [Plan(n, e, **kw) for n, e in keys]
        compile_parts(made, [(n, e, kw) for n, e in keys], workers=workers)
        for k, p in zip(keys, made):
            self.plans[k] = p.bind(self.device.index)

    def _layout(self, group):
        p = self.plan(group[0].plan_key)
        shared = group[0].weights_key is not None
        have_counts = shared
        work = p.estimate_workspace(len(group), w_batched=not shared, have_counts=have_counts)
        if shared and (group[0].plan_key, group[0].weights_key) not in self.counts:
            work = max(work, p.estimate_workspace(0))
        n2 = p.n * p.n
        stacked = len(group) * n2 * 8 + (0 if shared else len(group) * n2 * 4)
        outputs = 2 * len(group) * p.ntrip * 8
        return p, shared, work, stacked + outputs

    def footprint(self, group):
        _, _, work, rest = self._layout(group)
        return work + rest

    def launch(self, group):
        torch = self.torch
        p, shared, work_bytes, _ = self._layout(group)
        sid = self.free_streams.pop()
        st = self.streams[sid]
        with torch.cuda.stream(st):
            work = torch.empty(work_bytes, dtype=torch.uint8, device=self.device)
            grids = torch.stack([r.grid for r in group])
            n_given = None
            if shared:
                key = (group[0].plan_key, group[0].weights_key)   # counts belong to a plan
                w = group[0].weights
                if key not in self.counts:
                    N0 = p.counts(w, work=work)
                    ev = torch.cuda.Event()
                    ev.record(st)
                    self.counts[key] = (N0, ev)
                n_given, ev = self.counts[key]
                st.wait_event(ev)
            else:
                w = torch.stack([r.weights for r in group])
            B, N = p.estimate(grids, w, w_batched=not shared, n_given=n_given, work=work)
            done = torch.cuda.Event()
            done.record(st)
        h = self._next
        self._next += 1
        # keep every buffer alive until the batch has finished on its stream
        self.jobs[h] = (sid, done, (B, N), (work, grids, w))
        return h

    def done(self, h):
        return self.jobs[h][1].query()

    def result(self, h):
        sid, _, (B, N), _ = self.jobs.pop(h)
        self.free_streams.append(sid)
        return [(B[i], N[i]) for i in range(B.shape[0])]
