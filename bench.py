"""Throughput of the bispectrum hot path on one MI355X.

One step = gridding of nvis = n^2 visibilities for a batch of realisations of one
MWA-shaped channel (shared baselines, Eq. 9) followed by the estimator of Eq. (12)
for the batch (ring FFTs, triplet contraction, normalisation), with the gridded
counts as INV_COUNT weights: every step recomputes the weight fields and the triangle
counts N_t from those counts.  Inputs are resident in HBM before timing.  The baseline
set is sorted once before timing (abs_grid_sort; the realisations of every step share
it) and the visibilities are held in its slot order, so a step's gridding reads each
value once (abs_grid_sorted); the one-off sort, the permutation and the general
gridding call (abs_grid, which sorts on every call) are timed once and reported under
"baseline_set".

The default line is the large-ensemble shapes (8192^2 grids, 64 log rings, 15,229
triplets, realisations in batches of 16) in the plain FP32 form; it also carries, as
extra keys, the same workload in the BF16x3 and FP16x3 precision forms, the 1024^2 / 20-ring
single-channel workload, and the serving form's saturated rate and latencies.

Prints one JSON line: grids/s, bin-triplets/s, the roofline of the dominant kernel
(the triplet contraction; its duration comes from HIP events recorded by the library
around that launch on the call's stream) and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # MWA-shaped single channel: 1024^2 complex64, 20 log rings over 46 <= l < 1320
    "mwa1024": dict(n=1024, nbins=20, lmin=46.0, lmax=1320.0, batch=16, cfg=1,
                    desc="MWA-shaped single channel: 1024x1024 c64 grids, 20 log rings 46<=l<1320, "
                         "Poisson-density baselines + SNR-5 noise, INV_COUNT weights, 16 realisations a step"),
    # precision-form shapes: 4096^2, 32 log rings, edges x4
    "mwa4096": dict(n=4096, nbins=32, lmin=4 * 46.0, lmax=4 * 1320.0, batch=16, cfg=2,
                    desc="MWA-shaped 4096x4096 c64 grids, 32 log rings 4x(46<=l<1320), INV_COUNT weights, "
                         "16 realisations a step"),
    # large ensemble shapes: 8192^2, 64 log rings, edges x8 (realisations in batches of 16:
    # about 195 GiB of estimator workspace, which amortises the weight fields over 16 grids)
    "mwa8192": dict(n=8192, nbins=64, lmin=8 * 46.0, lmax=8 * 1320.0, batch=16, cfg=4,
                    desc="large ensemble: 8192x8192 c64 grids, 64 log rings 8x(46<=l<1320) (15229 triplets), "
                         "realisations of one channel, 16 a step, INV_COUNT weights from the gridded counts"),
    # multi-frequency form: 4 channels of the 1024^2 channel's geometry, 16 log rings; each
    # step grids and estimates 4 multi-frequency grids (16 channel grids), every channel
    # triplet (ring triplet x channel combination)
    "mf1024": dict(n=1024, nbins=16, lmin=46.0, lmax=1320.0, batch=4, cfg=1, nchan=4,
                   desc="multi-frequency: 4 channels of 1024x1024 c64 grids, 16 log rings 46<=l<1320, every "
                        "channel triplet, 4 multi-frequency grids (16 channel grids) a step, INV_COUNT weights"),
}
DEFAULT_WORKLOAD = "mwa8192"


class HipEvents:
    """Raw HIP events (the library records them on the call's stream)."""

    def __init__(self, count):
        import ctypes
        self._c = ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7")   # the runtime torch already loaded
        self.ev = []
        for _ in range(2 * count):
            e = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e)

    def pair(self, k):
        return self.ev[2 * k], self.ev[2 * k + 1]

    def elapsed_ms(self, k):
        ms = self._c.c_float()
        a, b = self.pair(k)
        if self.hip.hipEventElapsedTime(self._c.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)
        self.ev = []


# MI355X published peaks
PEAK_FP32_VECTOR = 157.3e12   # FP32 vector (counts packed dual-issue FP32)
PEAK_VALU_NONPACKED = 78.6e12  # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz: one FP32 FMA a lane
                               # and clock, the ceiling without packed FP32, which this library
                               # does not use
PEAK_MFMA_16BIT = 2.5e15       # dense BF16 / FP16 matrix peak
PEAK_HBM = 8.0e12

# HBM bytes per launch of the timed contraction kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by a 1 GiB copy (2.0 x FETCH_SIZE + 1.0 x WRITE_SIZE), for the
# kernels as they stand in this tree and the workload's default batch, summed over the level launches
# (profiles/counters_mwa8192_batch16.md, profiles/counters_mwa4096_batch16.md); keyed by
# (workload, precision).  A workload or precision without an entry reports null.
MEASURED_TRAFFIC = {("mwa8192", "fp32"): 167.92e9, ("mwa4096", "fp32"): 19.07e9}


def edges_of(W):
    nb = W["nbins"]
    return (W["lmin"] / (2 * np.pi)) * ((W["lmax"] / W["lmin"]) ** (np.arange(nb + 1) / nb))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS) + ["serve", "copy", "sim4096"])
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: admission budget")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the workload itself (no precision-form, 1024^2 or serving keys)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def _cores():
    try:
        from threadpoolctl import threadpool_info
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        blas = 1
    try:
        fft = len(os.sched_getaffinity(0))
    except Exception:
        fft = os.cpu_count() or 1
    return blas, fft


def cpu_baseline_full(n, edges, trips, uv, vis, norm, budget_s):
    """The FP64 oracle as it stands (gridding + estimator) on whole realisations."""
    from oracle import estimator as oest
    from oracle import gridding as ogrid
    blas, fft = _cores()
    done, t0 = 0, time.perf_counter()
    while True:
        g, w, _ = ogrid.grid_visibilities(n, 1.0, uv, vis[done % len(vis)])
        oest.estimate(g, w, edges, norm, wmode=oest.INV_COUNT, trips=trips)
        done += 1
        if time.perf_counter() - t0 >= budget_s or done >= 16:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "grids/s", "cores": int(max(blas, fft)), "kind": "oracle",
            "sample": "%d whole realisation(s): FP64 gridding of %d visibilities + estimator "
                      "(scipy FFT on %d threads, BLAS on %d threads), %.1f s" % (done, len(uv), fft, blas, dt)}


def cpu_baseline_sampled(n, edges, trips, uv, vis0, norm):
    """The FP64 oracle as it stands, timed on bounded samples of one realisation and
    scaled to one whole grid (a whole 8192^2 realisation takes the oracle minutes):
      gridding   grid_visibilities on 2^21 of the visibilities, minus its cost with none,
                 scaled by nvis / 2^21, plus that fixed cost;
      fields     the Hermitian parts of W V and W, and ring_fields (FP64 FFT) of 2 rings
                 (after one untimed call at the same size), scaled to the 2 x nbins data and
                 weight fields;
      sums       triple_sums (chunked FP64 GEMM) of all plan triplets over a slab of 128
                 rows of fields, scaled by n / 128, twice (numerator and denominator)."""
    from oracle import estimator as oest
    from oracle import gridding as ogrid
    from oracle import plan as oplan
    blas, fft = _cores()
    nb = len(edges) - 1
    nvis = len(uv)
    S = min(nvis, 1 << 21)
    T0 = time.perf_counter()
    t = time.perf_counter()
    ogrid.grid_visibilities(n, 1.0, uv[:0], vis0[:0])
    t_fix = time.perf_counter() - t
    t = time.perf_counter()
    g, w, _ = ogrid.grid_visibilities(n, 1.0, uv[:S], vis0[:S])
    t_s = time.perf_counter() - t
    t_grid = t_fix + max(t_s - t_fix, 0.0) * nvis / S
    t = time.perf_counter()
    W = oest.effective_weights(n, w, oest.INV_COUNT)
    X = oest.hermitian_part(W * g)
    Y = oest.hermitian_part(W.astype(np.complex128))
    t_herm = time.perf_counter() - t
    del Y, g, w
    rc = oplan.ring_of_cell(n, edges)
    k = 2
    ms = np.stack([rc == m for m in (0, nb - 1)][:k])
    oest.ring_fields(X, ms[:1])          # untimed: FFT plan and thread start-up at this size
    t = time.perf_counter()
    F = oest.ring_fields(X, ms)
    t_ring = (time.perf_counter() - t) / k
    del X, ms, rc
    R = 128
    slab = np.ascontiguousarray(np.concatenate([F[:, :R, :]] * ((nb + k - 1) // k))[:nb])
    del F
    t = time.perf_counter()
    oest.triple_sums(slab, trips)
    t_sum = time.perf_counter() - t
    t_total = t_grid + t_herm + t_ring * 2 * nb + 2 * t_sum * (n / R)
    return {"value": 1.0 / t_total, "unit": "grids/s", "cores": int(max(blas, fft)), "kind": "oracle",
            "sample": "one realisation in bounded pieces, %.1f s of CPU work, scaled to a whole grid "
                      "(%.0f s): gridding of %d of %d visibilities (%.2f s, scaled %.1f s); Hermitian parts "
                      "%.2f s; FP64 FFT of %d ring fields %.2f s each, x %d fields; FP64 GEMM triple sums of "
                      "all %d triplets over %d of %d rows %.2f s, x %d x 2; scipy FFT on %d threads, BLAS on "
                      "%d threads" % (time.perf_counter() - T0, t_total, S, nvis, t_s, t_grid, t_herm, k,
                                      t_ring, 2 * nb, len(trips), R, n, t_sum, n // R, fft, blas)}


def sim_bench(a):
    """Visibility simulation (Eq. 4 through the Eq. 5 beam) at the paper's geometry: 4096^2
    skies of 0.029 deg pixels, 2^20 baselines with density ~ exp(-U / 62.5) inside U = 250
    wavelengths, 4 skies a step.  Reports visibilities/s, and the HBM fraction of the
    transform (its algorithmic bytes: the row transforms write N x M complex values, the
    transpose reads and writes them, the column transforms read them and write M^2; 8 bytes
    a value) from HIP events around the whole call."""
    import torch

    import paper_2412_02246_amd as A
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    nsky, dth, nvis, batch = 4096, np.deg2rad(0.029), 1 << 20, a.batch or 4
    d_lam = 4.0 * 154.25e6 / 299792458.0
    gen = torch.Generator(device=dev)
    gen.manual_seed(20241202)
    sky = torch.randn((batch, nsky, nsky), dtype=torch.float32, device=dev, generator=gen)
    r = -62.5 * torch.log1p(-torch.rand(nvis, dtype=torch.float64, device=dev, generator=gen) *
                            (1 - np.exp(-250.0 / 62.5)))
    ph = 2 * np.pi * torch.rand(nvis, dtype=torch.float64, device=dev, generator=gen)
    uv = torch.stack([r * torch.cos(ph), r * torch.sin(ph)], dim=1).contiguous()
    for _ in range(a.warmup):
        A.simulate(sky, dth, uv, beam=A.BEAM_MWA, beam_param=d_lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        V = A.simulate(sky, dth, uv, beam=A.BEAM_MWA, beam_param=d_lam)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    m = 2 * nsky
    fft_bytes = 8.0 * (nsky * m + 2 * nsky * m + nsky * m + m * m) * batch
    out = {"metric": "simulated visibilities/s at 1 GPU (Eq. 4, MWA beam, non-uniform FFT)",
           "value": nvis * batch / dt, "unit": "visibilities/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "4096^2 skies of 0.029 deg pixels, MWA tile beam, 2^20 baselines within U = 250, "
                                  "%d skies a step" % batch, "skies_per_s": batch / dt,
                      "transform_alg_bytes": fft_bytes,
                      "transform_bytes_over_call_frac_hbm": fft_bytes / dt / 8.0e12}}
    del V
    print(json.dumps(out), flush=True)


def copy_probe(a):
    """A plain device copy of a known size (1 GiB read + 1 GiB written per launch), run
    under the same rocprofv3 counters as the kernels to calibrate FETCH_SIZE and
    WRITE_SIZE against bytes actually moved; also the copy's achieved HBM rate, the
    practical ceiling next to the 8 TB/s datasheet figure."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.warmup):
        dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(a.steps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    nbytes = 2 * src.numel() * 4
    print(json.dumps({"copy_probe_bytes_per_launch": nbytes, "launches": a.warmup + a.steps,
                      "copy_gb_per_s": nbytes * a.steps / (t0.elapsed_time(t1) * 1e-3) / 1e9}),
          flush=True)


def serve_specs(nreq, seed=4242, channels=16):
    """The serving stream: `channels` channels, each a grid size uniform over
    {512, 1024, 2048, 4096}^2 with 16..32 log rings (46 <= l < 1320, radii scaled by n/1024)
    and its own baseline counts; half the requests are realisations of one of them (the
    channel's plan and weights, so its triangle counts are computed once and batches can
    form), half are channels of their own (grid size, rings and weights drawn afresh).
    Returns [(n, edges, channel or None)] and the generator."""
    rng = np.random.default_rng(seed)

    def draw():
        n = int(rng.choice([512, 1024, 2048, 4096]))
        nb = int(rng.integers(16, 33))
        s = n / 1024.0
        return n, tuple((46.0 * s / (2 * np.pi)) * (1320.0 / 46.0) ** (np.arange(nb + 1) / nb))

    chans = [draw() for _ in range(channels)]
    specs = []
    for _ in range(nreq):
        if rng.random() < 0.5:
            c = int(rng.integers(channels))
            specs.append(chans[c] + (c,))
        else:
            specs.append(draw() + (None,))
    return specs, rng


def serve_run(precision, nreq, budget_gib, compiled=None, log=sys.stderr):
    """Serving form: a Poisson stream of requests, each one channel or one realisation.
    The saturated rate mu is measured first (all requests at t = 0), then streams at
    rho mu, rho in {0.5, 0.8, 0.95}, report p50/p99 latency, grids/s and the mean batch."""
    import torch

    import paper_2412_02246_amd as A
    from paper_2412_02246_amd.serve import GpuExecutor, Request, Scheduler, latency_stats, run_stream

    specs, rng = serve_specs(nreq)
    prec = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[precision]
    slots, max_batch = 4, 8
    keys = list(dict.fromkeys((n, e) for n, e, _ in specs))
    kw = dict(wmode=A.W_INV_COUNT, precision=prec, max_batch=max_batch)
    if compiled is None:
        from paper_2412_02246_amd.jit import compile_parts
        t0 = time.perf_counter()
        plans = [A.Plan(n, e, **kw) for n, e in keys]
        compile_parts(plans, [(n, e, kw) for n, e in keys], workers=16)
        print("serve: %d plans compiled in %.1f s" % (len(plans), time.perf_counter() - t0), file=log, flush=True)
    else:
        plans = compiled
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    ex = GpuExecutor(A.W_INV_COUNT, precision=prec, max_batch=max_batch, slots=slots)
    for k, p in zip(keys, plans):
        ex.plans[k] = p.bind(0)
    # device-resident inputs: 4 grids and 4 per-request count masks per size, one count
    # mask per channel
    gen = torch.Generator(device=dev)
    gen.manual_seed(4242)
    pool, own, lams = {}, {}, {}
    for n in (512, 1024, 2048, 4096):
        g = torch.arange(n, device=dev)
        g = torch.where(g < n // 2, g, g - n).double()
        r = torch.sqrt(g[:, None] ** 2 + g[None, :] ** 2)
        lams[n] = 4.0 * torch.exp(-r / (n / 8.0))
        pool[n] = [torch.randn((n, n), dtype=torch.complex64, device=dev, generator=gen) for _ in range(4)]
        own[n] = [torch.poisson(lams[n], generator=gen).float() for _ in range(4)]
    chan = {}
    for n, e, c in specs:
        if c is not None and c not in chan:
            chan[c] = torch.poisson(lams[n], generator=gen).float()
    torch.cuda.synchronize()

    def requests(arrivals):
        out = []
        for k, ((n, e, c), t) in enumerate(zip(specs, arrivals)):
            grid = pool[n][k % 4]
            if c is not None:
                out.append(Request(k, n, e, grid, chan[c], ("chan", c), t))
            else:
                out.append(Request(k, n, e, grid, own[n][k % 4], None, t))
        return out

    budget = int(budget_gib * (1 << 30))
    # warm-up pass (first launches, cached counts), then the saturated rate
    run_stream(Scheduler(ex, budget, max_batch, slots), requests(np.zeros(len(specs)))[:32])
    torch.cuda.synchronize()
    sat = latency_stats(run_stream(Scheduler(ex, budget, max_batch, slots), requests(np.zeros(len(specs)))))
    mu = sat["grids_per_s"]
    print("serve %s: saturated %.1f grids/s" % (precision, mu), file=log, flush=True)
    loads = {}
    for rho in (0.5, 0.8, 0.95):
        arr = np.cumsum(rng.exponential(1.0 / (rho * mu), len(specs)))
        sch = Scheduler(ex, budget, max_batch, slots)
        st = latency_stats(run_stream(sch, requests(arr)))
        st["peak_budget_gib"] = sch.peak_used / (1 << 30)
        st["rejected"] = len(sch.rejected)
        loads["rho=%.2f" % rho] = st
        print("serve %s: rho %.2f -> %s" % (precision, rho, st), file=log, flush=True)
    for p in plans:
        p.close()
    del ex
    torch.cuda.empty_cache()
    return {"saturated": sat, "poisson": loads, "slots": slots, "max_batch": max_batch,
            "requests": len(specs), "plans": len(keys)}


def serve_child(precision, nreq, budget_gib):
    """Run the serving bench (--workload serve) as a child process and return its
    measurements; its progress lines are passed on to stderr."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "serve", "--precision", precision,
           "--requests", str(nreq), "--budget-gib", str(budget_gib)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    sys.stderr.write(r.stderr)
    sys.stderr.flush()
    if r.returncode != 0:
        raise RuntimeError("serving bench failed (%d)" % r.returncode)
    line = json.loads(r.stdout.strip().splitlines()[-1])
    res = dict(line["config"])
    res.pop("workload", None)
    res["saturated_grids_per_s"] = line["value"]
    return res


def serve_bench(a):
    out = serve_run(a.precision, a.requests, a.budget_gib)
    mu = out["saturated"]["grids_per_s"]
    line = {
        "metric": "bispectrum grids/s at 1 GPU (serving, continuous batching)",
        "value": mu, "unit": "grids/s", "n_gpus": 1, "steps": a.requests, "warmup": 32,
        "ms_per_step": 1e3 / mu, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3 (f32 acc)", "fp16x3": "fp16x3 (f32 acc)"}[a.precision],
        "data": "synthetic",
        "config": {"workload": "serving: %d requests, n in {512,1024,2048,4096}, 16-32 log rings; 50%% "
                               "realisations of 16 channels (their plan and counts), 50%% channels of their "
                               "own; budget %.0f GiB" % (a.requests, a.budget_gib), **out},
    }
    print(json.dumps(line), flush=True)


def presort(plan, uv_d, vis_d, log=sys.stderr):
    """Sort the workload's baseline set once and put its visibilities into slot order (the
    realisations share the baselines); returns (BaselineSet, visibility records in slot order,
    timings of the two one-off calls and of the general gridding call on the same input)."""
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    bset = plan.grid_sort(uv_d)
    sort_ms = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    vs = bset.permute(vis_d)
    torch.cuda.synchronize()
    perm_ms = 1e3 * (time.perf_counter() - t)
    plan.grid(uv_d, vis_d)           # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        plan.grid(uv_d, vis_d)
    torch.cuda.synchronize()
    gen_ms = 1e3 * (time.perf_counter() - t) / 3
    plan._work = None
    torch.cuda.empty_cache()
    info = {"sort_ms": sort_ms, "permute_ms": perm_ms, "unsorted_gridding_ms": gen_ms, "kept": bset.kept}
    print("bench: baseline set sorted in %.1f ms, visibilities permuted in %.1f ms (general gridding %.2f ms)"
          % (sort_ms, perm_ms, gen_ms), file=log, flush=True)
    return bset, vs, info


def measure(name, precision, plan, bset, vs, steps, warmup, log=sys.stderr, cached_counts=False):
    """Time `steps` gridding + estimator steps of one workload after `warmup` untimed ones:
    the batch's visibilities (in the slot order of the sorted baseline set `bset`) gridded,
    then the estimator with the set's counts as weights.  The contraction's launches are
    bracketed by HIP events on every timed step, and a few extra steps carry events around
    the gridding, column-pass and row-pass stages."""
    import torch

    import paper_2412_02246_amd as A
    W = WORKLOADS[name]
    n, nb = W["n"], W["nbins"]
    C = plan.nchan
    batch = vs.shape[1] // C      # grids (multi-frequency grids of C channel grids each)
    nvis = bset.kept

    # cached_counts: the triangle counts N_t depend on the weights alone, which the baseline
    # set fixes; abs_counts gives them once and every step then skips the weight fields
    nt = plan.counts(bset.wsum) if cached_counts else None

    def step():
        g = plan.grid_sorted(bset, vs)
        return plan.estimate(g, bset.wsum, n_given=nt)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    L = A._lib
    ev = HipEvents(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        L.lib().abs_profile(plan.handle, L.STAGE_CONTRACT, *ev.pair(k))
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.lib().abs_profile(plan.handle, L.STAGE_CONTRACT, None, None)
    con_ms = float(np.mean([ev.elapsed_ms(k) for k in range(steps)]))
    ev.close()
    ms = 1e3 * dt / steps
    grids_s = batch * steps / dt
    print("bench: %s %s%s %.3f ms/step, %.2f grids/s, contraction %.3f ms"
          % (name, precision, " (cached N_t)" if cached_counts else "", ms, grids_s, con_ms), file=log, flush=True)
    if cached_counts:
        return {"grids_per_s": grids_s, "ms_per_step": ms, "contraction_ms": con_ms}
    nsets = batch   # the contraction launches timed are the data-set ones (the weight set runs in FP64)
    # algorithmic flops per pixel: two per triplet (product with the pair, add) plus the
    # pair products, counted for the orientation with the fewest distinct pairs ((i, j) or
    # (j, k) of i <= j <= k); each resolution level sums its triplets over its own m^2
    # pixels (the least work that level's sum needs), so the launch's flops are the sum
    # over levels; "flops_per_launch_at_n" counts every triplet over n^2 pixels instead
    def level_flops(ijk, npix):
        pairs = min(len({(int(x[0]), int(x[1])) for x in ijk}), len({(int(x[1]), int(x[2])) for x in ijk}))
        return float(nsets) * npix * (pairs + 2 * len(ijk))
    ijk_all = np.asarray(plan.triplets).reshape(-1, 3)
    flops = sum(level_flops(ijk_all[lv["tmap"]], lv["m"] ** 2) for lv in plan.levels)
    flops_n = level_flops(ijk_all, n * n)
    achieved = flops / (con_ms * 1e-3)
    traffic = MEASURED_TRAFFIC.get((name, precision)) if batch == W["batch"] else None
    if precision == "fp32":
        roof = {"kernel": "abs_contract (plan-specialised FP32 triplet contraction)", "bound": "alu",
                "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic, "avg_ms": con_ms,
                "flops_per_launch": flops, "flops_per_launch_at_n": flops_n,
                "levels": [[lv["m"], lv["ntrip"]] for lv in plan.levels],
                "peak_nonpacked_valu": PEAK_VALU_NONPACKED / 1e12,
                "frac_nonpacked_valu": achieved / PEAK_VALU_NONPACKED}
    else:
        # 3 split MFMAs per 16 x 16 tile and pixel, each level's tiles over its m^2 pixels,
        # for the levels the plan runs on the matrix units (the others take the FP32 kernel,
        # which has code parts of its own)
        mf = [lv for lv in plan.levels if lv["contract"][0] == 0]
        issued = float(nsets) * sum(lv["mfma_tiles"] * lv["m"] ** 2 for lv in mf) * 3 * 512
        roof = {"kernel": "mfma_contract_kernel (%s triplet contraction; levels %s on the matrix units, the rest "
                          "in the FP32 kernel)" % (precision, [lv["m"] for lv in mf]), "bound": "mfma",
                "achieved": achieved / 1e12, "peak": PEAK_MFMA_16BIT / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_MFMA_16BIT, "traffic": traffic, "avg_ms": con_ms,
                "flops_per_launch": flops, "flops_per_launch_at_n": flops_n,
                "levels": [[lv["m"], lv["ntrip"]] for lv in plan.levels],
                "mfma_issued_tflops": issued / (con_ms * 1e-3) / 1e12,
                "mfma_issued_frac": issued / (con_ms * 1e-3) / PEAK_MFMA_16BIT}
    # HBM fraction of the gridding and FFT stages, from HIP events the library records
    # around each stage on a few extra (untimed) steps; algorithmic bytes per step:
    #   gridding: values read (8 B a visibility and realisation), grids written (8 B a cell
    #             and realisation); the baselines and counts belong to the sorted set
    #   column pass: the pruned intermediate written (8 B x m x ncols a set and level)
    #   row pass: that intermediate read and the FP32 fields written (4 B x nbins x m^2 a set and level)
    stages = {}
    nprof = 3
    evs = {st: HipEvents(nprof) for st in (L.STAGE_GRID, L.STAGE_COLPASS, L.STAGE_ROWPASS)}
    for k in range(nprof):
        for st, e in evs.items():
            L.lib().abs_profile(plan.handle, st, *e.pair(k))
        step()
    torch.cuda.synchronize()
    # column pass and row pass of every resolution level (m, its rings and columns)
    zbytes = sum(8.0 * lv["m"] * lv["ncols"] for lv in plan.levels) * batch * C
    fbytes = sum(4.0 * lv["nbins"] * lv["m"] ** 2 for lv in plan.levels) * batch * C
    alg = {L.STAGE_GRID: batch * C * (8.0 * nvis + 8.0 * n * n),
           L.STAGE_COLPASS: zbytes,
           L.STAGE_ROWPASS: zbytes + fbytes}
    tot_b = tot_ms = 0.0
    for st, sname in ((L.STAGE_GRID, "gridding"), (L.STAGE_COLPASS, "column_pass"), (L.STAGE_ROWPASS, "row_pass")):
        L.lib().abs_profile(plan.handle, st, None, None)
        st_ms = float(np.mean([evs[st].elapsed_ms(k) for k in range(nprof)]))
        evs[st].close()
        stages[sname] = {"ms": st_ms, "alg_bytes": alg[st], "gb_per_s": alg[st] / (st_ms * 1e-3) / 1e9,
                         "frac_hbm": alg[st] / (st_ms * 1e-3) / PEAK_HBM}
        tot_b += alg[st]
        tot_ms += st_ms
    stages["gridding_and_fft"] = {"ms": tot_ms, "alg_bytes": tot_b, "gb_per_s": tot_b / (tot_ms * 1e-3) / 1e9,
                                  "frac_hbm": tot_b / (tot_ms * 1e-3) / PEAK_HBM}
    return {"grids_per_s": grids_s, "ms_per_step": ms, "grids_per_step": batch,
            "bin_triplets_per_s": grids_s * plan.ntrip, "roofline": roof, "stages_hbm": stages}


def _dtype(precision):
    return {"fp32": "f32", "bf16x3": "bf16x3 (f32 acc)", "fp16x3": "fp16x3 (f32 acc)"}[precision]


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: measures one GPU only (--gpus 1); %d GPUs is not supported"
              % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.workload == "serve":
        return serve_bench(a)
    if a.workload == "copy":
        return copy_probe(a)
    if a.workload == "sim4096":
        return sim_bench(a)
    import torch

    import paper_2412_02246_amd as A
    import synth
    from paper_2412_02246_amd.jit import compile_parts

    P = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}
    name = a.workload
    W = WORKLOADS[name]
    n, nb, batch = W["n"], W["nbins"], (a.batch or W["batch"])
    edges = edges_of(W)
    nvis = n * n
    extras = not a.no_extras and name == DEFAULT_WORKLOAD and not a.batch
    print("bench: workload %s n=%d rings=%d batch=%d nvis=%d precision %s" % (name, n, nb, batch, nvis, a.precision),
          file=sys.stderr, flush=True)
    # every plan's contraction code is compiled in worker processes before this process
    # touches the GPU
    jobs = [(name, a.precision, batch)]
    if extras:
        jobs += [(name, "bf16x3", batch), (name, "fp16x3", batch), ("mwa1024", "fp32", WORKLOADS["mwa1024"]["batch"])]
    t0 = time.perf_counter()
    plans, specs = [], []
    for wname, prec, b in jobs:
        Wj = WORKLOADS[wname]
        kw = dict(wmode=A.W_INV_COUNT, max_batch=b, precision=P[prec], nchan=Wj.get("nchan", 1))
        plans.append(A.Plan(Wj["n"], edges_of(Wj), **kw))
        specs.append((Wj["n"], tuple(edges_of(Wj)), kw))
    compile_parts(plans, specs, workers=16)
    print("bench: %d plans (%d code parts) compiled in %.1f s" %
          (len(plans), sum(p.jit_parts for p in plans), time.perf_counter() - t0), file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    def inputs(wname, b):
        Wj = WORKLOADS[wname]
        t = time.perf_counter()
        uv_d, vis_d = synth.mwa_visibilities_device(Wj["n"], Wj["n"] ** 2, edges_of(Wj)[-1],
                                                    synth.seed_for(Wj["cfg"], 0), batch=b, device=dev)
        torch.cuda.synchronize()
        print("bench: %s inputs drawn on the device in %.1f s" % (wname, time.perf_counter() - t),
              file=sys.stderr, flush=True)
        return uv_d, vis_d

    uv_d, vis_d = inputs(name, batch * W.get("nchan", 1))
    main_plan = plans[0].bind()
    bset, vs, sinfo = presort(main_plan, uv_d, vis_d)
    res = measure(name, a.precision, main_plan, bset, vs, a.steps, a.warmup)
    # the same steps with N_t computed once for the baseline set's counts
    rcached = measure(name, a.precision, main_plan, bset, vs, a.steps, a.warmup, cached_counts=True) \
        if extras else None
    ntrip = int(main_plan.ntrip)
    main_plan.close()
    main_plan._work = None
    torch.cuda.empty_cache()
    out = {
        "metric": "bispectrum grids/s at 1 GPU (gridding + estimator)",
        "value": res["grids_per_s"], "unit": "grids/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": _dtype(a.precision), "data": "synthetic",
        "config": {"workload": W["desc"], "n": n, "nbins": nb, "grids_per_step": batch,
                   "nvis_per_grid": nvis, "ntrip": ntrip, "precision": a.precision,
                   "bin_triplets_per_s": res["bin_triplets_per_s"], "parallelism": "1 GPU"},
        "roofline": res["roofline"],
        "stages_hbm": res["stages_hbm"],
        "baseline_set": sinfo,
    }
    if extras:
        out["cached_counts"] = rcached
        for k, prec in ((1, "bf16x3"), (2, "fp16x3")):
            pk = plans[k].bind()
            rk = measure(name, prec, pk, bset, vs, a.steps, a.warmup)
            pk.close()
            pk._work = None
            torch.cuda.empty_cache()
            rk["speedup_vs_fp32"] = rk["grids_per_s"] / res["grids_per_s"]
            out["precision_form_" + prec] = rk
    uv_h = vis_h = None
    if not a.no_cpu:
        uv_h = uv_d.cpu().numpy()
        vis_h = vis_d[:1].cpu().numpy()
    del uv_d, vis_d, bset, vs
    torch.cuda.empty_cache()
    if extras:
        uv1, vis1 = inputs("mwa1024", WORKLOADS["mwa1024"]["batch"])
        p1 = plans[3].bind()
        b1, vs1, s1 = presort(p1, uv1, vis1)
        r1 = measure("mwa1024", "fp32", p1, b1, vs1, a.steps, a.warmup)
        r1["workload"] = WORKLOADS["mwa1024"]["desc"]
        r1["baseline_set"] = s1
        p1.close()
        del uv1, vis1, b1, vs1
        torch.cuda.empty_cache()
        out["mwa1024_fp32"] = r1
        # the serving form in a process of its own (as a server would run), one per precision
        out["serving"] = {prec: serve_child(prec, a.requests, a.budget_gib) for prec in ("fp32", "bf16x3", "fp16x3")}
    if not a.no_cpu:
        from oracle import plan as oplan   # noqa: F401  (oracle import only for the baseline)
        trips = A.Plan(n, edges).triplets
        if n <= 2048:
            out["cpu_baseline"] = cpu_baseline_full(n, edges, trips, uv_h, vis_h, out_norm(A, n, edges),
                                                    a.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline_sampled(n, edges, trips, uv_h, vis_h[0], out_norm(A, n, edges))
    print(json.dumps(out), flush=True)


def out_norm(A, n, edges):
    return A.Plan(n, edges).norm


if __name__ == "__main__":
    main()
