"""Throughput of the bispectrum hot path on one MI355X.

One step = gridding of nvis = n^2 visibilities for a batch of realisations of one
MWA-shaped channel (shared baselines, Eq. 9) followed by the estimator of Eq. (12)
for the batch (ring FFTs, triplet contraction, normalisation), with the gridded
counts as shared INV_COUNT weights.  Inputs are resident in HBM before timing.

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
                    desc="MWA-shaped single channel: 1024x1024 c64 grid, 20 log rings 46<=l<1320, "
                         "Poisson baseline mask + SNR-5 noise, INV_COUNT weights"),
    # precision-form shapes: 4096^2, 32 log rings, edges x4
    "mwa4096": dict(n=4096, nbins=32, lmin=4 * 46.0, lmax=4 * 1320.0, batch=16, cfg=2,
                    desc="MWA-shaped 4096x4096 c64 grid, 32 log rings 4x(46<=l<1320), INV_COUNT weights"),
    # large ensemble shapes: 8192^2, 64 log rings, edges x8 (realisations in batches of 4)
    "mwa8192": dict(n=8192, nbins=64, lmin=8 * 46.0, lmax=8 * 1320.0, batch=4, cfg=4,
                    desc="MWA-shaped 8192x8192 c64 grid, 64 log rings 8x(46<=l<1320), INV_COUNT weights"),
}
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


PEAK_VALU_FP32 = 78.6e12   # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, no packed FP32
PEAK_MFMA_16BIT = 2.5e15   # dense BF16 / FP16 matrix peak
PEAK_HBM = 8.0e12

# HBM bytes per launch of the timed contraction kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by a 1 GiB copy (2.0 x FETCH_SIZE + 1.0 x WRITE_SIZE), for the
# kernel as it stands in this tree (profiles/counters_mwa1024_batch16.md); a workload or
# precision without an entry reports null.
MEASURED_TRAFFIC = {("mwa1024", "fp32"): 1348.6e6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mwa1024", choices=sorted(WORKLOADS) + ["serve", "copy"])
    ap.add_argument("--requests", type=int, default=512, help="serve: number of requests")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve: admission budget")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def cpu_baseline(n, edges, trips, uv, vis, norm, budget_s):
    """The FP64 oracle as it stands (gridding + estimator) on a bounded sample."""
    from oracle import estimator as oest
    from oracle import gridding as ogrid
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = 1
    done, t0 = 0, time.perf_counter()
    while True:
        g, w, _ = ogrid.grid_visibilities(n, 1.0, uv, vis[done % len(vis)])
        oest.estimate(g, w, edges, norm, wmode=oest.INV_COUNT, trips=trips)
        done += 1
        if time.perf_counter() - t0 >= budget_s or done >= 16:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "grids/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d realisation(s): FP64 gridding of %d visibilities + estimator "
                      "(numpy FFT, BLAS %d threads), %.1f s" % (done, len(uv), cores, dt)}


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


def serve_bench(a):
    """Serving form: a Poisson stream of requests, each one channel or one realisation,
    grid sizes uniform over {512, 1024, 2048, 4096}^2 complex64 with 16..32 log rings
    (46 <= l < 1320, radii scaled by n/1024); half the requests are realisations sharing
    their channel's weights (cached triangle counts), half channels with their own.
    The saturated rate mu is measured first (all requests at t = 0), then streams at
    rho mu, rho in {0.5, 0.8, 0.95}, report p50/p99 latency and grids/s."""
    import torch

    import paper_2412_02246_amd as A
    from paper_2412_02246_amd.serve import GpuExecutor, Request, Scheduler, latency_stats, run_stream

    rng = np.random.default_rng(4242)
    sizes = [512, 1024, 2048, 4096]
    specs = []
    for k in range(a.requests):
        n = int(rng.choice(sizes))
        nb = int(rng.integers(16, 33))
        s = n / 1024.0
        edges = tuple((46.0 * s / (2 * np.pi)) * (1320.0 / 46.0) ** (np.arange(nb + 1) / nb))
        specs.append((n, edges, bool(rng.random() < 0.5)))
    prec = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[a.precision]
    slots, max_batch = 4, 8
    # compile every plan in worker processes before the GPU is touched
    from paper_2412_02246_amd.jit import compile_parts
    keys = list(dict.fromkeys((n, e) for n, e, _ in specs))
    kw = dict(wmode=A.W_INV_COUNT, precision=prec, max_batch=max_batch)
    t0 = time.perf_counter()
    plans = [A.Plan(n, e, **kw) for n, e in keys]
    compile_parts(plans, [(n, e, kw) for n, e in keys], workers=16)
    print("serve: %d plans compiled in %.1f s" % (len(plans), time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    ex = GpuExecutor(A.W_INV_COUNT, precision=prec, max_batch=max_batch, slots=slots)
    for k, p in zip(keys, plans):
        ex.plans[k] = p.bind(0)
    # device-resident inputs: 4 grids per size, one shared (channel) mask per size and 4
    # per-request masks per size
    gen = torch.Generator(device=dev)
    gen.manual_seed(4242)
    pool, chan, own = {}, {}, {}
    for n in sizes:
        g = torch.arange(n, device=dev)
        g = torch.where(g < n // 2, g, g - n).double()
        r = torch.sqrt(g[:, None] ** 2 + g[None, :] ** 2)
        lam = 4.0 * torch.exp(-r / (n / 8.0))
        pool[n] = [torch.randn((n, n), dtype=torch.complex64, device=dev, generator=gen) for _ in range(4)]
        chan[n] = torch.poisson(lam, generator=gen).float()
        own[n] = [torch.poisson(lam, generator=gen).float() for _ in range(4)]
    torch.cuda.synchronize()

    def requests(arrivals):
        out = []
        for k, ((n, e, shared), t) in enumerate(zip(specs, arrivals)):
            grid = pool[n][k % 4]
            if shared:
                out.append(Request(k, n, e, grid, chan[n], ("chan", n), t))
            else:
                out.append(Request(k, n, e, grid, own[n][k % 4], None, t))
        return out

    budget = int(a.budget_gib * (1 << 30))
    # warm-up pass (first launches, cached counts), then the saturated rate
    run_stream(Scheduler(ex, budget, max_batch, slots), requests(np.zeros(len(specs)))[:32])
    torch.cuda.synchronize()
    sat = latency_stats(run_stream(Scheduler(ex, budget, max_batch, slots),
                                   requests(np.zeros(len(specs)))))
    mu = sat["grids_per_s"]
    print("serve: saturated %.1f grids/s" % mu, file=sys.stderr, flush=True)
    loads = {}
    for rho in (0.5, 0.8, 0.95):
        arr = np.cumsum(rng.exponential(1.0 / (rho * mu), len(specs)))
        sch = Scheduler(ex, budget, max_batch, slots)
        st = latency_stats(run_stream(sch, requests(arr)))
        st["peak_budget_gib"] = sch.peak_used / (1 << 30)
        st["rejected"] = len(sch.rejected)
        loads["rho=%.2f" % rho] = st
        print("serve: rho %.2f -> %s" % (rho, st), file=sys.stderr, flush=True)
    out = {
        "metric": "bispectrum grids/s at 1 GPU (serving, continuous batching)",
        "value": mu, "unit": "grids/s", "n_gpus": 1, "steps": len(specs), "warmup": 32,
        "ms_per_step": 1e3 / mu, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3 (f32 acc)", "fp16x3": "fp16x3 (f32 acc)"}[a.precision],
        "data": "synthetic",
        "config": {"workload": "serving: %d requests, n in {512,1024,2048,4096}, 16-32 log rings, "
                               "50%% shared-mask realisations / 50%% channels, budget %.0f GiB"
                               % (len(specs), a.budget_gib),
                   "slots": slots, "max_batch": max_batch, "saturated": sat, "poisson": loads},
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); %d GPUs is not supported"
              % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.workload == "serve":
        return serve_bench(a)
    if a.workload == "copy":
        return copy_probe(a)
    import torch

    import paper_2412_02246_amd as A
    import synth

    W = WORKLOADS[a.workload]
    n, nb, batch = W["n"], W["nbins"], (a.batch or W["batch"])
    edges = (W["lmin"] / (2 * np.pi)) * ((W["lmax"] / W["lmin"]) ** (np.arange(nb + 1) / nb))
    nvis = n * n
    print("bench: workload %s n=%d rings=%d batch=%d nvis=%d" % (a.workload, n, nb, batch, nvis),
          file=sys.stderr, flush=True)
    prec = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[a.precision]
    # the plan's contraction code is compiled in worker processes before this process
    # touches the GPU
    t0 = time.perf_counter()
    plan = A.Plan(n, edges, wmode=A.W_INV_COUNT, max_batch=batch, precision=prec)
    plan.compile(workers=16)
    print("bench: plan ntrip=%d npairs=%d, %d code parts compiled in %.1f s" %
          (plan.ntrip, plan.npairs, plan.jit_parts, time.perf_counter() - t0), file=sys.stderr, flush=True)
    uv, vis = synth.mwa_visibilities(n, nvis, edges[-1], synth.seed_for(W["cfg"], 0), batch=batch)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    plan.bind()
    print("bench: inputs generated", file=sys.stderr, flush=True)
    uv_d = torch.from_numpy(uv).to(dev)
    vis_d = torch.from_numpy(vis).to(dev)

    def step():
        g, w, _ = plan.grid(uv_d, vis_d)
        return plan.estimate(g, w)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    L = A._lib
    ev = HipEvents(a.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        L.lib().abs_profile(plan.handle, L.STAGE_CONTRACT, *ev.pair(k))
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.lib().abs_profile(plan.handle, L.STAGE_CONTRACT, None, None)
    con_ms = float(np.mean([ev.elapsed_ms(k) for k in range(a.steps)]))
    ev.close()
    ms = 1e3 * dt / a.steps
    grids_s = batch * a.steps / dt
    nsets = batch  # the contraction launch timed is the data-set one (the weight set runs in FP64)
    # algorithmic flops per pixel: two per triplet (product with the pair, add) plus the
    # pair products, counted for the orientation with the fewest distinct pairs ((i, j) or
    # (j, k) of i <= j <= k)
    ijk = np.asarray(plan.triplets).reshape(-1, 3)
    pairs = min(len({(int(x[0]), int(x[1])) for x in ijk}), len({(int(x[1]), int(x[2])) for x in ijk}))
    flops = float(nsets) * n * n * (pairs + 2 * plan.ntrip)
    achieved = flops / (con_ms * 1e-3)
    if a.precision == "fp32":
        roof = {"kernel": "abs_contract (plan-specialised FP32 triplet contraction)", "bound": "alu",
                "achieved": achieved / 1e12, "peak": PEAK_VALU_FP32 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_VALU_FP32, "avg_ms": con_ms,
                "traffic": MEASURED_TRAFFIC.get((a.workload, a.precision)) if batch == W["batch"] else None,
                "flops_per_launch": flops}
    else:
        issued = float(nsets) * n * n * plan.mfma_tiles * 3 * 512   # 3 split MFMAs per tile
        roof = {"kernel": "mfma_contract_kernel (%s triplet contraction)" % a.precision, "bound": "mfma",
                "achieved": achieved / 1e12, "peak": PEAK_MFMA_16BIT / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_MFMA_16BIT, "avg_ms": con_ms,
                "traffic": MEASURED_TRAFFIC.get((a.workload, a.precision)) if batch == W["batch"] else None,
                "flops_per_launch": flops,
                "mfma_issued_tflops": issued / (con_ms * 1e-3) / 1e12,
                "mfma_issued_frac": issued / (con_ms * 1e-3) / PEAK_MFMA_16BIT}
    # HBM fraction of the gridding and FFT stages, from HIP events the library records
    # around each stage on a few extra (untimed) steps; algorithmic bytes per step:
    #   gridding: uv read once (16 B a visibility), values read (8 B a visibility and
    #             realisation), grids written (8 B a cell and realisation), counts (4 B a cell)
    #   column pass: the pruned intermediate written (8 B x n x ncols a set)
    #   row pass: that intermediate read and the FP32 fields written (4 B x nbins x n^2 a set)
    stages = {}
    nprof = 5
    evs = {st: HipEvents(nprof) for st in (L.STAGE_GRID, L.STAGE_COLPASS, L.STAGE_ROWPASS)}
    for k in range(nprof):
        for st, e in evs.items():
            L.lib().abs_profile(plan.handle, st, *e.pair(k))
        step()
    torch.cuda.synchronize()
    zbytes = 8.0 * n * plan.ncols * batch
    alg = {L.STAGE_GRID: 16.0 * nvis + batch * (8.0 * nvis + 8.0 * n * n) + 4.0 * n * n,
           L.STAGE_COLPASS: zbytes,
           L.STAGE_ROWPASS: zbytes + 4.0 * nb * n * n * batch}
    tot_b = tot_ms = 0.0
    for st, name in ((L.STAGE_GRID, "gridding"), (L.STAGE_COLPASS, "column_pass"), (L.STAGE_ROWPASS, "row_pass")):
        L.lib().abs_profile(plan.handle, st, None, None)
        st_ms = float(np.mean([evs[st].elapsed_ms(k) for k in range(nprof)]))
        evs[st].close()
        stages[name] = {"ms": st_ms, "alg_bytes": alg[st], "gb_per_s": alg[st] / (st_ms * 1e-3) / 1e9,
                        "frac_hbm": alg[st] / (st_ms * 1e-3) / PEAK_HBM}
        tot_b += alg[st]
        tot_ms += st_ms
    stages["gridding_and_fft"] = {"ms": tot_ms, "alg_bytes": tot_b, "gb_per_s": tot_b / (tot_ms * 1e-3) / 1e9,
                                  "frac_hbm": tot_b / (tot_ms * 1e-3) / PEAK_HBM}
    out = {
        "metric": "bispectrum grids/s at 1 GPU (gridding + estimator)",
        "value": grids_s, "unit": "grids/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3 (f32 acc)", "fp16x3": "fp16x3 (f32 acc)"}[a.precision],
        "data": "synthetic",
        "config": {"workload": W["desc"], "n": n, "nbins": nb, "grids_per_step": batch,
                   "nvis_per_grid": nvis, "ntrip": int(plan.ntrip), "precision": a.precision,
                   "bin_triplets_per_s": grids_s * plan.ntrip, "parallelism": "1 GPU"},
        "roofline": roof,
        "stages_hbm": stages,
    }
    if not a.no_cpu:
        e_sample = min(batch, 2)
        out["cpu_baseline"] = cpu_baseline(n, edges, plan.triplets, uv, vis[:e_sample], plan.norm,
                                           a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
