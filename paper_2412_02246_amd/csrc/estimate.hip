// abs_plan_bind, abs_estimate, abs_counts and abs_sync: the estimator of Eq. (12) of
// Gill et al. (2024) as a sequence of launches on the caller's stream:
//   column pass -> row pass (ring fields D_m and I_m, Eqs. 10-11)
//   -> triplet contraction (sum_theta of the triple products, per workgroup)
//   -> finaliser (FP64 sum over workgroups, per-triangle normalisation, B = S / (A N)).
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "abs_internal.h"

namespace abs_impl {
hipError_t launch_herm_data(const abs_plan_s* p, const void* grids, int dtype, const float* w, int w_batched,
                            int batch, void* xc, unsigned long long* wmin, hipStream_t st, int spg);
hipError_t launch_herm_weight(const abs_plan_s* p, const float* w, int w_batched, int nsets, void* xc,
                              unsigned long long* wmin, hipStream_t st, const WeightMod* mod);
hipError_t launch_colpass_f32(const abs_plan_s* p, int nsets, const void* xc, float2* Z, long long zset,
                              hipStream_t st);
hipError_t launch_colpass_f64(const abs_plan_s* p, int nsets, const void* xc, double2* Z, long long zset,
                              hipStream_t st);
hipError_t launch_rowpass_f32(const abs_plan_s* p, int nsets, const float2* Z, long long zset,
                              float* F, long long fset, unsigned* fmax_bits, hipStream_t st);
hipError_t launch_mfma_contract(const abs_plan_s* p, const float* F, long long fset, int nsets,
                                double* part, const unsigned* fmax_bits, hipStream_t st);

__global__ void fill_u32_kernel(unsigned* __restrict__ a, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long* __restrict__ a, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;   // FP64 +inf
hipError_t launch_rowpass_f64(const abs_plan_s* p, int nsets, const double2* Z, long long zset,
                              double* F, long long fset, hipStream_t st);

// Sum of nblk workgroup partials part[k * ntrip + pos[t]] of triplet t (pos: the
// triplet's position in the writing kernel's order, NULL for t itself) for the block's
// 64 triplets, in a fixed order: wave w of the kFinWaves adds its share of k in sequence,
// then the shares are added in order w = 0, 1, ...  Every thread of the block must call it.
constexpr int kFinWaves = 16, kFinBlock = 64 * kFinWaves;
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nblk, int ntrip,
                                               const int* __restrict__ pos, int t) {
  __shared__ double q[kFinWaves][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k0 = (int)((long long)nblk * wave / kFinWaves), k1 = (int)((long long)nblk * (wave + 1) / kFinWaves);
  double s = 0.0;
  if (t < ntrip) {
    const int c = pos ? pos[t] : t;
    for (int k = k0; k < k1; ++k) s += part[(long long)k * ntrip + c];
  }
  __syncthreads();   // q is reused by the next call
  q[wave][lane] = s;
  __syncthreads();
  double r = q[0][lane];
  for (int w = 1; w < kFinWaves; ++w) r += q[w][lane];
  return r;
}

// Weight-set sum over all pixels from the half-plane partials: block 0 (rows 0 and n/2,
// their own mirrors) plus twice blocks 1 .. nblk64 - 1 (rows 1 .. n/2 - 1, each standing
// for itself and its mirror row).  The factor 2 is exact.
__device__ __forceinline__ double sum_partials_half(const double* __restrict__ part64, int nblk64,
                                                    int ntrip, const int* __restrict__ pos64, int t) {
  const double rest = sum_partials(part64 + ntrip, nblk64 - 1, ntrip, pos64, t);
  const double b0 = t < ntrip ? part64[pos64 ? pos64[t] : t] : 0.0;
  return b0 + 2.0 * rest;
}

// Smallest non-zero ring-cell weight over the spw data sets of grid b (its channels, or the
// four sets of a complex grid), from the bit patterns the Hermitian-part pass recorded.
__device__ __forceinline__ double min_weight(const unsigned long long* __restrict__ wmin_bits, int b, int spw) {
  unsigned long long m = wmin_bits[(long long)b * spw];
  for (int c = 1; c < spw; ++c) m = m < wmin_bits[(long long)b * spw + c] ? m : wmin_bits[(long long)b * spw + c];
  return __longlong_as_double((long long)m);
}

// B[b][t] = S / (A N), S and N the per-triangle sums: workgroup partials are added
// in FP64 in a fixed order and divided by n^2 (the sum over pixels of a product of
// three DFTs counts every closed triangle n^2 times; m^2 for a level of size m).
// Block: 64 triplets of grid b.  A level plan's triplet t is the parent's tmap[t]: its
// cached count, B and N are at that index of rows of ntrip_out values.
// Empty triplets: with non-negative weights each closed triangle whose three cells carry
// weight adds at least w_min^3 to N_t (w_min: the smallest non-zero ring-cell weight of
// grid b, recorded by the Hermitian-part pass), so N_t < w_min^3 / 2 means no weighted
// triangle (N_t is then rounding noise of an exact zero) and B_t is NaN.
__global__ void __launch_bounds__(kFinBlock)
finalize_kernel(const double* __restrict__ part, long long partset, int nblk, const int* __restrict__ pos,
                const double* __restrict__ part64, long long partset64, int nblk64,
                const int* __restrict__ pos64, int ntrip, int batch, int nisets,
                const double* __restrict__ n_given, const unsigned long long* __restrict__ wmin_bits, int spw,
                double inv_npix, double norm, const int* __restrict__ tmap, int ntrip_out,
                double* __restrict__ B, double* __restrict__ N) {
  const int t = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y;
  const int to = t < ntrip && tmap ? tmap[t] : t;
  const double s = sum_partials(part + (long long)b * partset, nblk, ntrip, pos, t) * inv_npix;
  double nn;
  if (nisets == 0) {
    nn = t < ntrip ? n_given[to] : 0.0;
  } else {
    const int is = nisets > 1 ? b : 0;
    nn = sum_partials_half(part64 + (long long)is * partset64, nblk64, ntrip, pos64, t) * inv_npix;
  }
  if (threadIdx.x < 64 && t < ntrip) {
    const double wm = min_weight(wmin_bits, b, spw);
    B[(long long)b * ntrip_out + to] = nn < 0.5 * wm * wm * wm ? __builtin_nan("") : s / (norm * nn);
    if (N) N[(long long)b * ntrip_out + to] = nn;
  }
}

// Complex input: with W V = H + i G (H and G Hermitian, their ring fields F and E real),
// S = sum (F + i E)(F + i E)(F + i E) has Re S = FFF - (FEE + EFE + EEF) and
// Im S = (EFF + FEF + FFE) - EEE.  The four sets of grid b hold the triple sums of H, G,
// H + G and H - G: T0 = FFF, T1 = EEE, T2 = FFF + sym(EFF) + sym(FEE) + EEE and
// T3 = FFF - sym(EFF) + sym(FEE) - EEE, so Re S = 2 T0 - (T2 + T3) / 2 and
// Im S = (T2 - T3) / 2 - 2 T1.  B[b][t] = (Re S, Im S) / (A N), NaN for empty triplets.
__global__ void __launch_bounds__(kFinBlock)
finalize_complex_kernel(const double* __restrict__ part, long long partset, int nblk, const int* __restrict__ pos,
                        const double* __restrict__ part64, long long partset64, int nblk64,
                        const int* __restrict__ pos64, int ntrip, int nisets, const double* __restrict__ n_given,
                        const unsigned long long* __restrict__ wmin_bits, int spw, double inv_npix, double norm,
                        const int* __restrict__ tmap, int ntrip_out, double* __restrict__ B,
                        double* __restrict__ N) {
  const int t = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y;
  const int to = t < ntrip && tmap ? tmap[t] : t;
  double T[4];
  for (int v = 0; v < 4; ++v)
    T[v] = sum_partials(part + (long long)(4 * b + v) * partset, nblk, ntrip, pos, t) * inv_npix;
  double nn;
  if (nisets == 0) {
    nn = t < ntrip ? n_given[to] : 0.0;
  } else {
    const int is = nisets > 1 ? b : 0;
    nn = sum_partials_half(part64 + (long long)is * partset64, nblk64, ntrip, pos64, t) * inv_npix;
  }
  if (threadIdx.x < 64 && t < ntrip) {
    const double re = 2.0 * T[0] - 0.5 * (T[2] + T[3]);
    const double im = 0.5 * (T[2] - T[3]) - 2.0 * T[1];
    const double wm = min_weight(wmin_bits, b, spw);
    const bool empty = nn < 0.5 * wm * wm * wm;
    B[2 * ((long long)b * ntrip_out + to)] = empty ? __builtin_nan("") : re / (norm * nn);
    B[2 * ((long long)b * ntrip_out + to) + 1] = empty ? __builtin_nan("") : im / (norm * nn);
    if (N) N[(long long)b * ntrip_out + to] = nn;
  }
}

// abs_counts: N_t alone from the weight-set partials.
__global__ void __launch_bounds__(kFinBlock)
counts_kernel(const double* __restrict__ part64, int nblk64, const int* __restrict__ pos64, int ntrip,
              double inv_npix, const int* __restrict__ tmap, double* __restrict__ N) {
  const int t = blockIdx.x * 64 + (threadIdx.x & 63);
  const double nn = sum_partials_half(part64, nblk64, ntrip, pos64, t) * inv_npix;
  if (threadIdx.x < 64 && t < ntrip) N[tmap ? tmap[t] : t] = nn;
}

abs_status ensure_device(abs_plan_s* p) {
  if (!p->dev) return ABS_ERR_UNBOUND;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return ABS_ERR_DEVICE;
  if (cur != p->device) return ABS_ERR_INVALID;  // the plan is bound to another device
  return ABS_OK;
}

// Workgroups: one slice of `waves` triplet groups x one pixel block, numbered so that the
// slices of one pixel block go to one XCD (the kernel decodes blockIdx.x the same way);
// one launch per compiled part of the given kind.
abs_status launch_contract(const abs_plan_s* p, int kind, int waves, const void* F, long long fset,
                           long long npix, int ppb, int nblk, int ntrip, int nsets, double* part,
                           hipStream_t st) {
  // the generated kernels walk a block in pairs of 64-pixel chunks
  if (ppb % 128 != 0 || npix % 128 != 0) return ABS_ERR_INVALID;
  void* Fp = const_cast<void*>(F);
  void* args[] = {&Fp, &fset, &npix, &ppb, &part, &nblk, &ntrip};
  for (const JitPart& q : p->parts) {
    if (q.kind != kind) continue;
    const unsigned gx = 8u * (unsigned)((nblk + 7) / 8) * (unsigned)(q.z1 - q.z0);
    if (hipModuleLaunchKernel(q.fn, gx, (unsigned)nsets, 1, (unsigned)(64 * waves), 1, 1, 0, st, args,
                              nullptr) != hipSuccess)
      return ABS_ERR_DEVICE;
  }
  return ABS_OK;
}

// The plans that run kernels with their workspace layouts and bases: the level plans and
// their parts of the workspace, or the plan itself and the whole workspace.
struct RunLevel {
  const abs_plan_s* q;
  const WorkLayout* wl;
  char* base;
};
std::vector<RunLevel> run_levels(const abs_plan_s* p, const WorkLayout& wl, char* work) {
  std::vector<RunLevel> r;
  if (p->lv.empty()) {
    r.push_back({p, &wl, work});
  } else {
    for (size_t L = 0; L < p->lv.size(); ++L) r.push_back({p->lv[L], &wl.lv[L], work + wl.lvbase[L]});
  }
  return r;
}

// Data sets (FP32) for `batch` grids, then `nisets` weight sets (FP64); partials of
// the data sets first, weight sets after them.  The Hermitian part (and each set's
// smallest ring-cell weight) is formed once for the plan; every level plan transforms its
// own rings from it at its own size and contracts its own triplets.  Stages run one after
// the other over all levels, so that the timing hooks bracket whole stages.  When a call
// has both, the weight sets (which share nothing with the data sets but the cleared wmin
// slots) run on the plan's second stream, forked from `st` after the clearing and joined
// back into `st` at the end, so that their kernels overlap the data sets' ones (1024^2 x
// 16: 0.744 -> 0.678 ms a step; 8192^2 x 16 within the run-to-run spread).
// batch: data sets (spg per grid: 1, or 4 for complex input).
abs_status run_fields_and_contract(abs_plan_s* p, const WorkLayout& wl, int dtype, const void* grids,
                                   const float* w, int w_batched, char* work, hipStream_t st,
                                   const WeightMod* mod, int spg = 1) {
  const std::vector<RunLevel> lv = run_levels(p, wl, work);
  // data sets (spg per grid and channel), and the sets the contraction sees: a
  // multi-frequency grid's nchan channel sets are one set of nbc channel rings
  const int batch = wl.ndsets, C = p->nchan;
  unsigned long long* wmin = reinterpret_cast<unsigned long long*>(work + wl.wmin);
  // Hermitian parts: the data sets', then the weight sets'
  void* xc = work + wl.xc;
  void* xcw = work + wl.xc + (size_t)batch * (size_t)(p->hmax + 1) * (size_t)(2 * p->hmax + 1) * 8;
  {
    const int cnt = batch + wl.nisets;
    fill_u64_kernel<<<(cnt + kBlock - 1) / kBlock, kBlock, 0, st>>>(wmin, cnt, kInfBits);
  }
  auto weight_sets = [&](hipStream_t sw) -> abs_status {
    if (launch_herm_weight(p, w, w_batched, wl.nisets, xcw, wmin + batch, sw, mod) != hipSuccess)
      return ABS_ERR_DEVICE;
    for (const RunLevel& r : lv)
      if (launch_colpass_f64(r.q, wl.nisets, xcw, reinterpret_cast<double2*>(r.base + r.wl->zi), r.wl->zset,
                             sw) != hipSuccess)
        return ABS_ERR_DEVICE;
    for (const RunLevel& r : lv)
      if (launch_rowpass_f64(r.q, wl.nisets, reinterpret_cast<const double2*>(r.base + r.wl->zi), r.wl->zset,
                             reinterpret_cast<double*>(r.base + r.wl->fi), r.wl->fset64, sw) != hipSuccess)
        return ABS_ERR_DEVICE;
    for (const RunLevel& r : lv) {
      const abs_plan_s* q = r.q;
      const abs_status s = launch_contract(q, 1, q->waves64, r.base + r.wl->fi, C * r.wl->fset64, q->npix64,
                                           q->pix_per_block64, q->nblk64, (int)q->ntrip, wl.nipsets,
                                           reinterpret_cast<double*>(r.base + r.wl->part64), sw);
      if (s != ABS_OK) return s;
    }
    return ABS_OK;
  };
  auto data_sets = [&]() -> abs_status {
    prof_begin(p, ABS_STAGE_COLPASS, st);
    if (launch_herm_data(p, grids, dtype, w, w_batched, batch, xc, wmin, st, spg) != hipSuccess)
      return ABS_ERR_DEVICE;
    for (const RunLevel& r : lv)
      if (launch_colpass_f32(r.q, batch, xc, reinterpret_cast<float2*>(r.base + r.wl->zd), r.wl->zset, st) !=
          hipSuccess)
        return ABS_ERR_DEVICE;
    prof_end(p, ABS_STAGE_COLPASS, st);
    // FP16 splits need a power-of-two scale per (grid, ring): the row pass records max |F|
    // for the levels contracted on the matrix units
    auto fp16_level = [&](const abs_plan_s* q) { return p->precision == ABS_FP16X3 && q->use_mfma; };
    for (const RunLevel& r : lv)
      if (fp16_level(r.q)) {
        const int cnt = batch * r.q->nb;
        fill_u32_kernel<<<(cnt + kBlock - 1) / kBlock, kBlock, 0, st>>>(
            reinterpret_cast<unsigned*>(r.base + r.wl->fmax), cnt, 0u);
      }
    prof_begin(p, ABS_STAGE_ROWPASS, st);
    for (const RunLevel& r : lv) {
      unsigned* fmax = fp16_level(r.q) ? reinterpret_cast<unsigned*>(r.base + r.wl->fmax) : nullptr;
      if (launch_rowpass_f32(r.q, batch, reinterpret_cast<const float2*>(r.base + r.wl->zd), r.wl->zset,
                             reinterpret_cast<float*>(r.base + r.wl->fd), r.wl->fset, fmax, st) != hipSuccess)
        return ABS_ERR_DEVICE;
    }
    prof_end(p, ABS_STAGE_ROWPASS, st);
    prof_begin(p, ABS_STAGE_CONTRACT, st);
    for (const RunLevel& r : lv) {
      const abs_plan_s* q = r.q;
      const float* F = reinterpret_cast<const float*>(r.base + r.wl->fd);
      double* part = reinterpret_cast<double*>(r.base + r.wl->part);
      abs_status s;
      if (!q->use_mfma) {
        s = launch_contract(q, 0, q->waves, F, C * r.wl->fset, (long long)q->n * q->n, q->pix_per_block,
                            q->nblk, (int)q->ntrip, wl.npsets, part, st);
      } else {
        const unsigned* fmax =
            p->precision == ABS_FP16X3 ? reinterpret_cast<const unsigned*>(r.base + r.wl->fmax) : nullptr;
        s = launch_mfma_contract(q, F, C * r.wl->fset, wl.npsets, part, fmax, st) == hipSuccess ? ABS_OK
                                                                                               : ABS_ERR_DEVICE;
      }
      if (s != ABS_OK) return s;
    }
    prof_end(p, ABS_STAGE_CONTRACT, st);
    return ABS_OK;
  };
  // the column- and row-pass timing hooks bracket those stages alone: with either set, the
  // weight sets run after the data sets on `st`
  const bool hooked = p->prof[ABS_STAGE_COLPASS][0] || p->prof[ABS_STAGE_COLPASS][1] ||
                      p->prof[ABS_STAGE_ROWPASS][0] || p->prof[ABS_STAGE_ROWPASS][1];
  if (batch > 0 && wl.nisets > 0 && p->aux != nullptr && !hooked) {
    if (hipEventRecord(p->fork, st) != hipSuccess || hipStreamWaitEvent(p->aux, p->fork, 0) != hipSuccess)
      return ABS_ERR_DEVICE;
    const abs_status sw = weight_sets(p->aux);
    const bool recorded = hipEventRecord(p->join, p->aux) == hipSuccess;
    const abs_status sd = data_sets();
    // joined also after a failed launch, so that `st` does not run ahead of queued work
    const bool joined = recorded && hipStreamWaitEvent(st, p->join, 0) == hipSuccess;
    if (sd != ABS_OK) return sd;
    if (sw != ABS_OK) return sw;
    return joined ? ABS_OK : ABS_ERR_DEVICE;
  }
  if (batch > 0) {
    const abs_status sd = data_sets();
    if (sd != ABS_OK) return sd;
  }
  return wl.nisets > 0 ? weight_sets(st) : ABS_OK;
}

// Device tables of a run plan: partial positions and, for a level plan, its triplet map.
const int* dev_pos32(const abs_plan_s* q) {
  return !q->use_mfma ? reinterpret_cast<const int*>(static_cast<const char*>(q->dev) + q->dl.pos32)
                                  : nullptr;   // the precision form writes partials by triplet index
}
const int* dev_pos64(const abs_plan_s* q) {
  return reinterpret_cast<const int*>(static_cast<const char*>(q->dev) + q->dl.pos64);
}
const int* dev_tmap(const abs_plan_s* q) {
  return q->is_level ? reinterpret_cast<const int*>(static_cast<const char*>(q->dev) + q->dl.tmap) : nullptr;
}

}  // namespace abs_impl

using namespace abs_impl;

namespace abs_impl {

// Load a run plan's compiled code and upload its tables to mem (its part of the plan
// memory): twiddles, rings, column tiles, the precision form's tables, partial positions
// and a level's triplet map.
abs_status bind_tables(abs_plan_s* p, void* mem, hipStream_t st) {
  for (JitPart& q : p->parts) {
    if (q.module) {
      (void)hipModuleUnload(q.module);
      q.module = nullptr;
      q.fn = nullptr;
    }
    if (hipModuleLoadData(&q.module, q.code.data()) != hipSuccess) {
      q.module = nullptr;
      return ABS_ERR_JIT;
    }
    if (hipModuleGetFunction(&q.fn, q.module, "abs_contract") != hipSuccess) return ABS_ERR_JIT;
  }
  // host image of the tables
  std::vector<char> img(p->dl.total, 0);
  float2* tw = reinterpret_cast<float2*>(img.data() + p->dl.tw);
  double2* tw64 = reinterpret_cast<double2*>(img.data() + p->dl.tw64);
  for (int k = 0; k < p->n; ++k) {
    const double a = -2.0 * M_PI * (double)k / (double)p->n;  // forward DFT sign
    tw64[k] = make_double2(std::cos(a), std::sin(a));
    tw[k] = make_float2((float)tw64[k].x, (float)tw64[k].y);
  }
  BinDev* bins = reinterpret_cast<BinDev*>(img.data() + p->dl.bins);
  for (int m = 0; m < p->nb; ++m) {
    // integer bounds: for an integer d, d >= x exactly when d >= ceil(x), and d < x
    // exactly when d < ceil(x)
    auto ibound = [](double x) { return (int32_t)std::min(std::max(std::ceil(x), 0.0), 2147483647.0); };
    bins[m].d2lo = ibound(p->lo2[m]);
    bins[m].d2hi = ibound(p->hi2[m]);
    bins[m].h = p->h[m];
    bins[m].cols = p->cols[m];
    bins[m].zoff = p->zoff[m];
  }
  std::memcpy(img.data() + p->dl.tiles, p->tiles.data(), p->tiles.size() * sizeof(ColTile));
  std::memcpy(img.data() + p->dl.tiles64, p->tiles64.data(), p->tiles64.size() * sizeof(ColTile));
  auto put = [&](size_t off, const std::vector<int>& v) {
    std::memcpy(img.data() + off, v.data(), v.size() * sizeof(int));
  };
  put(p->dl.pt_pairs, p->pt_pairs);
  put(p->dl.mt_ptile, p->mt_ptile);
  put(p->dl.mt_bins, p->mt_bins);
  put(p->dl.mt_trip, p->mt_trip);
  put(p->dl.wave_tiles, p->wave_tiles);
  put(p->dl.pos32, p->pos32);
  put(p->dl.pos64, p->pos64);
  put(p->dl.tmap, p->tmap);
  if (hipMemcpyAsync(mem, img.data(), img.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    return ABS_ERR_DEVICE;
  // the host image is a local: wait for the copy before it goes out of scope
  if (hipStreamSynchronize(st) != hipSuccess) return ABS_ERR_DEVICE;
  p->dev = mem;
  return ABS_OK;
}

}  // namespace abs_impl

extern "C" {

abs_status abs_plan_bind(abs_plan_t p, void* mem, size_t bytes, void* stream) {
  if (!p || !mem) return ABS_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(mem) & 255) return ABS_ERR_INVALID;
  if (bytes < p->dl.total) return ABS_ERR_NOMEM;
  for (abs_plan_s* q : run_plans(p))
    for (int k = 0; k < (int)q->parts.size(); ++k) {
      const abs_status s = compile_jit(q, k);
      if (s != ABS_OK) return s;
    }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return ABS_ERR_DEVICE;
  for (abs_plan_s* q : run_plans(p)) {
    const abs_status s = bind_tables(q, static_cast<char*>(mem) + q->dev_off, st);
    if (s != ABS_OK) return s;
    q->device = dev;
  }
  // the second stream and events of the weight sets, on this device (default priority)
  if (p->aux_device != dev) {
    release_aux(p);
    if (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->join, hipEventDisableTiming) != hipSuccess) {
      p->aux_device = dev;
      release_aux(p);
      return ABS_ERR_DEVICE;
    }
    p->aux_device = dev;
  }
  p->dev = mem;
  p->device = dev;
  return ABS_OK;
}

}  // extern "C"

namespace abs_impl {

// Argument checks shared by abs_estimate and abs_estimate_noalloc (everything but the
// workspace).
abs_status check_estimate_args(abs_plan_t p, int32_t batch, int32_t dtype, const void* grids,
                               const float* w, int32_t w_batched, const double* n_given, double* B) {
  if (!p) return ABS_ERR_INVALID;
  abs_status s = ensure_device(p);
  if (s != ABS_OK) return s;
  if (batch < 1 || batch > p->max_batch) return ABS_ERR_INVALID;
  if (dtype != ABS_C64 && dtype != ABS_C128) return ABS_ERR_INVALID;
  if (!grids || !B) return ABS_ERR_INVALID;
  if (!w && p->wmode != ABS_W_UNIT) return ABS_ERR_INVALID;
  if (n_given && w_batched) return ABS_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(grids) & 15) return ABS_ERR_INVALID;
  return ABS_OK;
}

// The launches of one estimate on a workspace of at least work_layout(...).total bytes.
abs_status estimate_on(abs_plan_t p, const WorkLayout& wl, int32_t batch, int32_t dtype, const void* grids,
                       const float* w, int32_t w_batched, const double* n_given, char* wk, double* B,
                       double* N, hipStream_t st) {
  (void)hipGetLastError();
  abs_status s = run_fields_and_contract(p, wl, dtype, grids, w, w_batched, wk, st, nullptr);
  if (s != ABS_OK) return s;
  const unsigned long long* wmin = reinterpret_cast<const unsigned long long*>(wk + wl.wmin);
  for (const RunLevel& r : run_levels(p, wl, wk)) {
    const abs_plan_s* q = r.q;
    const double inv = 1.0 / ((double)q->n * (double)q->n);
    const dim3 g((unsigned)((q->ntrip + 63) / 64), (unsigned)batch);
    finalize_kernel<<<g, kFinBlock, 0, st>>>(reinterpret_cast<const double*>(r.base + r.wl->part), r.wl->partset,
                                          q->nblk, dev_pos32(q), reinterpret_cast<const double*>(r.base + r.wl->part64),
                                          r.wl->partset64, q->nblk64, dev_pos64(q), (int)q->ntrip, batch,
                                          wl.nipsets, n_given, wmin, p->nchan, inv, p->norm, dev_tmap(q),
                                          (int)p->ntrip, B, N);
  }
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

// Scratch of the allocation-free entry point: one static array per GPU (each device holds
// its own copy at its own address until the process ends).  Host code never passes the
// array's name to a kernel: that names a host-side stand-in.  Its device address is
// looked up once per device with hipGetSymbolAddress and kept in scratch_ptr.
constexpr size_t kScratchBytes = ABS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use there).
abs_status scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ABS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ABS_ERR_DEVICE;
    scratch_ptr[dev] = ptr;
  }
  *out = scratch_ptr[dev];
  return ABS_OK;
}

}  // namespace abs_impl

extern "C" {

abs_status abs_estimate(abs_plan_t p, int32_t batch, int32_t dtype, const void* grids,
                        const float* w, int32_t w_batched, const double* n_given, void* work,
                        size_t work_bytes, double* B, double* N, void* stream) {
  abs_status s = check_estimate_args(p, batch, dtype, grids, w, w_batched, n_given, B);
  if (s != ABS_OK) return s;
  if (!work || (reinterpret_cast<uintptr_t>(work) & 15)) return ABS_ERR_INVALID;
  const WorkLayout wl = work_layout(p, batch, w_batched, n_given != nullptr);
  if (work_bytes < wl.total) return ABS_ERR_NOMEM;
  return estimate_on(p, wl, batch, dtype, grids, w, w_batched, n_given, static_cast<char*>(work), B, N,
                     static_cast<hipStream_t>(stream));
}

abs_status abs_estimate_complex_workspace(abs_plan_t p, int32_t batch, int32_t w_batched, int32_t have_counts,
                                          size_t* bytes) {
  if (!p || !bytes || batch < 0 || batch > p->max_batch) return ABS_ERR_INVALID;
  *bytes = work_layout(p, batch, w_batched, have_counts, 4).total;
  return ABS_OK;
}

abs_status abs_estimate_complex(abs_plan_t p, int32_t batch, int32_t dtype, const void* grids, const float* w,
                                int32_t w_batched, const double* n_given, void* work, size_t work_bytes,
                                double* B, double* N, void* stream) {
  abs_status s = check_estimate_args(p, batch, dtype, grids, w, w_batched, n_given, B);
  if (s != ABS_OK) return s;
  if (p->nchan > 1) return ABS_ERR_INVALID;   // single-frequency plans only
  if (!work || (reinterpret_cast<uintptr_t>(work) & 15)) return ABS_ERR_INVALID;
  const WorkLayout wl = work_layout(p, batch, w_batched, n_given != nullptr, 4);
  if (work_bytes < wl.total) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wk = static_cast<char*>(work);
  (void)hipGetLastError();
  s = run_fields_and_contract(p, wl, dtype, grids, w, w_batched, wk, st, nullptr, 4);
  if (s != ABS_OK) return s;
  const unsigned long long* wmin = reinterpret_cast<const unsigned long long*>(wk + wl.wmin);
  for (const RunLevel& r : run_levels(p, wl, wk)) {
    const abs_plan_s* q = r.q;
    const dim3 g((unsigned)((q->ntrip + 63) / 64), (unsigned)batch);
    finalize_complex_kernel<<<g, kFinBlock, 0, st>>>(
        reinterpret_cast<const double*>(r.base + r.wl->part), r.wl->partset, q->nblk, dev_pos32(q),
        reinterpret_cast<const double*>(r.base + r.wl->part64), r.wl->partset64, q->nblk64, dev_pos64(q),
        (int)q->ntrip, wl.nipsets, n_given, wmin, 4, 1.0 / ((double)q->n * (double)q->n), p->norm, dev_tmap(q),
        (int)p->ntrip, B, N);
  }
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

abs_status abs_estimate_noalloc(abs_plan_t p, int32_t batch, int32_t dtype, const void* grids,
                                const float* w, int32_t w_batched, const double* n_given, double* B,
                                double* N, void* stream) {
  abs_status s = check_estimate_args(p, batch, dtype, grids, w, w_batched, n_given, B);
  if (s != ABS_OK) return s;
  const WorkLayout wl = work_layout(p, batch, w_batched, n_given != nullptr);
  if (wl.total > kScratchBytes) return ABS_ERR_SCRATCH;
  void* work = nullptr;
  if ((s = scratch_on_current_device(&work)) != ABS_OK) return s;
  return estimate_on(p, wl, batch, dtype, grids, w, w_batched, n_given, static_cast<char*>(work), B, N,
                     static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace abs_impl {

// N_t of one weight set into N (device, ntrip), on a workspace of work_layout(p, 0, 0, 0)
// bytes, with the weights optionally modulated (mod); the smallest non-zero ring-cell
// weight of the set lands in the workspace's wmin slot 0.
abs_status counts_into(abs_plan_s* p, const float* w, char* wk, const WeightMod* mod, double* N,
                       hipStream_t st) {
  const WorkLayout wl = work_layout(p, 0, 0, 0);
  (void)hipGetLastError();
  // batch 0: the single set is the weight set
  abs_status s = run_fields_and_contract(p, wl, ABS_C64, nullptr, w, 0, wk, st, mod);
  if (s != ABS_OK) return s;
  for (const RunLevel& r : run_levels(p, wl, wk)) {
    const abs_plan_s* q = r.q;
    counts_kernel<<<(unsigned)((q->ntrip + 63) / 64), kFinBlock, 0, st>>>(
        reinterpret_cast<const double*>(r.base + r.wl->part64), q->nblk64, dev_pos64(q), (int)q->ntrip,
        1.0 / ((double)q->n * (double)q->n), dev_tmap(q), N);
  }
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

}  // namespace abs_impl

extern "C" {

abs_status abs_counts(abs_plan_t p, const float* w, void* work, size_t work_bytes, double* N,
                      void* stream) {
  if (!p) return ABS_ERR_INVALID;
  abs_status s = ensure_device(p);
  if (s != ABS_OK) return s;
  if (!work || !N || (!w && p->wmode != ABS_W_UNIT)) return ABS_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(work) & 15) return ABS_ERR_INVALID;
  if (work_bytes < work_layout(p, 0, 0, 0).total) return ABS_ERR_NOMEM;
  return counts_into(p, w, static_cast<char*>(work), nullptr, N, static_cast<hipStream_t>(stream));
}

abs_status abs_profile(abs_plan_t p, int32_t stage, void* ev_begin, void* ev_end) {
  if (!p || stage < 0 || stage > 3) return ABS_ERR_INVALID;
  p->prof[stage][0] = static_cast<hipEvent_t>(ev_begin);
  p->prof[stage][1] = static_cast<hipEvent_t>(ev_end);
  return ABS_OK;
}

abs_status abs_sync(abs_plan_t p, void* stream) {
  (void)p;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return ABS_ERR_DEVICE;
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

}  // extern "C"
