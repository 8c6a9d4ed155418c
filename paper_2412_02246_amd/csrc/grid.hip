// Gridding of visibilities onto the uv grid, Eq. (9) of Gill et al. (2024).
//
// Each visibility V_i at baseline U_i adds w~ w_i V_i to the cells around g = rint(U_i / du)
// and, since the sky is real (V(-U) = conj V(U), Eq. 4), w~ w_i conj(V_i) to the mirrored
// cells -g; the weight sums N_g collect w~ w_i at both.
//
// The batch of realisations shares the baselines, so the visibilities are sorted by
// their nearest cell once (counting sort) and every cell then gathers its own
// contributions: no floating-point atomics, and the sums are accumulated as 64-bit
// fixed-point integers with a power-of-two scale, so the result is independent of
// the order inside each cell (bitwise reproducible).
//   prep:    nearest cell per visibility, per-cell counts, largest |w V| and w, and a
//            realisation-minor copy of the values (one 8*batch-byte record per baseline)
//   scan:    exclusive prefix sum of the counts (three kernels)
//   fill:    visibility indices into per-cell lists
//   gather:  one thread per cell sums its list and the list of its mirror cell
//            (7 x 7 neighbouring lists for the Gaussian kernel) and writes FP32.
#include <algorithm>

#include "abs_internal.h"

namespace abs_impl {

struct GridScalars {
  unsigned int vmax_bits;   // largest |w V| component over all realisations (float bits)
  unsigned int wmax_bits;   // largest w
  unsigned long long dropped;
};

constexpr int kScanItems = 16;                    // per thread
constexpr int kScanTile = kBlock * kScanItems;    // per block

__global__ void __launch_bounds__(kBlock)
grid_clear_kernel(int* __restrict__ cnt, long long ncnt, GridScalars* sc) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ncnt; i += stride) cnt[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->vmax_bits = 0u;
    sc->wmax_bits = 0u;
    sc->dropped = 0ull;
  }
}

__device__ __forceinline__ float block_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  __shared__ float red[kBlock / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  float r = 0.f;
  for (int k = 0; k < kBlock / 64; ++k) r = fmaxf(r, red[k]);
  __syncthreads();
  return r;
}

// Nearest cell of baseline U (index iy * n + ix), or -1 when g or -g is off the grid.
__device__ __forceinline__ int nearest_cell(double2 U, double du, int n) {
  const double fx = rint(U.x / du), fy = rint(U.y / du);
  const double half = 0.5 * n;
  if (!(fx > -half && fx < half && fy > -half && fy < half)) return -1;  // NaN lands here too
  const int gx = (int)fx, gy = (int)fy;
  return (gy < 0 ? gy + n : gy) * n + (gx < 0 ? gx + n : gx);
}

__global__ void __launch_bounds__(kBlock)
grid_prep_kernel(int n, double du, long long nvis, int batch, const double2* __restrict__ uv,
                 const float2* __restrict__ vis, const float* __restrict__ vw, int* __restrict__ cell,
                 int* __restrict__ cnt, float2* __restrict__ visT, GridScalars* sc) {
  float vm = 0.f, wm = 0.f;
  unsigned long long ndrop = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const int c = nearest_cell(uv[i], du, n);
    cell[i] = c;
    if (c < 0) {
      ++ndrop;
      continue;
    }
    atomicAdd(&cnt[c], 1);
    const float wi = vw ? vw[i] : 1.0f;
    wm = fmaxf(wm, fabsf(wi));
    for (int b = 0; b < batch; ++b) {
      const float2 v = vis[(long long)b * nvis + i];
      visT[i * batch + b] = v;
      vm = fmaxf(vm, fabsf(wi) * fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  }
  vm = block_max(vm);
  wm = block_max(wm);
  for (int o = 32; o > 0; o >>= 1) ndrop += __shfl_xor(ndrop, o);
  if ((threadIdx.x & 63) == 0 && ndrop) atomicAdd(&sc->dropped, ndrop);
  if (threadIdx.x == 0) {
    // non-negative floats order like their bit patterns
    atomicMax(&sc->vmax_bits, __float_as_uint(vm));
    atomicMax(&sc->wmax_bits, __float_as_uint(wm));
  }
}

// Exclusive scan of cnt[0 .. ncells) into start[0 .. ncells], in three launches.
__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < kBlock / 64; ++k) {
    if (k < wave) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kBlock)
scan_tiles_kernel(const int* __restrict__ cnt, long long ncells, int* __restrict__ start,
                  int* __restrict__ tile_sum) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + k;
    v[k] = i < ncells ? cnt[i] : 0;
    s += v[k];
  }
  int total;
  int run = block_exclusive_scan(s, &total);
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + k;
    if (i < ncells) start[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock)
scan_sums_kernel(int* __restrict__ tile_sum, int ntiles, int* __restrict__ start, long long ncells) {
  // one block: exclusive scan of the tile totals, in chunks of kBlock
  int carry = 0;
  for (int c0 = 0; c0 < ntiles; c0 += kBlock) {
    const int i = c0 + threadIdx.x;
    const int v = i < ntiles ? tile_sum[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, &total);
    if (i < ntiles) tile_sum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) start[ncells] = carry;
}

__global__ void __launch_bounds__(kBlock)
scan_add_kernel(int* __restrict__ start, long long ncells, const int* __restrict__ tile_sum) {
  const long long base = (long long)blockIdx.x * kScanTile;
  const int add = tile_sum[blockIdx.x];
  for (int k = threadIdx.x; k < kScanTile; k += blockDim.x) {
    const long long i = base + k;
    if (i < ncells) start[i] += add;
  }
}

__global__ void __launch_bounds__(kBlock)
grid_fill_kernel(long long nvis, const int* __restrict__ cell, const int* __restrict__ start,
                 int* __restrict__ cnt, int* __restrict__ list) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const int c = cell[i];
    if (c < 0) continue;
    const int slot = atomicSub(&cnt[c], 1) - 1;   // counts run down to zero
    list[start[c] + slot] = (int)i;
  }
}

// Power-of-two scale 2^E such that 2 * nvis contributions of magnitude <= maxval fit
// in 62 bits (each visibility reaches a cell at most twice: directly and mirrored).
__device__ __forceinline__ double fixed_scale(float maxval, long long nvis) {
  if (!(maxval > 0.f)) return 1.0;
  int e;
  (void)frexpf(maxval, &e);               // maxval < 2^e
  int lg = 0;
  while ((1ll << lg) < 2 * (nvis > 0 ? nvis : 1)) ++lg;
  return ldexp(1.0, 61 - e - lg);
}

__device__ __forceinline__ long long fx(double v, double s) { return llrint(v * s); }

// One thread per cell (iy, ix): sums the visibilities whose nearest cell is within
// R cells of it, directly (V) and through the mirror (conj V).  B is the compile-time
// batch chunk held in registers; `b0` selects the chunk.
template <int R, int B>
__global__ void __launch_bounds__(kBlock)
grid_gather_kernel(int n, double du, double pit2, long long nvis, int batch, int b0,
                   const double2* __restrict__ uv, const float2* __restrict__ visT,
                   const float* __restrict__ vw, const int* __restrict__ start,
                   const int* __restrict__ list, int integer_counts, const GridScalars* sc,
                   float2* __restrict__ grid, float* __restrict__ wsum) {
  const long long nn = (long long)n * n;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nn) return;
  const int iy = (int)(c / n), ix = (int)(c - (long long)iy * n);
  const int gy = iy < n / 2 ? iy : iy - n, gx = ix < n / 2 ? ix : ix - n;
  const double sv = fixed_scale(__uint_as_float(sc->vmax_bits), nvis);
  const double sw = integer_counts ? 1.0 : fixed_scale(__uint_as_float(sc->wmax_bits), nvis);
  const int nb = min(B, batch - b0);
  long long ar[B], ai[B];
#pragma unroll
  for (int b = 0; b < B; ++b) ar[b] = ai[b] = 0;
  long long aw = 0;
  const bool want_w = wsum != nullptr && b0 == 0;
  const int half = n / 2;
  if (gx > -half && gy > -half) {   // cells of the row / column -n/2 receive nothing
    for (int mir = 0; mir < 2; ++mir) {
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          // source cell s: direct pass s = g + d, mirrored pass s = -g + d
          const int sx = (mir ? -gx : gx) + dx, sy = (mir ? -gy : gy) + dy;
          if (!(sx > -half && sx < half && sy > -half && sy < half)) continue;
          const int sc_idx = (sy < 0 ? sy + n : sy) * n + (sx < 0 ? sx + n : sx);
          const int p0 = start[sc_idx], p1 = start[sc_idx + 1];
          for (int p = p0; p < p1; ++p) {
            const int i = list[p];
            double kw = 1.0;
            if (R > 0) {
              const double2 U = uv[i];
              // the contribution sits at the cell g (direct) or at -g (mirrored)
              const double ex = (mir ? -(double)gx : (double)gx) * du - U.x;
              const double ey = (mir ? -(double)gy : (double)gy) * du - U.y;
              kw = exp(-pit2 * (ex * ex + ey * ey));
            }
            const double cw = kw * (double)(vw ? vw[i] : 1.0f);
            if (want_w) aw += fx(cw, sw);
            const float2* vr = visT + (long long)i * batch + b0;
#pragma unroll
            for (int b = 0; b < B; ++b) {
              if (b < nb) {
                const float2 v = vr[b];
                ar[b] += fx(cw * (double)v.x, sv);
                ai[b] += mir ? -fx(cw * (double)v.y, sv) : fx(cw * (double)v.y, sv);
              }
            }
          }
        }
    }
  }
  const double iv = 1.0 / sv;  // a power of two: exact
#pragma unroll
  for (int b = 0; b < B; ++b)
    if (b < nb) grid[(long long)(b0 + b) * nn + c] = make_float2((float)((double)ar[b] * iv), (float)((double)ai[b] * iv));
  if (want_w) wsum[c] = (float)((double)aw / sw);
}

__global__ void grid_dropped_kernel(const GridScalars* sc, long long* dropped) {
  *dropped = (long long)sc->dropped;
}

struct GridWork {
  size_t sc, cell, cnt, start, tiles, list, visT, total;
};

GridWork grid_layout(long long n, long long nvis, int batch) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  GridWork g{};
  const long long cells = n * n;
  const long long ntiles = (cells + kScanTile - 1) / kScanTile;
  size_t off = 0;
  g.sc = off;
  off = al(off + sizeof(GridScalars));
  g.cell = off;
  off = al(off + (size_t)nvis * 4);
  g.cnt = off;
  off = al(off + (size_t)cells * 4);
  g.start = off;
  off = al(off + (size_t)(cells + 1) * 4);
  g.tiles = off;
  off = al(off + (size_t)ntiles * 4);
  g.list = off;
  off = al(off + (size_t)nvis * 4);
  g.visT = off;
  off = al(off + (size_t)nvis * batch * 8);
  g.total = off;
  return g;
}

}  // namespace abs_impl

using namespace abs_impl;

extern "C" abs_status abs_grid_workspace(abs_plan_t p, int64_t nvis, int32_t batch, size_t* bytes) {
  if (!p || !bytes || nvis < 0 || batch < 1 || batch > p->max_batch) return ABS_ERR_INVALID;
  if (nvis > 0x7fffffffLL) return ABS_ERR_INVALID;   // list entries are 32-bit indices
  *bytes = grid_layout(p->n, nvis, batch).total;
  return ABS_OK;
}

extern "C" abs_status abs_grid(abs_plan_t p, int64_t nvis, int32_t batch, const double* uv,
                               const float* vis, const float* vis_w, int32_t kernel, void* work,
                               size_t work_bytes, float* grid, float* wsum, int64_t* dropped,
                               void* stream) {
  if (!p) return ABS_ERR_INVALID;
  if (!p->dev) return ABS_ERR_UNBOUND;
  if (nvis < 0 || nvis > 0x7fffffffLL || batch < 1 || batch > p->max_batch) return ABS_ERR_INVALID;
  if (kernel != ABS_NEAREST && kernel != ABS_GAUSS7) return ABS_ERR_INVALID;
  if (!work || !grid || (nvis > 0 && (!uv || !vis))) return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(uv) | reinterpret_cast<uintptr_t>(vis) |
       reinterpret_cast<uintptr_t>(grid) | reinterpret_cast<uintptr_t>(work)) & 15)
    return ABS_ERR_INVALID;
  const GridWork gl = grid_layout(p->n, nvis, batch);
  if (work_bytes < gl.total) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wk = static_cast<char*>(work);
  GridScalars* sc = reinterpret_cast<GridScalars*>(wk + gl.sc);
  int* cell = reinterpret_cast<int*>(wk + gl.cell);
  int* cnt = reinterpret_cast<int*>(wk + gl.cnt);
  int* start = reinterpret_cast<int*>(wk + gl.start);
  int* tsum = reinterpret_cast<int*>(wk + gl.tiles);
  int* list = reinterpret_cast<int*>(wk + gl.list);
  float2* visT = reinterpret_cast<float2*>(wk + gl.visT);
  const long long cells = (long long)p->n * p->n;
  const int ntiles = (int)((cells + kScanTile - 1) / kScanTile);
  const int integer_counts = (vis_w == nullptr && kernel == ABS_NEAREST) ? 1 : 0;
  const double pi = 3.14159265358979323846;
  const double pit2 = pi * pi * p->theta0 * p->theta0;
  const double2* uvd = reinterpret_cast<const double2*>(uv);
  (void)hipGetLastError();
  prof_begin(p, ABS_STAGE_GRID, st);
  grid_clear_kernel<<<1024, kBlock, 0, st>>>(cnt, cells, sc);
  const unsigned gv = (unsigned)std::min<long long>(8192, std::max<long long>(1, (nvis + kBlock - 1) / kBlock));
  if (nvis > 0)
    grid_prep_kernel<<<gv, kBlock, 0, st>>>(p->n, p->du, nvis, batch, uvd,
                                            reinterpret_cast<const float2*>(vis), vis_w, cell, cnt,
                                            visT, sc);
  scan_tiles_kernel<<<ntiles, kBlock, 0, st>>>(cnt, cells, start, tsum);
  scan_sums_kernel<<<1, kBlock, 0, st>>>(tsum, ntiles, start, cells);
  scan_add_kernel<<<ntiles, kBlock, 0, st>>>(start, cells, tsum);
  if (nvis > 0) grid_fill_kernel<<<gv, kBlock, 0, st>>>(nvis, cell, start, cnt, list);
  const unsigned gc = (unsigned)((cells + kBlock - 1) / kBlock);
  constexpr int kChunk = 8;
  for (int b0 = 0; b0 < batch; b0 += kChunk) {
    if (kernel == ABS_GAUSS7)
      grid_gather_kernel<3, kChunk><<<gc, kBlock, 0, st>>>(
          p->n, p->du, pit2, nvis, batch, b0, uvd, visT, vis_w, start, list, integer_counts, sc,
          reinterpret_cast<float2*>(grid), wsum);
    else
      grid_gather_kernel<0, kChunk><<<gc, kBlock, 0, st>>>(
          p->n, p->du, pit2, nvis, batch, b0, uvd, visT, vis_w, start, list, integer_counts, sc,
          reinterpret_cast<float2*>(grid), wsum);
  }
  if (dropped) grid_dropped_kernel<<<1, 1, 0, st>>>(sc, reinterpret_cast<long long*>(dropped));
  prof_end(p, ABS_STAGE_GRID, st);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}
