// Gridding of visibilities onto the uv grid, Eq. (9) of Gill et al. (2024).
//
// Each visibility V_i at baseline U_i adds w~ w_i V_i to the cells around g = rint(U_i / du)
// and, since the sky is real (V(-U) = conj V(U), Eq. 4), w~ w_i conj(V_i) to the mirrored
// cells -g; the weight sums N_g collect w~ w_i at both.
//
// The batch of realisations shares the baselines, so the visibilities are sorted by
// their nearest cell once (counting sort) and every cell then gathers its own
// contributions: no floating-point atomics, and every sum is exact (FP64 sums that no
// rounding can touch, or 64-bit fixed-point integers with a power-of-two scale), so the
// result is independent of the order inside each cell (bitwise reproducible).
//   prep:    nearest cell per visibility, per-cell counts (the count before a
//            visibility's own increment is its rank in its cell), largest w
//   scan:    exclusive prefix sum of the counts (three kernels)
//   fill:    every visibility's values for all realisations copied, as one record of
//            8*batch bytes, to its slot start[cell] + rank in cell order (and its index,
//            when weights or the Gaussian kernel need it); largest |w V|
//   gather:  unit weights, nearest cell: one lane group per mirror pair of cells
//            (g, -g) sums each cell's records once and writes both cells; otherwise
//            one lane group per cell streams the records of its cell and of its mirror
//            cell (7 x 7 neighbouring cells for the Gaussian kernel).  16 realisations
//            per pass, FP32 out.
//
// A baseline set gridded many times (the realisations of a simulation share one baseline
// distribution, Sec. 3) is sorted once instead (abs_grid_sort): every visibility gets a
// slot, the slots ordered by mirror pair of cells (g, -g) and within a pair the visibilities
// nearest to g before those nearest to -g, and a table keeps where each pair's run starts.
// The caller keeps its visibilities in slot order, as records of the batch's values
// ([slot][batch], the layout the fill pass writes), and abs_grid_sorted is then the pair
// gather alone: every record read once, every cell written once.
#include <algorithm>

#include "abs_internal.h"

namespace abs_impl {

struct GridScalars {
  unsigned int vmax_bits;   // largest |w V| component over all realisations (float bits)
  unsigned int wmax_bits;   // largest w
  unsigned long long dropped;
  int maxcnt;               // most visibilities with one nearest cell
};

constexpr int kScanItems = 16;                    // per thread
constexpr int kScanTile = kBlock * kScanItems;    // per block
constexpr int kRec = 16;                          // realisations per fill / gather pass

__global__ void __launch_bounds__(kBlock)
grid_clear_kernel(int* __restrict__ cnt, long long ncnt, GridScalars* sc) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ncnt; i += stride) cnt[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->vmax_bits = 0u;
    sc->wmax_bits = 0u;
    sc->dropped = 0ull;
    sc->maxcnt = 0;
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

// The pair of cells (g, -g) has one representative cell (iy, ix): rows 0 .. n/2, and in
// rows 0 and n/2 only columns 0 .. n/2.  Pair index lc = iy * n + ix of the representative;
// (n/2 + 1) n indices, some unused.  Sort key of a visibility with nearest cell c: 2 lc if c
// is the representative of pair lc, 2 lc + 1 if c is its mirror; -1 for a dropped one.
__device__ __forceinline__ int pair_key(int c, int n) {
  if (c < 0) return -1;
  const int half = n / 2;
  const int iy = c / n, ix = c - iy * n;
  if (iy <= half && !((iy == 0 || iy == half) && ix > half)) return 2 * c;
  const int my = iy ? n - iy : 0, mx = ix ? n - ix : 0;
  return 2 * (my * n + mx) + 1;
}

// KEY = false: counting-sort key = nearest cell (abs_grid); true: pair_key (abs_grid_sort)
template <bool KEY>
__global__ void __launch_bounds__(kBlock)
grid_prep_kernel(int n, double du, long long nvis, const double2* __restrict__ uv,
                 const float* __restrict__ vw, int* __restrict__ cell, int* __restrict__ rank,
                 int* __restrict__ cnt, GridScalars* sc) {
  float wm = 0.f;
  unsigned long long ndrop = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const int c = KEY ? pair_key(nearest_cell(uv[i], du, n), n) : nearest_cell(uv[i], du, n);
    cell[i] = c;
    if (c < 0) {
      ++ndrop;
      continue;
    }
    rank[i] = atomicAdd(&cnt[c], 1);
    wm = fmaxf(wm, fabsf(vw ? vw[i] : 1.0f));
  }
  wm = block_max(wm);
  for (int o = 32; o > 0; o >>= 1) ndrop += __shfl_xor(ndrop, o);
  if ((threadIdx.x & 63) == 0 && ndrop) atomicAdd(&sc->dropped, ndrop);
  // non-negative floats order like their bit patterns
  if (threadIdx.x == 0) atomicMax(&sc->wmax_bits, __float_as_uint(wm));
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
                  int* __restrict__ tile_sum, GridScalars* sc) {
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
  int mx = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const long long i = base + k;
    if (i < ncells) start[i] = run;
    run += v[k];
    mx = max(mx, v[k]);
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(&sc->maxcnt, mx);
}

__global__ void __launch_bounds__(kBlock)
scan_sums_kernel(int* __restrict__ tile_sum, int ntiles, int* __restrict__ start, long long ncells,
                 const GridScalars* __restrict__ sc, long long* __restrict__ dropped) {
  // one block: exclusive scan of the tile totals, in chunks of kBlock; also hands out the
  // count of dropped visibilities (final once the prep pass has run), if asked for
  int carry = 0;
  for (int c0 = 0; c0 < ntiles; c0 += kBlock) {
    const int i = c0 + threadIdx.x;
    const int v = i < ntiles ? tile_sum[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, &total);
    if (i < ntiles) tile_sum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    start[ncells] = carry;
    if (dropped) *dropped = (long long)sc->dropped;
  }
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

// One workgroup per kBlock consecutive visibilities.  Each visibility's slot in its
// cell's run of the sorted order is its rank from the prep pass (no atomics here); the
// realisations' values are then copied into
// cell-sorted records sorted[pos * batch + b] through LDS, kRec realisations at a time,
// so that consecutive lanes store consecutive values of whole records (a batch of 16
// fills one 128-byte line per record).  Also finds the largest |w V| component.
__global__ void __launch_bounds__(kBlock)
grid_fill_kernel(long long nvis, int batch, const int* __restrict__ cell,
                 const int* __restrict__ start, const int* __restrict__ rank,
                 const float2* __restrict__ vis, const float* __restrict__ vw,
                 int* __restrict__ list, float2* __restrict__ sorted, GridScalars* sc) {
  __shared__ float2 tile[kRec][kBlock + 1];
  __shared__ int posl[kBlock];
  const long long i0 = (long long)blockIdx.x * kBlock;
  const long long i = i0 + threadIdx.x;
  // the first kRec realisations are loaded before the slot is looked up, so that all
  // the loads are in flight together
  float2 v0[kRec];
#pragma unroll
  for (int bb = 0; bb < kRec; ++bb)
    v0[bb] = (bb < batch && i < nvis) ? vis[(long long)bb * nvis + i] : make_float2(0.f, 0.f);
  int pos = -1;
  float wa = 0.f;
  if (i < nvis) {
    const int c = cell[i];
    if (c >= 0) {
      pos = start[c] + rank[i];
      wa = fabsf(vw ? vw[i] : 1.0f);
      if (list) list[pos] = (int)i;
    }
  }
  posl[threadIdx.x] = pos;
  const int nrow = (int)(nvis - i0 < kBlock ? nvis - i0 : kBlock);
  float vm = 0.f;
  for (int b0 = 0; b0 < batch; b0 += kRec) {
    const int nbc = min(kRec, batch - b0);
    __syncthreads();   // posl written; the previous chunk's tile consumed
#pragma unroll
    for (int bb = 0; bb < kRec; ++bb) {
      if (bb < nbc) {
        float2 v = v0[bb];
        if (b0 > 0) v = i < nvis ? vis[(long long)(b0 + bb) * nvis + i] : make_float2(0.f, 0.f);
        if (pos >= 0) vm = fmaxf(vm, wa * fmaxf(fabsf(v.x), fabsf(v.y)));
        tile[bb][threadIdx.x] = v;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nrow * nbc; e += kBlock) {
      const int r = e / nbc, bb = e - r * nbc;
      const int pr = posl[r];
      if (pr >= 0) sorted[(long long)pr * batch + b0 + bb] = tile[bb][r];
    }
  }
  vm = block_max(vm);
  if (threadIdx.x == 0) atomicMax(&sc->vmax_bits, __float_as_uint(vm));
}

// Sums are formed in fixed point held in FP64: every term is rounded to an integer
// multiple of 2^-E (E from a power-of-two scale) and the running sums stay below 2^52
// in magnitude, so every addition is exact and the sum does not depend on the order of
// its terms (bitwise reproducible).  Terms are at most maxval in size and a cell adds at
// most `terms` of them.
__device__ __forceinline__ double fixed_scale(float maxval, long long terms) {
  if (!(maxval > 0.f)) return 1.0;
  int e;
  (void)frexpf(maxval, &e);               // maxval < 2^e
  int lg = 0;
  while ((1ll << lg) < (terms > 0 ? terms : 1)) ++lg;
  return ldexp(1.0, 51 - e - lg);
}

// Per-visibility weights or the Gaussian kernel (unit weights with the nearest cell go
// through grid_gather_pairs_kernel).  LPC lanes per cell (iy, ix), lane q holding
// realisations b0 + 2q and b0 + 2q + 1: sums the visibilities whose nearest cell is within
// R cells of it, directly (V) and through the mirror (conj V).  The records of one source
// cell are contiguous in `sorted` (VEC: one 16-byte load per record and lane, batch even).
// Lane 0 of each cell also sums the weights when b0 == 0.
template <int R, int LPC, bool VEC>
__global__ void __launch_bounds__(kBlock)
grid_gather_kernel(int n, double du, double pit2, int batch, int b0,
                   const double2* __restrict__ uv, const float2* __restrict__ sorted,
                   const float* __restrict__ vw, const int* __restrict__ start,
                   const int* __restrict__ list, int integer_counts, const GridScalars* sc,
                   float2* __restrict__ grid, float* __restrict__ wsum) {
  const long long nn = (long long)n * n;
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long lc = gt / LPC;
  const int q = (int)(gt - lc * LPC);
  if (lc >= nn) return;
  // rows in the order |gy| = 0, 1, 1, 2, 2, ...: the densely sampled short baselines
  // (the longest lists) are gathered first and do not form a tail
  const int r = (int)(lc / n), ix = (int)(lc - (long long)r * n);
  const int iy = (r & 1) ? n - 1 - (r >> 1) : (r >> 1);
  const long long c = (long long)iy * n + ix;
  const int gy = iy < n / 2 ? iy : iy - n, gx = ix < n / 2 ? ix : ix - n;
  // a cell adds at most 2 (2R + 1)^2 maxcnt terms, each with kernel weight <= 1
  const long long terms = 2ll * (2 * R + 1) * (2 * R + 1) * (long long)sc->maxcnt;
  const double sv = fixed_scale(__uint_as_float(sc->vmax_bits), terms);
  const double sw = integer_counts ? 1.0 : fixed_scale(__uint_as_float(sc->wmax_bits), terms);
  const int bq = b0 + 2 * q;                 // this lane's first realisation
  const bool has0 = bq < batch, has1 = bq + 1 < batch;
  double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0, aw = 0.0;
  const bool want_w = wsum != nullptr && b0 == 0 && q == 0;
  const int half = n / 2;
  auto load = [&](int p) -> float4 {
    const float2* rec = sorted + (long long)p * batch + bq;
    if constexpr (VEC) {
      return has0 ? *reinterpret_cast<const float4*>(rec) : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      const float2 a = has0 ? rec[0] : make_float2(0.f, 0.f);
      const float2 b = has1 ? rec[1] : make_float2(0.f, 0.f);
      return make_float4(a.x, a.y, b.x, b.y);
    }
  };
  const bool inside = gx > -half && gy > -half;   // row / column -n/2 receive nothing
  if (inside) {
    for (int mir = 0; mir < 2; ++mir) {
      const double sgn = mir ? -1.0 : 1.0;
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          // source cell s: direct pass s = g + d, mirrored pass s = -g + d
          const int sx = (mir ? -gx : gx) + dx, sy = (mir ? -gy : gy) + dy;
          if (!(sx > -half && sx < half && sy > -half && sy < half)) continue;
          const int sc_idx = (sy < 0 ? sy + n : sy) * n + (sx < 0 ? sx + n : sx);
          const int p0 = start[sc_idx], p1 = start[sc_idx + 1];
          // two records in flight while one adds
          float4 nx1 = p0 < p1 ? load(p0) : make_float4(0.f, 0.f, 0.f, 0.f);
          float4 nx2 = p0 + 1 < p1 ? load(p0 + 1) : make_float4(0.f, 0.f, 0.f, 0.f);
          for (int p = p0; p < p1; ++p) {
            const float4 v = nx1;
            nx1 = nx2;
            if (p + 2 < p1) nx2 = load(p + 2);
            double cw = 1.0;
            if (R > 0 || vw) {
              const int i = list[p];
              if (R > 0) {
                const double2 U = uv[i];
                // the contribution sits at the cell g (direct) or at -g (mirrored)
                const double ex = (mir ? -(double)gx : (double)gx) * du - U.x;
                const double ey = (mir ? -(double)gy : (double)gy) * du - U.y;
                cw = exp(-pit2 * (ex * ex + ey * ey));
              }
              if (vw) cw *= (double)vw[i];
            }
            if (want_w) aw += rint(cw * sw);
            const double f = cw * sv;
            ar0 += rint((double)v.x * f);
            ai0 += sgn * rint((double)v.y * f);
            ar1 += rint((double)v.z * f);
            ai1 += sgn * rint((double)v.w * f);
          }
        }
    }
  }
  const double iv = 1.0 / sv;  // a power of two: exact
  if (has0) grid[(long long)bq * nn + c] = make_float2((float)(ar0 * iv), (float)(ai0 * iv));
  if (has1) grid[(long long)(bq + 1) * nn + c] = make_float2((float)(ar1 * iv), (float)(ai1 * iv));
  if (want_w) wsum[c] = (float)(aw / sw);
}

// Nearest cell, unit visibility weights: one group of LPC lanes per pair of mirror cells
// (g, -g), reading each cell's records once.  With S_g the exact sum of the records whose
// nearest cell is g, the grid gets S_g + conj S_-g at g and S_-g + conj S_g at -g (so the
// results are bit for bit those of gathering both lists at each cell); the weight sum is
// the record count of both cells.  Representatives:
// rows 0 .. n/2 in order (|gy| ascending: the long lists of short baselines first), and in
// rows 0 and n/2 only columns 0 .. n/2; row and column -n/2 receive nothing.
// The block's results go out through LDS, one realisation plane at a time, so that each
// plane receives runs of PB consecutive cells (and PB mirror cells) rather than runs of
// 64 / LPC.
template <int LPC>
struct PairCell {
  bool valid;        // a representative (not a mirror, not past the half plane)
  long long c, m;    // the cell and its mirror
};
template <int LPC>
__device__ __forceinline__ PairCell<LPC> pair_cell(long long lc, int n) {
  const int half = n / 2;
  PairCell<LPC> r{false, 0, 0};
  if (lc >= (long long)(half + 1) * n) return r;
  const int iy = (int)(lc / n), ix = (int)(lc - (long long)iy * n);
  if ((iy == 0 || iy == half) && ix > half) return r;   // the mirror of a representative
  const int my = iy ? n - iy : 0, mx = ix ? n - ix : 0;
  r.valid = true;
  r.c = (long long)iy * n + ix;
  r.m = (long long)my * n + mx;
  return r;
}

// KEYED = false: `start` holds each cell's run (abs_grid's counting sort by cell).  KEYED =
// true: `start` is a sorted baseline set's table (runs by pair: entry 2 lc, the visibilities
// nearest to g, then from entry 2 lc + 1 those nearest to -g), and records from `ld` on are
// not read.
// Threads a block of the pair gather: kBlock, or 512 with 8 lanes a pair on grids of 8192^2
// and more, where runs of 64 cells a realisation plane (not 32) write faster (16
// realisations of 8192^2: 4.75 against 5.41 ms; at 4096^2 the 256-thread blocks are faster,
// 1.07 against 1.25 ms).
int pair_threads(int n, int lpc) { return lpc == 8 && n >= 8192 ? 512 : kBlock; }

template <int LPC, bool VEC, bool KEYED, int NTH>
__global__ void __launch_bounds__(NTH)
grid_gather_pairs_kernel(int n, int batch, int b0, const float2* __restrict__ sorted,
                         const int* __restrict__ start, long long ld, float2* __restrict__ grid,
                         float* __restrict__ wsum) {
  constexpr int PB = NTH / LPC;   // pairs per block
  __shared__ float2 out_c[2 * LPC][PB + 1], out_m[2 * LPC][PB + 1];   // padded: rows 2q start in different banks
  const long long nn = (long long)n * n;
  const int half = n / 2;
  const int kp = threadIdx.x / LPC, q = threadIdx.x - kp * LPC;
  const long long lc = (long long)blockIdx.x * PB + kp;
  const PairCell<LPC> pc = pair_cell<LPC>(lc, n);
  const long long c = pc.c, m = pc.m;
  const int iy = (int)(c / n), ix = (int)(c - (long long)iy * n);
  const int gy = iy < half ? iy : iy - n, gx = ix < half ? ix : ix - n;
  const bool inside = pc.valid && gx > -half && gy > -half;   // the mirror is inside exactly then
  const int bq = b0 + 2 * q;
  const bool has0 = bq < batch, has1 = bq + 1 < batch;
  auto load = [&](int p) -> float4 {
    const float2* rec = sorted + (long long)p * batch + bq;
    if constexpr (VEC) {
      return has0 ? *reinterpret_cast<const float4*>(rec) : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      const float2 a = has0 ? rec[0] : make_float2(0.f, 0.f);
      const float2 b = has1 ? rec[1] : make_float2(0.f, 0.f);
      return make_float4(a.x, a.y, b.x, b.y);
    }
  };
  // walks one cell's records in chunks of kG with the next chunk's loads in flight
  auto walk = [&](int p0, int cnt, auto&& use) {
    constexpr int kG = 4;
    float4 cur[kG], nxt[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u) cur[u] = u < cnt ? load(p0 + u) : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i0 = 0; i0 < cnt; i0 += kG) {
#pragma unroll
      for (int u = 0; u < kG; ++u)
        nxt[u] = i0 + kG + u < cnt ? load(p0 + i0 + kG + u) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < kG; ++u) use(cur[u]);   // entries past cnt are zero
#pragma unroll
      for (int u = 0; u < kG; ++u) cur[u] = nxt[u];
    }
  };
  int p0 = 0, cd = 0, q0 = 0, cm = 0;
  if (inside && KEYED) {
    // pair index = the representative's cell index c
    const long long a = min((long long)start[2 * c], ld);
    const long long h = max(a, min((long long)start[2 * c + 1], ld));
    const long long e = max(h, min((long long)start[2 * c + 2], ld));
    p0 = (int)a;
    cd = (int)(h - a);
    q0 = (int)h;
    cm = m != c ? (int)(e - h) : cd;
  } else if (inside) {
    p0 = start[c];
    cd = start[c + 1] - p0;
    if (m != c) {
      q0 = start[m];
      cm = start[m + 1] - q0;
    } else {
      cm = cd;
    }
  }
  // One pass sums the pair's records in plain FP64 and bounds their binary exponents.  A
  // non-zero FP32 value x with biased exponent field a' and a = max(a', 1) is an integer
  // multiple of 2^(a - 150) and |x| < 2^(a - 126); so when a realisation's terms (both
  // cells, at most T = cd + cm per sum) satisfy ceil(log2 T) + amax - amin <= 29, every
  // partial sum is a multiple of 2^(amin - 150) below 2^(53 + amin - 150) in magnitude and
  // exact, in any order.  Otherwise (a far wider spread of magnitudes, or Inf / NaN) that
  // realisation is summed again, from the caches, in 64-bit fixed point with the unit
  // 2^(amax - 126 - 51 + lg): each term rounded to it, the sums exact and again
  // order-independent.  Either way the result does not depend on the order of the
  // records, and the decision depends on the values alone.
  const long long terms = (long long)cd + cm;
  int lg = 0;
  while ((1ll << lg) < (terms > 0 ? terms : 1)) ++lg;
  // the largest and smallest non-zero |x| of each realisation, as their bit patterns (which
  // order like the magnitudes); u - 1 sends a zero to the largest unsigned value, out of the
  // minimum
  unsigned umin0 = ~0u, umax0 = 0u, umin1 = ~0u, umax1 = 0u;
  auto expo = [](float x, unsigned& umin, unsigned& umax) {
    const unsigned u = __float_as_uint(x) & 0x7fffffffu;
    umax = max(umax, u);
    umin = min(umin, u - 1u);
  };
  double sc4[4] = {0.0, 0.0, 0.0, 0.0}, sm4[4] = {0.0, 0.0, 0.0, 0.0};
  walk(p0, cd, [&](float4 v) {
    expo(v.x, umin0, umax0);
    expo(v.y, umin0, umax0);
    expo(v.z, umin1, umax1);
    expo(v.w, umin1, umax1);
    sc4[0] += (double)v.x;
    sc4[1] += (double)v.y;
    sc4[2] += (double)v.z;
    sc4[3] += (double)v.w;
  });
  if (m != c) {
    walk(q0, cm, [&](float4 v) {
      expo(v.x, umin0, umax0);
      expo(v.y, umin0, umax0);
      expo(v.z, umin1, umax1);
      expo(v.w, umin1, umax1);
      sm4[0] += (double)v.x;
      sm4[1] += (double)v.y;
      sm4[2] += (double)v.z;
      sm4[3] += (double)v.w;
    });
  }
  // a = max(exponent field, 1) of the largest and the smallest of them (0 / 255 when none)
  const int amax0 = umax0 ? max((int)(umax0 >> 23), 1) : 0, amax1 = umax1 ? max((int)(umax1 >> 23), 1) : 0;
  const int amin0 = umin0 != ~0u ? max((int)((umin0 + 1u) >> 23), 1) : 255;
  const int amin1 = umin1 != ~0u ? max((int)((umin1 + 1u) >> 23), 1) : 255;
  const bool exact0 = amax0 == 0 || (amax0 < 255 && lg + amax0 - amin0 <= 29);
  const bool exact1 = amax1 == 0 || (amax1 < 255 && lg + amax1 - amin1 <= 29);
  double s0 = 1.0, s1 = 1.0;
  if (!(exact0 && exact1)) {
    // all four sums again: fixed point for the realisation(s) that need it, the plain
    // (exact) sums for the other
    if (!exact0) s0 = ldexp(1.0, 177 - min(amax0, 254) - lg);
    if (!exact1) s1 = ldexp(1.0, 177 - min(amax1, 254) - lg);
    auto t0 = [&](float x) { return exact0 ? (double)x : rint((double)x * s0); };
    auto t1 = [&](float x) { return exact1 ? (double)x : rint((double)x * s1); };
    for (int k = 0; k < 4; ++k) sc4[k] = sm4[k] = 0.0;
    walk(p0, cd, [&](float4 v) {
      sc4[0] += t0(v.x);
      sc4[1] += t0(v.y);
      sc4[2] += t1(v.z);
      sc4[3] += t1(v.w);
    });
    if (m != c) {
      walk(q0, cm, [&](float4 v) {
        sm4[0] += t0(v.x);
        sm4[1] += t0(v.y);
        sm4[2] += t1(v.z);
        sm4[3] += t1(v.w);
      });
    }
  }
  if (m == c)
    for (int k = 0; k < 4; ++k) sm4[k] = sc4[k];
  const double i0 = 1.0 / s0, i1 = 1.0 / s1;  // powers of two: exact
  out_c[2 * q][kp] = make_float2((float)((sc4[0] + sm4[0]) * i0), (float)((sc4[1] - sm4[1]) * i0));
  out_c[2 * q + 1][kp] = make_float2((float)((sc4[2] + sm4[2]) * i1), (float)((sc4[3] - sm4[3]) * i1));
  out_m[2 * q][kp] = make_float2((float)((sm4[0] + sc4[0]) * i0), (float)((sm4[1] - sc4[1]) * i0));
  out_m[2 * q + 1][kp] = make_float2((float)((sm4[2] + sc4[2]) * i1), (float)((sm4[3] - sc4[3]) * i1));
  if (pc.valid && wsum != nullptr && b0 == 0 && q == 0) {
    wsum[c] = (float)(cd + cm);
    wsum[m] = (float)(cd + cm);
  }
  __syncthreads();
  // plane r of the pass, pair k: consecutive threads take consecutive pairs
  for (int e = threadIdx.x; e < 2 * LPC * PB; e += NTH) {
    const int r = e / PB, k = e - r * PB;
    if (b0 + r >= batch) continue;
    const PairCell<LPC> w = pair_cell<LPC>((long long)blockIdx.x * PB + k, n);
    if (!w.valid) continue;
    float2* plane = grid + (long long)(b0 + r) * nn;
    plane[w.c] = out_c[r][k];
    if (w.m != w.c) plane[w.m] = out_m[r][k];
  }
}

// ---- baseline sets sorted once (abs_grid_sort / abs_grid_sorted) --------------------------

// Pair indices lc of a grid of side n: (n/2 + 1) n; the sort keys are twice that.
__host__ __device__ inline long long pair_count(int n) { return (long long)(n / 2 + 1) * n; }

// Slot of every kept visibility: perm[start[key] + rank] = i; slots from the kept count on
// get -1, and the kept count is handed out.
__global__ void __launch_bounds__(kBlock)
grid_place_kernel(long long nvis, const int* __restrict__ key, const int* __restrict__ rank,
                  const int* __restrict__ start, long long nkeys, int* __restrict__ perm,
                  long long* __restrict__ kept) {
  const long long total = start[nkeys];
  if (kept && blockIdx.x == 0 && threadIdx.x == 0) *kept = total;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const int k = key[i];
    if (k >= 0) perm[start[k] + rank[i]] = (int)i;
    if (i >= total) perm[i] = -1;
  }
}

// out[k][b] = vis[b][perm[k]] (0 where perm[k] is -1), k < ld: consecutive threads write
// consecutive values of the records.
__global__ void __launch_bounds__(kBlock)
grid_permute_kernel(long long nvis, int batch, const int* __restrict__ perm, long long ld,
                    const float2* __restrict__ vis, float2* __restrict__ out) {
  const long long total = ld * batch;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const long long k = e / batch, b = e - k * batch;
    const int i = perm[k];
    out[e] = (i >= 0 && i < nvis) ? vis[b * nvis + i] : make_float2(0.f, 0.f);
  }
}

// The keyed pair gather for realisations b0 .. b0 + 2 lpc - 1 of `batch` (lanes per pair as
// abs_grid picks them); batch = 0 writes only the counts.
void launch_keyed_pairs(int n, int batch, int b0, int lpc, const float2* rec, const int* start, long long ld,
                        float2* grid, float* wsum, hipStream_t st) {
  const int nth = pair_threads(n, lpc);
  const unsigned gp = (unsigned)((pair_count(n) * lpc + nth - 1) / nth);
  const bool vec = (batch & 1) == 0;
#define ABS_KPAIRS_T(LL, VV, TT) \
  grid_gather_pairs_kernel<LL, VV, true, TT><<<gp, TT, 0, st>>>(n, batch, b0, rec, start, ld, grid, wsum)
#define ABS_KPAIRS(LL, VV) ABS_KPAIRS_T(LL, VV, kBlock)
  switch (lpc * 2 + (vec ? 1 : 0)) {
    case 2: ABS_KPAIRS(1, false); break;
    case 3: ABS_KPAIRS(1, true); break;
    case 4: ABS_KPAIRS(2, false); break;
    case 5: ABS_KPAIRS(2, true); break;
    case 8: ABS_KPAIRS(4, false); break;
    case 9: ABS_KPAIRS(4, true); break;
    case 16: if (nth == 512) ABS_KPAIRS_T(8, false, 512); else ABS_KPAIRS(8, false); break;
    default: if (nth == 512) ABS_KPAIRS_T(8, true, 512); else ABS_KPAIRS(8, true); break;
  }
#undef ABS_KPAIRS
#undef ABS_KPAIRS_T
}

// lanes per cell: enough pairs of realisations for one pass of up to kRec of them
int lanes_per_cell(int batch) {
  const int nbc = std::min(batch, kRec);
  return nbc <= 2 ? 1 : nbc <= 4 ? 2 : nbc <= 8 ? 4 : 8;
}

struct SortWork {
  size_t sc, key, rank, cnt, tiles, total;
};

SortWork sort_layout(long long n, long long nvis) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const long long nkeys = 2 * pair_count((int)n);
  const long long ntiles = (nkeys + kScanTile - 1) / kScanTile;
  SortWork g{};
  size_t off = 0;
  g.sc = off;
  off = al(off + sizeof(GridScalars));
  g.key = off;
  off = al(off + (size_t)nvis * 4);
  g.rank = off;
  off = al(off + (size_t)nvis * 4);
  g.cnt = off;
  off = al(off + (size_t)nkeys * 4);
  g.tiles = off;
  off = al(off + (size_t)ntiles * 4);
  g.total = off;
  return g;
}

size_t set_bytes_of(int n) { return (size_t)(2 * pair_count(n) + 1) * 4; }

struct GridWork {
  size_t sc, cell, rank, cnt, start, tiles, list, sorted, total;
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
  g.rank = off;
  off = al(off + (size_t)nvis * 4);
  g.cnt = off;
  off = al(off + (size_t)cells * 4);
  g.start = off;
  off = al(off + (size_t)(cells + 1) * 4);
  g.tiles = off;
  off = al(off + (size_t)ntiles * 4);
  g.list = off;
  off = al(off + (size_t)nvis * 4);
  g.sorted = off;
  off = al(off + (size_t)nvis * batch * 8);
  g.total = off;
  return g;
}

}  // namespace abs_impl

using namespace abs_impl;

extern "C" abs_status abs_grid_workspace(abs_plan_t p, int64_t nvis, int32_t batch, size_t* bytes) {
  if (!p || !bytes || nvis < 0 || batch < 1 || batch > p->max_batch * p->nchan) return ABS_ERR_INVALID;
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
  if (nvis < 0 || nvis > 0x7fffffffLL || batch < 1 || batch > p->max_batch * p->nchan) return ABS_ERR_INVALID;
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
  int* rank = reinterpret_cast<int*>(wk + gl.rank);
  int* cnt = reinterpret_cast<int*>(wk + gl.cnt);
  int* start = reinterpret_cast<int*>(wk + gl.start);
  int* tsum = reinterpret_cast<int*>(wk + gl.tiles);
  int* list = reinterpret_cast<int*>(wk + gl.list);
  float2* sorted = reinterpret_cast<float2*>(wk + gl.sorted);
  const long long cells = (long long)p->n * p->n;
  const int ntiles = (int)((cells + kScanTile - 1) / kScanTile);
  const int integer_counts = (vis_w == nullptr && kernel == ABS_NEAREST) ? 1 : 0;
  const double pi = 3.14159265358979323846;
  const double pit2 = pi * pi * p->theta0 * p->theta0;
  const double2* uvd = reinterpret_cast<const double2*>(uv);
  // the original index of each sorted entry is needed for per-visibility weights and
  // for the Gaussian kernel's distances
  int* lst = (vis_w != nullptr || kernel == ABS_GAUSS7) ? list : nullptr;
  (void)hipGetLastError();
  prof_begin(p, ABS_STAGE_GRID, st);
  grid_clear_kernel<<<1024, kBlock, 0, st>>>(cnt, cells, sc);
  const unsigned gv = (unsigned)std::min<long long>(8192, std::max<long long>(1, (nvis + kBlock - 1) / kBlock));
  if (nvis > 0) grid_prep_kernel<false><<<gv, kBlock, 0, st>>>(p->n, p->du, nvis, uvd, vis_w, cell, rank, cnt, sc);
  scan_tiles_kernel<<<ntiles, kBlock, 0, st>>>(cnt, cells, start, tsum, sc);
  scan_sums_kernel<<<1, kBlock, 0, st>>>(tsum, ntiles, start, cells, sc, reinterpret_cast<long long*>(dropped));
  scan_add_kernel<<<ntiles, kBlock, 0, st>>>(start, cells, tsum);
  if (nvis > 0)
    grid_fill_kernel<<<(unsigned)((nvis + kBlock - 1) / kBlock), kBlock, 0, st>>>(
        nvis, batch, cell, start, rank, reinterpret_cast<const float2*>(vis), vis_w, lst, sorted, sc);
  const bool vec = (batch & 1) == 0;
  float2* g2 = reinterpret_cast<float2*>(grid);
  const int lpc = lanes_per_cell(batch);
  const unsigned gc = (unsigned)((cells * lpc + kBlock - 1) / kBlock);
  for (int b0 = 0; b0 < batch; b0 += 2 * lpc) {
#define ABS_GATHER(RR, LL, VV)                                                                  \
  grid_gather_kernel<RR, LL, VV><<<gc, kBlock, 0, st>>>(p->n, p->du, pit2, batch, b0, uvd, sorted, \
                                                        vis_w, start, lst, integer_counts, sc, g2, wsum)
#define ABS_GATHER_L(RR, VV)                 \
  switch (lpc) {                             \
    case 1: ABS_GATHER(RR, 1, VV); break;    \
    case 2: ABS_GATHER(RR, 2, VV); break;    \
    case 4: ABS_GATHER(RR, 4, VV); break;    \
    default: ABS_GATHER(RR, 8, VV); break;   \
  }
    if (kernel == ABS_GAUSS7) {
      if (vec) { ABS_GATHER_L(3, true) } else { ABS_GATHER_L(3, false) }
    } else if (vis_w != nullptr) {
      if (vec) { ABS_GATHER_L(0, true) } else { ABS_GATHER_L(0, false) }
    } else {
      // unit weights: one lane group per mirror pair of cells
      const int nth = pair_threads(p->n, lpc);
      const unsigned gp = (unsigned)(((long long)(p->n / 2 + 1) * p->n * lpc + nth - 1) / nth);
#define ABS_PAIRS_T(LL, VV, TT)                                                                       \
  grid_gather_pairs_kernel<LL, VV, false, TT><<<gp, TT, 0, st>>>(p->n, batch, b0, sorted, start, 0, g2, wsum)
#define ABS_PAIRS(LL, VV) ABS_PAIRS_T(LL, VV, kBlock)
      switch (lpc * 2 + (vec ? 1 : 0)) {
        case 2: ABS_PAIRS(1, false); break;
        case 3: ABS_PAIRS(1, true); break;
        case 4: ABS_PAIRS(2, false); break;
        case 5: ABS_PAIRS(2, true); break;
        case 8: ABS_PAIRS(4, false); break;
        case 9: ABS_PAIRS(4, true); break;
        case 16: if (nth == 512) ABS_PAIRS_T(8, false, 512); else ABS_PAIRS(8, false); break;
        default: if (nth == 512) ABS_PAIRS_T(8, true, 512); else ABS_PAIRS(8, true); break;
      }
#undef ABS_PAIRS
#undef ABS_PAIRS_T
    }
#undef ABS_GATHER_L
#undef ABS_GATHER
  }
  prof_end(p, ABS_STAGE_GRID, st);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

extern "C" abs_status abs_grid_sort_workspace(abs_plan_t p, int64_t nvis, size_t* set_bytes,
                                              size_t* work_bytes) {
  if (!p || nvis < 0 || nvis > 0x7fffffffLL) return ABS_ERR_INVALID;
  if (set_bytes) *set_bytes = set_bytes_of(p->n);
  if (work_bytes) *work_bytes = sort_layout(p->n, nvis).total;
  return ABS_OK;
}

extern "C" abs_status abs_grid_sort(abs_plan_t p, int64_t nvis, const double* uv, void* set,
                                    size_t set_bytes, void* work, size_t work_bytes, int32_t* perm,
                                    float* wsum, int64_t* kept, void* stream) {
  if (!p) return ABS_ERR_INVALID;
  if (!p->dev) return ABS_ERR_UNBOUND;
  if (nvis < 0 || nvis > 0x7fffffffLL || !set || !work || (nvis > 0 && (!uv || !perm)))
    return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(uv) | reinterpret_cast<uintptr_t>(set) |
       reinterpret_cast<uintptr_t>(work)) & 15)
    return ABS_ERR_INVALID;
  const SortWork sl = sort_layout(p->n, nvis);
  if (set_bytes < set_bytes_of(p->n) || work_bytes < sl.total) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wk = static_cast<char*>(work);
  GridScalars* sc = reinterpret_cast<GridScalars*>(wk + sl.sc);
  int* key = reinterpret_cast<int*>(wk + sl.key);
  int* rank = reinterpret_cast<int*>(wk + sl.rank);
  int* cnt = reinterpret_cast<int*>(wk + sl.cnt);
  int* tsum = reinterpret_cast<int*>(wk + sl.tiles);
  int* start = static_cast<int*>(set);
  const long long npair = pair_count(p->n), nkeys = 2 * npair;
  const int ntiles = (int)((nkeys + kScanTile - 1) / kScanTile);
  const double2* uvd = reinterpret_cast<const double2*>(uv);
  (void)hipGetLastError();
  grid_clear_kernel<<<1024, kBlock, 0, st>>>(cnt, nkeys, sc);
  const unsigned gv = (unsigned)std::min<long long>(8192, std::max<long long>(1, (nvis + kBlock - 1) / kBlock));
  if (nvis > 0) grid_prep_kernel<true><<<gv, kBlock, 0, st>>>(p->n, p->du, nvis, uvd, nullptr, key, rank, cnt, sc);
  scan_tiles_kernel<<<ntiles, kBlock, 0, st>>>(cnt, nkeys, start, tsum, sc);
  scan_sums_kernel<<<1, kBlock, 0, st>>>(tsum, ntiles, start, nkeys, sc, nullptr);
  scan_add_kernel<<<ntiles, kBlock, 0, st>>>(start, nkeys, tsum);
  grid_place_kernel<<<gv, kBlock, 0, st>>>(nvis, key, rank, start, nkeys, perm, reinterpret_cast<long long*>(kept));
  if (wsum) launch_keyed_pairs(p->n, 0, 0, 1, nullptr, start, (long long)nvis, nullptr, wsum, st);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

extern "C" abs_status abs_grid_permute(abs_plan_t p, int64_t nvis, int32_t batch, const int32_t* perm,
                                       int64_t ld, const float* vis, float* out, void* stream) {
  if (!p) return ABS_ERR_INVALID;
  if (nvis < 0 || nvis > 0x7fffffffLL || ld < 0 || ld > nvis || batch < 1) return ABS_ERR_INVALID;
  if (ld > 0 && (!perm || !vis || !out)) return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(vis) | reinterpret_cast<uintptr_t>(out)) & 7) return ABS_ERR_INVALID;
  if (ld == 0) return ABS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const long long total = ld * (long long)batch;
  const unsigned g = (unsigned)std::min<long long>(16384, (total + kBlock - 1) / kBlock);
  grid_permute_kernel<<<g, kBlock, 0, st>>>(nvis, batch, perm, ld, reinterpret_cast<const float2*>(vis),
                                            reinterpret_cast<float2*>(out));
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

extern "C" abs_status abs_grid_sorted(abs_plan_t p, const void* set, size_t set_bytes, int32_t batch,
                                      int64_t ld, const float* vis, float* grid, float* wsum, void* stream) {
  if (!p) return ABS_ERR_INVALID;
  if (!p->dev) return ABS_ERR_UNBOUND;
  if (batch < 1 || batch > p->max_batch * p->nchan || ld < 0 || ld > 0x7fffffffLL) return ABS_ERR_INVALID;
  if (!set || !grid || (ld > 0 && !vis)) return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(set) | reinterpret_cast<uintptr_t>(vis) |
       reinterpret_cast<uintptr_t>(grid)) & 15)
    return ABS_ERR_INVALID;
  if (set_bytes < set_bytes_of(p->n)) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int lpc = lanes_per_cell(batch);
  (void)hipGetLastError();
  prof_begin(p, ABS_STAGE_GRID, st);
  for (int b0 = 0; b0 < batch; b0 += 2 * lpc)
    launch_keyed_pairs(p->n, batch, b0, lpc, reinterpret_cast<const float2*>(vis), static_cast<const int*>(set),
                       (long long)ld, reinterpret_cast<float2*>(grid), b0 == 0 ? wsum : nullptr, st);
  prof_end(p, ABS_STAGE_GRID, st);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}
