// Ring fields by pruned 2-D FFT (Eqs. 10 and 11 of Gill et al. 2024).
//
// For ring m the field is F_m(x, y) = sum_{g in a_m} X(g) exp(-2 pi i (gx x + gy y) / n),
// real because X is Hermitian.  It is computed in two passes:
//   column pass: Z_m(gx, y) = sum_gy X_m(gx, gy) exp(-2 pi i gy y / n) for the
//                half-plane columns 0 <= gx <= h_m only (the other half follows from
//                Z_m(-gx, y) = conj Z_m(gx, y)); the ring mask and the Hermitian
//                symmetrisation with the weights are applied while loading;
//   row pass:    F_m(x, y) = sum_{|gx| <= h_m} Z_m(gx, y) exp(-2 pi i gx x / n) for two
//                rows at once: the complex FFT of Z(., y) + i Z(., y') has real part
//                F(., y) and imaginary part F(., y').
//
// Each length-n transform is a self-sorting (Stockham) FFT run by n/16 threads (two
// radix-16 butterflies per thread at n = 8192): radix-16 passes, then one radix-2, 4
// or 8 pass, with n a compile-time constant.  The first pass reads its inputs straight
// from memory (skipping the all-zero slabs of the pruned input), passes exchange data
// through a padded LDS buffer (one slot of padding every 16 elements keeps strided
// accesses off a single bank), and a thread keeps its butterflies and twiddles in
// registers.  The row pass writes the last pass's output in natural order straight to
// global memory; the column pass gathers its tile's outputs in LDS first.
//
// Before the column pass, the Hermitian part of the weighted grid is copied into a
// column-major array (herm_kernel) so that each column transform reads its input
// contiguously.
//
// Data fields D (Eq. 10) are computed in FP32.  Weight fields I (Eq. 11) are computed
// in FP64: their triple sums N_t can be tiny next to the size of the individual
// products (bins with few triangles), so FP32 field rounding would dominate N_t.
#include "fft_engine.h"

namespace abs_impl {

// Threads per row-pass workgroup: 8192-point rows use 512 (one radix-16 butterfly per
// thread, half the registers of two, so more waves fit a SIMD); others kBlock.  At 4096
// and 8192 points a workgroup runs one transform at a time, so the row pairs 2q and 2q + 1,
// whose inputs share each 32-byte group of the column pass's output, read it in turn and
// the group comes from memory twice (counters: 18.8 GB read for 9.8 GB written at
// 8192^2 x 8; the field stores below are non-temporal, which keeps most of those lines
// for the second read).  Measured alternatives: two transforms a workgroup read it once but ran
// slower at 8192 points (1024 threads: row pass 24.2 against 22.3 ms) and were mixed at 4096
// (512 threads: 9.17 against 8.97 ms at 8192^2 x 8, 2.30 against 2.40 ms at 4096^2 x 16);
// loading the odd pair's inputs with the even pair's took 30-60 more registers a lane.
constexpr int row_block(int log2n) { return log2n == 13 ? 512 : kBlock; }

// Row pass with the compile-time engine.  blockIdx.x = ring m * blocks per ring + block,
// each block covering G * iters row pairs; blockIdx.y = set.  FMAX records the largest
// |F| per (set, ring) for the FP16 split form.  HALF (even fields, the weights): only the
// row pairs up to row n/2 are transformed and the rows land in the half-plane layout,
// row 0 at 0, row n/2 at n, row r in 1 .. n/2 - 1 at hb + (r - 1) n; rstride is the
// values per ring (n^2, or the half-plane size).
template <typename R, int LOG2N, bool FMAX, bool HALF>
__global__ void __launch_bounds__(row_block(LOG2N))
rowpass_fixed_kernel(int iters, const BinDev* __restrict__ bins, const typename Cx<R>::T* __restrict__ tw,
                     const typename Cx<R>::T* __restrict__ Z, long long zset, R* __restrict__ F,
                     long long fset, long long rstride, int hb, unsigned* __restrict__ fmax_bits, int nb) {
  using T = typename Cx<R>::T;
  constexpr int RB = row_block(LOG2N);
  using FF = Fft<LOG2N, RB>;
  constexpr int n = FF::N;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // g = 0 spelled out for one transform a workgroup, so the row offsets stay scalar
  const int g = FF::G == 1 ? 0 : (int)threadIdx.x / FF::TG, t = threadIdx.x - g * FF::TG;
  T* buf = reinterpret_cast<T*>(lds_raw) + g * FF::L;
  // The twiddle tables sit in LDS after the FFT buffers: at most 5.4 KB (FP32) instead
  // of the full table (8 or 16 bytes per point), so more blocks fit a CU.
  TwiddlesSplit<R, LOG2N, RB> twr;
  twr.stage(tw, reinterpret_cast<T*>(lds_raw) + FF::G * FF::L, threadIdx.x, RB);
  __syncthreads();
  const int per_block = FF::G * iters;
  constexpr int npairs = HALF ? n / 4 + 1 : n / 2;   // HALF: rows 0 .. n/2 (+ n/2 + 1)
  const int nrb = (npairs + per_block - 1) / per_block;
  const int m = blockIdx.x / nrb, blk = blockIdx.x - m * nrb;
  const int set = blockIdx.y;
  const BinDev bin = bins[m];
  const int H = bin.h, cols = bin.cols;
  R* __restrict__ fs = F + (long long)set * fset + (long long)m * rstride;
  // offset of row r in the ring's output, -1 for a row the layout does not keep
  auto roff = [&](int r) -> long long {
    if constexpr (!HALF) return (long long)r * n;
    if (r == 0) return 0;
    if (r == n / 2) return n;
    if (r < n / 2) return (long long)hb + (long long)(r - 1) * n;
    return -1;
  };
  const T* __restrict__ zs = Z + (long long)set * zset + bin.zoff;
  R vmax = R(0);
  constexpr int S = n / 16;
  for (int it = 0; it < iters; ++it) {
    const int pair = blk * per_block + it * FF::G + g;
    const bool active = pair < npairs;
    const long long o0 = active ? roff(2 * pair) : -1, o1 = active ? roff(2 * pair + 1) : -1;
    if (cols == 0) {   // ring without lattice cells: its field is zero
      for (int k = t; k < n; k += FF::TG) {
        if (o0 >= 0) fs[o0 + k] = R(0);
        if (o1 >= 0) fs[o1 + k] = R(0);
      }
      continue;
    }
    // Input k of the row pair (ya, ya + 1): Z(gx, ya) + i Z(gx, ya + 1) at gx = k (k <= H)
    // or gx = k - n (k >= n - H), using Z(-gx, y) = conj Z(gx, y); zero elsewhere.  The
    // column pass stored both forms, P(gx) = Z(gx, ya) + i Z(gx, ya + 1) at zp[4 gx] and
    // Q(gx) = conj Z(gx, ya) + i conj Z(gx, ya + 1) next to it (blocks of 4 rows).  Slab r
    // of the first pass covers k in [r n/16, (r + 1) n/16); all-zero slabs are not read.
    const int pr = active ? pair : 0;
    const T* __restrict__ zp = zs + (long long)(pr >> 1) * 4 * cols + 2 * (pr & 1);
    auto in = [&](int k, int, int r) -> T {
      T x = Cx<R>::mk(R(0), R(0));
      if (active && (r * S <= H || (r + 1) * S - 1 >= n - H)) {
        if (k <= H) x = zp[4 * k];
        else if (k >= n - H) x = zp[4 * (n - k) + 1];
      }
      return x;
    };
    // One transform a workgroup (G = 1): `active` is the same for the whole workgroup, so an
    // inactive iteration is skipped (no barrier is left half taken) and, for full fields,
    // every row of an active pair is kept: the stores need no per-store test.
    constexpr bool UNIFORM = FF::G == 1 && !HALF;
    if (UNIFORM && !active) continue;
    R* __restrict__ row0 = fs + (o0 >= 0 ? o0 : 0);
    R* __restrict__ row1 = fs + (o1 >= 0 ? o1 : 0);
    // The fields are stored non-temporally: streamed past the L2, they no longer evict the
    // column-pass lines whose other half the next row pair reads (8192^2 x 8: reads 18.8 ->
    // 10.6 GB at 8192 points, 16.8 -> 11.6 GB at 4096; row pass 0.8 ms faster a step).
    auto out = [&](int k, int, int, T v) {
      if (UNIFORM || o0 >= 0) __builtin_nontemporal_store(v.x, &row0[k]);
      if (UNIFORM || o1 >= 0) __builtin_nontemporal_store(v.y, &row1[k]);
      if constexpr (FMAX)
        if (active) vmax = fmax(vmax, fmax(fabs(v.x), fabs(v.y)));
    };
    fft_sync<FF::WAVE>();   // the previous transform's last reads are done
    // The thread index is hidden from loop-invariant code motion: the twiddle and LDS
    // offsets derived from it are recomputed per transform instead of being held in
    // registers across the loop.
    int tl = t;
    asm volatile("" : "+v"(tl));
    __builtin_assume(tl >= 0 && tl < FF::TG);   // its range survives the hiding
    fft_passes<R, LOG2N, 0, RB>(buf, tl, tw, twr, in, out);
  }
  if constexpr (FMAX) {
    float v = (float)vmax;
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    // non-negative floats order like their bit patterns
    if ((threadIdx.x & 63) == 0) atomicMax(&fmax_bits[(long long)set * nb + m], __float_as_uint(v));
  }
}

// Weight W(g) of one cell for the plan's weight mode (Sec. 2, after Eq. 10).
template <typename R>
__device__ __forceinline__ R weight_of(const float* __restrict__ w, int wmode, long long idx) {
  if (wmode == ABS_W_UNIT) return R(1);
  const R v = (R)w[idx];
  if (wmode == ABS_W_INV_COUNT) return v >= R(0.5) ? R(1) / v : R(0);
  return v;
}

__device__ __forceinline__ float2 load_vis(const float2* __restrict__ g, long long idx) { return g[idx]; }
__device__ __forceinline__ float2 load_vis(const double2* __restrict__ g, long long idx) {
  const double2 v = g[idx];
  return make_float2((float)v.x, (float)v.y);
}

// Hermitian part of the weighted grid on the half-plane columns 0 <= gx <= hm and rows
// |gy| <= hm (hm: the largest |gx| of any ring cell), stored column by column as
// xc[set][gx][gy + hm] with column length lc = 2 hm + 1, so that the column pass reads
// each column contiguously.  DATA: X(g) = (W(g) V(g) + conj(W(-g) V(-g))) / 2 (FP32);
// otherwise Y(g) = (W(g) + W(-g)) / 2 (FP64, real).  The grid is read by rows (coalesced
// in gx) and written by columns through an LDS tile of kHx x kHy cells.
constexpr int kHx = 64, kHy = 16;
template <bool DATA> struct HermT;
template <> struct HermT<true> { using T = float2; };
template <> struct HermT<false> { using T = double; };

//
// Each block also records, for the empty-triplet rule of the finaliser, the smallest
// non-zero Y(g) over its cells that lie in some ring (lo2 <= |g|^2 < hi2: the rings are
// contiguous), as a running minimum of FP64 bit patterns in wmin[set] (non-negative
// doubles order like their bits; the caller sets it to +inf first).  Y is even, so the
// half plane gx >= 0 holds every value.
//
// Complex input (spg = 4 data sets per grid): set 4 b + v of grid b holds, for v = 0 .. 3,
// H, G, H + G and H - G, where H is the Hermitian part above and G = (W V(g) - conj(W V(-g)))
// / (2 i) the anti-Hermitian part divided by i (Hermitian as well), so W V = H + i G and
// every set's field is real (abs_estimate_complex combines their triple sums).
template <bool DATA, typename GT>
__global__ void __launch_bounds__(kBlock)
herm_kernel(const GT* __restrict__ grids, const float* __restrict__ w, int w_batched, int spg, int wmode,
            int n, int hm, int lc, double lo2, double hi2, typename HermT<DATA>::T* __restrict__ xc,
            unsigned long long* __restrict__ wmin, WeightMod mod) {
  using OT = typename HermT<DATA>::T;
  __shared__ OT tile[kHy][kHx + 1];
  __shared__ double wred[kBlock / 64];
  const int set = blockIdx.z;
  const int gi = set / spg, part = set - gi * spg;   // grid and, for complex input, variant
  const int gx0 = blockIdx.x * kHx, gy0 = blockIdx.y * kHy - hm;
  const long long nn = (long long)n * n;
  const GT* __restrict__ gs = DATA ? grids + (long long)gi * nn : nullptr;
  const float* __restrict__ ws = (w && w_batched) ? w + (long long)gi * nn : w;
  const int tx = threadIdx.x & (kHx - 1), ty = threadIdx.x / kHx;
  double ymin = __builtin_inf();
  for (int yy = ty; yy < kHy; yy += kBlock / kHx) {
    const int gx = gx0 + tx, gy = gy0 + yy;
    OT v{};
    if (gx <= hm && gy <= hm) {
      const int iy = gy < 0 ? gy + n : gy;
      const int my = gy > 0 ? n - gy : -gy, mx = gx > 0 ? n - gx : 0;
      const long long i0 = (long long)iy * n + gx, i1 = (long long)my * n + mx;
      double y = 0.5 * (weight_of<double>(ws, wmode, i0) + weight_of<double>(ws, wmode, i1));
      if (!DATA && mod.c) {
        const double cs = 0.5 * ((double)mod.c[i0] + (double)mod.c[i1]);
        const double cmax = (double)__uint_as_float(*mod.cmax_bits);
        if (cmax > 0.0) y *= 1.0 + mod.sgn * cs / cmax;
      }
      const double r2 = (double)((long long)gx * gx + (long long)gy * gy);
      if (r2 >= lo2 && r2 < hi2 && y != 0.0) ymin = fmin(ymin, fabs(y));
      if constexpr (DATA) {
        const float w0 = weight_of<float>(ws, wmode, i0), w1 = weight_of<float>(ws, wmode, i1);
        const float2 a = load_vis(gs, i0), b = load_vis(gs, i1);
        const float2 h = make_float2(0.5f * (w0 * a.x + w1 * b.x), 0.5f * (w0 * a.y - w1 * b.y));
        if (spg == 1 || part == 0) {
          v = h;
        } else {
          const float2 q = make_float2(0.5f * (w0 * a.y + w1 * b.y), -0.5f * (w0 * a.x - w1 * b.x));
          v = part == 1 ? q : part == 2 ? make_float2(h.x + q.x, h.y + q.y) : make_float2(h.x - q.x, h.y - q.y);
        }
      } else {
        v = y;
      }
    }
    tile[yy][tx] = v;
  }
  for (int o = 32; o > 0; o >>= 1) ymin = fmin(ymin, __shfl_xor(ymin, o));
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = ymin;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wred[0];
    for (int k = 1; k < kBlock / 64; ++k) m = fmin(m, wred[k]);
    if (m < __builtin_inf()) atomicMin(&wmin[set], (unsigned long long)__double_as_longlong(m));
  }
  for (int e = threadIdx.x; e < kHx * kHy; e += kBlock) {
    const int c = e / kHy, yy = e - c * kHy;
    const int gx = gx0 + c, gy = gy0 + yy;
    if (gx <= hm && gy <= hm) xc[((long long)set * (hm + 1) + gx) * lc + gy + hm] = tile[yy][c];
  }
}

// Column pass: one transform per (ring, column gx), Z_m(gx, y) = sum over the ring's
// cells in column gx of X(gx, gy) exp(-2 pi i gy y / n).  A block takes `tpb` column
// tiles (G columns of one ring each) in turn; blockIdx.y = set.  Input k of a column is
// the cell gy = k (k <= H) or gy = k - n (k >= n - H) when it lies in the ring, read
// from the column-major Hermitian part.  Z_m is stored in blocks of 4 rows,
// Z_m[y / 4][gx][y % 4] (zidx), so that the tile's outputs, gathered in LDS, leave as
// runs of 4 ncols consecutive elements (whole 128-byte lines for 4 FP32 columns) and
// the row pass reads each input of a row pair with one load.
// Column-pass twiddles: held in registers when a thread needs few (FP32), otherwise the
// two-level LDS table.
template <typename R, int LOG2N>
constexpr bool col_tw_reg() { return sizeof(R) == 4 && Fft<LOG2N, col_engine(LOG2N, true)>::NTW <= 32; }

// Transforms per column-pass workgroup (the columns of one tile).
template <typename R, int LOG2N>
constexpr int col_transforms() { return col_block(LOG2N, sizeof(R) == 4) / Fft<LOG2N, col_engine(LOG2N, sizeof(R) == 4)>::TG; }

template <typename R, int LOG2N>
__global__ void __launch_bounds__(col_block(LOG2N, sizeof(R) == 4))
colpass_fixed_kernel(const typename HermT<sizeof(R) == 4>::T* __restrict__ xc, int hm, int lc,
                     const ColTile* __restrict__ tiles, int ntiles, int tpb,
                     const BinDev* __restrict__ bins, const typename Cx<R>::T* __restrict__ tw,
                     typename Cx<R>::T* __restrict__ Z, long long zset) {
  using T = typename Cx<R>::T;
  constexpr int CB = col_block(LOG2N, sizeof(R) == 4), EB = col_engine(LOG2N, sizeof(R) == 4);
  using FF = Fft<LOG2N, EB>;
  constexpr int CG = col_transforms<R, LOG2N>();   // transforms (columns) per workgroup
  constexpr int n = FF::N, S = n / 16;
  constexpr bool DATA = sizeof(R) == 4;
  constexpr bool REG = col_tw_reg<R, LOG2N>();
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int g = threadIdx.x / FF::TG, t = threadIdx.x - g * FF::TG;
  T* buf = reinterpret_cast<T*>(lds_raw) + g * FF::L;
  const int set = blockIdx.y;
  using TW = std::conditional_t<REG, Twiddles<R, LOG2N, true, EB>, TwiddlesSplit<R, LOG2N, EB>>;
  TW twr;
  if constexpr (REG) twr.load(tw, t);
  else twr.stage(tw, reinterpret_cast<T*>(lds_raw) + CG * FF::L, threadIdx.x, CB);   // the loop's first barrier publishes it
  // consecutive tiles (neighbouring columns of a ring, whose outputs share cache lines) in
  // runs on one XCD
  const int bx = (int)xcd_block(blockIdx.x);
  for (int it = 0; it < tpb; ++it) {
    const int ti = bx * tpb + it;
    if (ti >= ntiles) break;   // the same for the whole block
    const ColTile tile = tiles[ti];
    const BinDev bin = bins[tile.m];
    const bool active = g < tile.ncols;
    const int gx = tile.gx0 + (active ? g : 0);
    const int H = bin.h, cols = bin.cols;
    const int d2lo = bin.d2lo, d2hi = bin.d2hi;
    // column gx of the Hermitian part: cell gy at col0[gy + hm] (a non-negative 32-bit index)
    const auto* __restrict__ col0 = xc + ((long long)set * (hm + 1) + gx) * lc;
    auto in = [&](int k, int, int r) -> T {
      T x = Cx<R>::mk(R(0), R(0));
      if (active && (r * S <= H || (r + 1) * S - 1 >= n - H)) {
        const int gy = k <= H ? k : k - n;
        if (k <= H || k >= n - H) {
          // |g| <= n/2 in each component: 24-bit products (full-rate multiplies), 32-bit sum
          const int d2 = __mul24(gx, gx) + __mul24(gy, gy);
          if (d2 >= d2lo && d2 < d2hi) {
            const unsigned iy = (unsigned)(gy + hm);
            if constexpr (DATA) x = col0[iy];
            else x = Cx<R>::mk(col0[iy], R(0));
          }
        }
      }
      return x;
    };
    // outputs of the block's transforms gathered as stage[y * CG + g] (over the FFT
    // buffers, once every transform has finished reading them)
    T* stage = reinterpret_cast<T*>(lds_raw);
    constexpr int PL = FF::NPASS - 1, NBL = FF::nb(PL), RPL = 1 << FF::lrp(PL), NSL = 1 << (4 * PL);
    T res[NBL][RPL];   // output (j, q) of the last pass is element t + TG j + q NSL
    auto out = [&](int, int j, int q, T v) { res[j][q] = v; };
    __syncthreads();   // the previous tile's stage has been written out
    int tl = t;   // hidden from loop-invariant code motion, as in the row pass
    asm volatile("" : "+v"(tl));
    fft_passes<R, LOG2N, 0, EB>(buf, tl, tw, twr, in, out);
    __syncthreads();   // every transform has read its buffer
#pragma unroll
    for (int j = 0; j < NBL; ++j)
#pragma unroll
      for (int q = 0; q < RPL; ++q) stage[(t + FF::TG * j + q * NSL) * CG + g] = res[j][q];
    __syncthreads();
    // row pair (2p, 2p + 1) of column gx is stored as P = a + i b and Q = conj a + i conj b
    // (a, b the two rows): the row pass takes P for gx >= 0 and Q for the mirrored
    // column -gx, one value per input
    const int nc = tile.ncols, run = 4 * nc;
    T* __restrict__ zs = Z + (long long)set * zset + bin.zoff + 4LL * tile.gx0;
    for (int e = threadIdx.x; e < n * nc; e += CB) {
      const int yb = e / run, rem = e - yb * run, c = rem >> 2, yi = rem & 3;
      const int y0 = 4 * yb + (yi & 2);
      const T a = stage[y0 * CG + c], b = stage[(y0 + 1) * CG + c];
      zs[(long long)yb * 4 * cols + rem] =
          (yi & 1) ? Cx<R>::mk(a.x + b.y, -a.y + b.x) : Cx<R>::mk(a.x - b.y, a.y + b.x);
    }
  }
}

namespace {
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
// Row pairs (per transform) a row-pass block walks in turn, and column tiles a column-pass
// block takes: measured per size (1024^2 x 16: 2 iterations 316 against 326 us with 4, one
// tile 70 against 75 us with 2; 4096^2 x 16: 8 iterations 8.65 against 8.92 ms with 4, two
// tiles 2.0 against 2.2 ms with 1; 8192^2 x 4: 8 iterations 20.4 ms, 2 iterations 21.6 ms);
// 2048 keeps 4 and 2.
constexpr int row_iters(int log2n) { return log2n <= 10 ? 2 : log2n >= 12 ? 8 : 4; }
constexpr int col_tiles_per_block(int log2n) { return log2n <= 10 ? 1 : 2; }
}  // namespace

template <bool DATA, typename GT>
hipError_t launch_herm(const abs_plan_s* p, const GT* grids, const float* w, int w_batched, int nsets,
                       typename HermT<DATA>::T* xc, unsigned long long* wmin, hipStream_t st,
                       const WeightMod* mod = nullptr, int spg = 1) {
  const int hm = p->hmax, lc = 2 * p->hmax + 1;
  const dim3 grid((unsigned)((hm + kHx) / kHx), (unsigned)((lc + kHy - 1) / kHy), (unsigned)nsets);
  herm_kernel<DATA, GT><<<grid, kBlock, 0, st>>>(grids, w, w_batched, spg, p->wmode, p->n, hm, lc, p->lo2[0],
                                                 p->hi2[p->nb - 1], xc, wmin, mod ? *mod : WeightMod{});
  return hipGetLastError();
}

template <typename R, int LOG2N>
hipError_t launch_colpass_n(const abs_plan_s* p, int nsets, const typename HermT<sizeof(R) == 4>::T* xc,
                            typename Cx<R>::T* Z, long long zset, const typename Cx<R>::T* tw,
                            hipStream_t st) {
  constexpr bool F32 = sizeof(R) == 4;
  constexpr int CB = col_block(LOG2N, F32), EB = col_engine(LOG2N, F32);
  using FF = Fft<LOG2N, EB>;
  const char* base = static_cast<const char*>(p->dev);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const ColTile* tiles = reinterpret_cast<const ColTile*>(base + (F32 ? p->dl.tiles : p->dl.tiles64));
  const int ntiles = (int)(F32 ? p->tiles.size() : p->tiles64.size());
  if (ntiles == 0) return hipSuccess;
  if ((F32 ? p->ct : p->ct64) != col_transforms<R, LOG2N>()) return hipErrorInvalidValue;
  constexpr int tpb = col_tiles_per_block(LOG2N);
  const dim3 grid(xcd_grid((ntiles + tpb - 1) / tpb), (unsigned)nsets);
  const size_t lds = (size_t)col_transforms<R, LOG2N>() * FF::L * sizeof(typename Cx<R>::T) +
                     (col_tw_reg<R, LOG2N>() ? 0 : TwiddlesSplit<R, LOG2N, EB>::ENTRIES * sizeof(typename Cx<R>::T));
  auto k = colpass_fixed_kernel<R, LOG2N>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  // the Hermitian part read is the one formed for the plan, or for its parent (level
  // plans), whose half extent xc_hm covers the plan's rings
  k<<<grid, CB, lds, st>>>(xc, p->xc_hm, 2 * p->xc_hm + 1, tiles, ntiles, tpb, bins, tw,
                           Z, zset);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_colpass(const abs_plan_s* p, int nsets, const typename HermT<sizeof(R) == 4>::T* xc,
                          typename Cx<R>::T* Z, long long zset, const typename Cx<R>::T* tw,
                          hipStream_t st) {
  switch (p->log2n) {
#define ABS_COL_CASE(L) \
  case L: return launch_colpass_n<R, L>(p, nsets, xc, Z, zset, tw, st);
    ABS_COL_CASE(4) ABS_COL_CASE(5) ABS_COL_CASE(6) ABS_COL_CASE(7) ABS_COL_CASE(8)
    ABS_COL_CASE(9) ABS_COL_CASE(10) ABS_COL_CASE(11) ABS_COL_CASE(12) ABS_COL_CASE(13)
#undef ABS_COL_CASE
    default: return hipErrorInvalidValue;
  }
}

// Hermitian part of a batch of grids (FP32 complex) or of the weights (FP64 real) for the
// plan's rings, and the smallest non-zero ring-cell weight of each set.
hipError_t launch_herm_data(const abs_plan_s* p, const void* grids, int dtype, const float* w, int w_batched,
                            int batch, void* xc, unsigned long long* wmin, hipStream_t st, int spg) {
  float2* x = static_cast<float2*>(xc);
  return dtype == ABS_C128
             ? launch_herm<true, double2>(p, static_cast<const double2*>(grids), w, w_batched, batch, x, wmin, st,
                                          nullptr, spg)
             : launch_herm<true, float2>(p, static_cast<const float2*>(grids), w, w_batched, batch, x, wmin, st,
                                         nullptr, spg);
}

hipError_t launch_herm_weight(const abs_plan_s* p, const float* w, int w_batched, int nsets, void* xc,
                              unsigned long long* wmin, hipStream_t st, const WeightMod* mod) {
  return launch_herm<false, float2>(p, nullptr, w, w_batched, nsets, static_cast<double*>(xc), wmin, st, mod);
}

// Ring-masked column FFTs of plan p (a plan, or one of its levels) from a Hermitian part.
hipError_t launch_colpass_f32(const abs_plan_s* p, int nsets, const void* xc, float2* Z, long long zset,
                              hipStream_t st) {
  const float2* tw = reinterpret_cast<const float2*>(static_cast<const char*>(p->dev) + p->dl.tw);
  return launch_colpass<float>(p, nsets, static_cast<const float2*>(xc), Z, zset, tw, st);
}

hipError_t launch_colpass_f64(const abs_plan_s* p, int nsets, const void* xc, double2* Z, long long zset,
                              hipStream_t st) {
  const double2* tw = reinterpret_cast<const double2*>(static_cast<const char*>(p->dev) + p->dl.tw64);
  return launch_colpass<double>(p, nsets, static_cast<const double*>(xc), Z, zset, tw, st);
}

template <typename R, int LOG2N>
hipError_t launch_rowpass_n(const abs_plan_s* p, int nsets, const typename Cx<R>::T* Z, long long zset,
                            R* F, long long fset, unsigned* fmax_bits, const BinDev* bins,
                            const typename Cx<R>::T* tw, hipStream_t st) {
  constexpr int RB = row_block(LOG2N);
  using FF = Fft<LOG2N, RB>;
  // FP64 rows are the weight fields: even, half plane
  constexpr bool HALF = sizeof(R) == 8;
  constexpr int npairs = HALF ? FF::N / 4 + 1 : FF::N / 2;
  const long long rstride = HALF ? p->npix64 : (long long)FF::N * FF::N;
  const int hb = HALF ? p->pix_per_block64 : 0;
  const int iters = std::max(1, std::min(row_iters(LOG2N), npairs / FF::G));
  const int per_block = FF::G * iters;
  const int nrb = (npairs + per_block - 1) / per_block;
  const dim3 grid((unsigned)(p->nb * nrb), (unsigned)nsets);
  using T = typename Cx<R>::T;
  const size_t lds = (size_t)(FF::G * FF::L + TwiddlesSplit<R, LOG2N, RB>::ENTRIES) * sizeof(T);
  hipError_t e;
  if constexpr (sizeof(R) == 4) {
    if (fmax_bits) {   // FP16 split form: largest |F| per (set, ring)
      auto k = rowpass_fixed_kernel<R, LOG2N, true, false>;
      if ((e = allow_lds(k, lds)) != hipSuccess) return e;
      k<<<grid, RB, lds, st>>>(iters, bins, tw, Z, zset, F, fset, rstride, hb, fmax_bits, p->nb);
      return hipGetLastError();
    }
  }
  {
    auto k = rowpass_fixed_kernel<R, LOG2N, false, HALF>;
    if ((e = allow_lds(k, lds)) != hipSuccess) return e;
    k<<<grid, RB, lds, st>>>(iters, bins, tw, Z, zset, F, fset, rstride, hb, nullptr, p->nb);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_rowpass(const abs_plan_s* p, int nsets, const typename Cx<R>::T* Z,
                          long long zset, R* F, long long fset, unsigned* fmax_bits, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const bool f64 = sizeof(R) == 8;
  const auto* tw = reinterpret_cast<const typename Cx<R>::T*>(base + (f64 ? p->dl.tw64 : p->dl.tw));
  switch (p->log2n) {
#define ABS_ROW_CASE(L) \
  case L: return launch_rowpass_n<R, L>(p, nsets, Z, zset, F, fset, fmax_bits, bins, tw, st);
    ABS_ROW_CASE(4) ABS_ROW_CASE(5) ABS_ROW_CASE(6) ABS_ROW_CASE(7) ABS_ROW_CASE(8)
    ABS_ROW_CASE(9) ABS_ROW_CASE(10) ABS_ROW_CASE(11) ABS_ROW_CASE(12) ABS_ROW_CASE(13)
#undef ABS_ROW_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rowpass_f32(const abs_plan_s* p, int nsets, const float2* Z, long long zset,
                              float* F, long long fset, unsigned* fmax_bits, hipStream_t st) {
  return launch_rowpass<float>(p, nsets, Z, zset, F, fset, fmax_bits, st);
}
// Zeros of the half-plane weight layout: [2n, hb) after rows 0 and n/2, and the tail
// after rows 1 .. n/2 - 1, for every (set, ring); blockIdx.x = set * nb + ring.
__global__ void __launch_bounds__(kBlock)
half_pad_kernel(double* __restrict__ F, long long fset, long long rstride, int n, int hb) {
  const int set = blockIdx.y;
  double* f = F + (long long)set * fset + (long long)blockIdx.x * rstride;
  for (long long i = 2ll * n + threadIdx.x; i < hb; i += kBlock) f[i] = 0.0;
  for (long long i = hb + (long long)(n / 2 - 1) * n + threadIdx.x; i < rstride; i += kBlock) f[i] = 0.0;
}

hipError_t launch_rowpass_f64(const abs_plan_s* p, int nsets, const double2* Z, long long zset,
                              double* F, long long fset, hipStream_t st) {
  half_pad_kernel<<<dim3((unsigned)p->nb, (unsigned)nsets), kBlock, 0, st>>>(F, fset, p->npix64, p->n,
                                                                             p->pix_per_block64);
  return launch_rowpass<double>(p, nsets, Z, zset, F, fset, nullptr, st);
}

}  // namespace abs_impl
