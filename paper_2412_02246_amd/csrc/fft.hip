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
// or 8 pass.  The block first stages the (mostly zero) inputs of its transforms in a
// padded LDS buffer (one slot of padding every 16 elements keeps strided accesses off
// a single bank); a thread keeps its butterflies in registers between passes, and the
// last pass writes the output in natural order straight to global memory.
//
// Data fields D (Eq. 10) are computed in FP32.  Weight fields I (Eq. 11) are computed
// in FP64: their triple sums N_t can be tiny next to the size of the individual
// products (bins with few triangles), so FP32 field rounding would dominate N_t.
#include "abs_internal.h"

namespace abs_impl {

template <typename R> struct Cx;
template <> struct Cx<float> {
  using T = float2;
  static __device__ __forceinline__ T mk(float a, float b) { return make_float2(a, b); }
};
template <> struct Cx<double> {
  using T = double2;
  static __device__ __forceinline__ T mk(double a, double b) { return make_double2(a, b); }
};

template <typename T> __device__ __forceinline__ T cadd(T a, T b) { T r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { T r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a * (-i)
template <typename T> __device__ __forceinline__ T cmi(T a) { T r; r.x = a.y; r.y = -a.x; return r; }

// a * exp(-2 pi i M / 16)
template <typename R, int M>
__device__ __forceinline__ typename Cx<R>::T w16mul(typename Cx<R>::T a) {
  if constexpr (M == 0) return a;
  else if constexpr (M == 4) return cmi(a);
  else if constexpr (M == 8) return Cx<R>::mk(-a.x, -a.y);
  else {
    constexpr double c[10] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977, 0.0,
                              -0.38268343236508977, -0.70710678118654752, -0.92387953251128674, -1.0,
                              -0.92387953251128674};
    constexpr double s[10] = {0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
                              -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
                              0.0, 0.38268343236508977};
    return cmul(a, Cx<R>::mk((R)c[M], (R)s[M]));
  }
}

// Forward DFT-4 in place on a[0], a[s], a[2s], a[3s], natural order.
template <typename T>
__device__ __forceinline__ void dft4(T* a, int s) {
  const T s02 = cadd(a[0], a[2 * s]), d02 = csub(a[0], a[2 * s]);
  const T s13 = cadd(a[s], a[3 * s]), d13 = csub(a[s], a[3 * s]);
  a[0] = cadd(s02, s13);
  a[2 * s] = csub(s02, s13);
  a[s] = cadd(d02, cmi(d13));
  a[3 * s] = csub(d02, cmi(d13));
}

// Forward DFT of RP points in registers v[0 .. RP), natural order in and out.
template <typename R, int RP>
__device__ __forceinline__ void dft(typename Cx<R>::T* v) {
  using T = typename Cx<R>::T;
  if constexpr (RP == 2) {
    const T a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else if constexpr (RP == 4) {
    dft4(v, 1);
  } else if constexpr (RP == 8) {
    // i = 2 i2 + i1: DFT-4 over i2, twiddle exp(-2 pi i i1 k1 / 8), DFT-2 over i1
    dft4(v, 2);
    dft4(v + 1, 2);
    v[3] = w16mul<R, 2>(v[3]);
    v[5] = w16mul<R, 4>(v[5]);
    v[7] = w16mul<R, 6>(v[7]);
    T o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
      o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = o[q];
  } else {
    // i = 4 i2 + i1: DFT-4 over i2, twiddle exp(-2 pi i i1 k1 / 16), DFT-4 over i1
#pragma unroll
    for (int i1 = 0; i1 < 4; ++i1) dft4(v + i1, 4);
    v[5] = w16mul<R, 1>(v[5]);
    v[6] = w16mul<R, 2>(v[6]);
    v[7] = w16mul<R, 3>(v[7]);
    v[9] = w16mul<R, 2>(v[9]);
    v[10] = w16mul<R, 4>(v[10]);
    v[11] = w16mul<R, 6>(v[11]);
    v[13] = w16mul<R, 3>(v[13]);
    v[14] = w16mul<R, 6>(v[14]);
    v[15] = w16mul<R, 9>(v[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v + 4 * k1, 1);
    T o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = o[q];
  }
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// One Stockham pass of radix RP over a length-n transform held by Tg threads; thread t
// owns butterflies b = t + Tg * j, j < 16 U / RP.  Input comes from buf (padded); LAST
// writes out(k, value), otherwise the output goes back to buf.
template <typename R, int RP, int U, bool FIRST, bool LAST, class Out>
__device__ __forceinline__ void stockham_pass(typename Cx<R>::T* buf, int n, int log2n, int lns,
                                              int t, int Tg, const typename Cx<R>::T* __restrict__ tw,
                                              Out& out) {
  using T = typename Cx<R>::T;
  constexpr int NB = 16 * U / RP;
  constexpr int LRP = RP == 16 ? 4 : RP == 8 ? 3 : RP == 4 ? 2 : 1;
  const int stride = n >> LRP;       // n / RP
  const int Ns = 1 << lns;
  T v[NB][RP];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int b = t + Tg * j;
#pragma unroll
    for (int r = 0; r < RP; ++r) v[j][r] = buf[lpad(b + r * stride)];
  }
  __syncthreads();  // every read of this pass precedes every write
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int b = t + Tg * j;
    const int m = b & (Ns - 1);
    if (!FIRST && m != 0) {
      const int sh = log2n - lns - LRP;   // twiddle exp(-2 pi i r m / (Ns RP)) = tw[(r m) << sh]
#pragma unroll
      for (int r = 1; r < RP; ++r) v[j][r] = cmul(v[j][r], tw[(r * m) << sh]);
    }
    dft<R, RP>(v[j]);
    const int idxD = ((b >> lns) << (lns + LRP)) + m;
#pragma unroll
    for (int q = 0; q < RP; ++q) {
      const int k = idxD + q * Ns;
      if constexpr (LAST) out(k, v[j][q]);
      else buf[lpad(k)] = v[j][q];
    }
  }
  if constexpr (!LAST) __syncthreads();
}

// Length-n forward FFT (16 <= n <= 8192) of the sequence staged in buf (padded, natural
// order), by Tg = n / (16 U) threads, output in natural order through out(k, value);
// every thread of the block must call it (it synchronises the block).
template <typename R, int U, class Out>
__device__ void stockham_fft(typename Cx<R>::T* buf, int n, int log2n, int t, int Tg,
                             const typename Cx<R>::T* __restrict__ tw, Out out) {
  const int np16 = log2n >> 2, lrest = log2n & 3;
  const int npass = np16 + (lrest ? 1 : 0);
  int lns = 0;
  for (int p = 0; p < npass; ++p) {
    const bool first = p == 0, last = p == npass - 1;
    const int lr = p < np16 ? 4 : lrest;
    if (lr == 4) {
      if (first && last) stockham_pass<R, 16, U, true, true>(buf, n, log2n, lns, t, Tg, tw, out);
      else if (first) stockham_pass<R, 16, U, true, false>(buf, n, log2n, lns, t, Tg, tw, out);
      else if (last) stockham_pass<R, 16, U, false, true>(buf, n, log2n, lns, t, Tg, tw, out);
      else stockham_pass<R, 16, U, false, false>(buf, n, log2n, lns, t, Tg, tw, out);
    } else if (lr == 3) {
      stockham_pass<R, 8, U, false, true>(buf, n, log2n, lns, t, Tg, tw, out);
    } else if (lr == 2) {
      stockham_pass<R, 4, U, false, true>(buf, n, log2n, lns, t, Tg, tw, out);
    } else {
      stockham_pass<R, 2, U, false, true>(buf, n, log2n, lns, t, Tg, tw, out);
    }
    lns += lr;
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

// FFT geometry of a block of kBlock threads: G transforms at once, Tg threads each.
struct FftGeom {
  int G, Tg;
};
__host__ __device__ inline FftGeom fft_geom(int n) {
  const int per = n >= 16 ? n / 16 : 1;          // butterflies of a radix-16 pass
  const int Tg = per < kBlock ? per : kBlock;
  return {kBlock / Tg, Tg};
}
__host__ __device__ inline int fft_lds_elems(int n) { return n + n / 16; }

// Column pass: one transform per (ring, column gx); blockIdx.x = column tile (G columns
// of one ring), blockIdx.y = set.  DATA: stage X = (W V(g) + conj(W V(-g)))/2 of grid
// `set`; otherwise Y = (W(g) + W(-g))/2 of weight array `set`.
template <typename R, int U, bool DATA, typename GT>
__global__ void __launch_bounds__(kBlock)
colpass_kernel(const GT* __restrict__ grids, const float* __restrict__ w, int w_batched, int wmode,
               int n, int log2n, const ColTile* __restrict__ tiles, const BinDev* __restrict__ bins,
               const typename Cx<R>::T* __restrict__ tw, typename Cx<R>::T* __restrict__ Z,
               long long zset) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const FftGeom geo = fft_geom(n);
  const int g = threadIdx.x / geo.Tg, t = threadIdx.x - g * geo.Tg;
  T* buf = reinterpret_cast<T*>(lds_raw) + g * fft_lds_elems(n);
  const ColTile tile = tiles[blockIdx.x];
  const int set = blockIdx.y;
  const long long nn = (long long)n * n;
  const float* __restrict__ ws = (w && w_batched) ? w + (long long)set * nn : w;
  const BinDev bin = bins[tile.m];
  const bool active = g < tile.ncols;
  const int gx = tile.gx0 + (active ? g : 0);
  const int H = bin.h;
  (void)gx;
  const double lo2 = bin.lo2, hi2 = bin.hi2;
  const GT* __restrict__ gs = DATA ? grids + (long long)set * nn : nullptr;
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int L = fft_lds_elems(n);
  for (int q = threadIdx.x; q < geo.G * L; q += blockDim.x) lds[q] = Cx<R>::mk(R(0), R(0));
  __syncthreads();
  // stage the ring cells of the tile's columns: gy in [-H, H], column-fastest for
  // coalesced reads of the grid rows
  const int nc = tile.ncols, nrows = 2 * H + 1;
  for (int q = threadIdx.x; q < nrows * nc; q += blockDim.x) {
    const int r = q / nc, c = q - r * nc;
    const int gy = r - H, cx = tile.gx0 + c;
    const double d2 = (double)((long long)cx * cx + (long long)gy * gy);
    if (!(d2 >= lo2 && d2 < hi2)) continue;
    const int iy = gy < 0 ? gy + n : gy;
    const int my = gy > 0 ? n - gy : -gy, mx = cx > 0 ? n - cx : 0;
    const long long i0 = (long long)iy * n + cx, i1 = (long long)my * n + mx;
    const R w0 = weight_of<R>(ws, wmode, i0), w1 = weight_of<R>(ws, wmode, i1);
    T v;
    if constexpr (DATA) {
      const float2 a = load_vis(gs, i0), b = load_vis(gs, i1);
      v = Cx<R>::mk(R(0.5) * (w0 * a.x + w1 * b.x), R(0.5) * (w0 * a.y - w1 * b.y));
    } else {
      v = Cx<R>::mk(R(0.5) * (w0 + w1), R(0));
    }
    lds[c * L + lpad(iy)] = v;
  }
  __syncthreads();
  T* __restrict__ zs = Z + (long long)set * zset + bin.zoff;
  const int cols = bin.cols;
  auto out = [&](int k, T v) {
    if (active) zs[(long long)k * cols + gx] = v;
  };
  stockham_fft<R, U>(buf, n, log2n, t, geo.Tg, tw, out);
}

// Row pass: one transform per (ring, row pair); blockIdx.x = ring m * blocks per ring +
// block, each block covering G * iters row pairs; blockIdx.y = set.
template <typename R, int U>
__global__ void __launch_bounds__(kBlock)
rowpass_kernel(int n, int log2n, int iters, const BinDev* __restrict__ bins,
               const typename Cx<R>::T* __restrict__ tw, const typename Cx<R>::T* __restrict__ Z,
               long long zset, R* __restrict__ F, long long fset, unsigned* __restrict__ fmax_bits,
               int nb) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const FftGeom geo = fft_geom(n);
  const int g = threadIdx.x / geo.Tg, t = threadIdx.x - g * geo.Tg;
  T* buf = reinterpret_cast<T*>(lds_raw) + g * fft_lds_elems(n);
  const int per_block = geo.G * iters;
  const int nrb = (n / 2 + per_block - 1) / per_block;
  const int m = blockIdx.x / nrb, blk = blockIdx.x - m * nrb;
  const int set = blockIdx.y;
  const BinDev bin = bins[m];
  const int H = bin.h, cols = bin.cols;
  const long long nn = (long long)n * n;
  R* __restrict__ fs = F + (long long)set * fset + (long long)m * nn;
  const T* __restrict__ zs = Z + (long long)set * zset + bin.zoff;
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int L = fft_lds_elems(n);
  const int span = 2 * H + 1;
  R vmax = R(0);   // largest |F| written by this thread (recorded when fmax_bits is given)
  for (int it = 0; it < iters; ++it) {
    const int pair0 = blk * per_block + it * geo.G;
    const int pair = pair0 + g;
    const bool active = pair < n / 2;
    const int ya = 2 * (active ? pair : 0);
    auto out = [&](int k, T v) {
      if (active) {
        fs[(long long)ya * n + k] = v.x;
        fs[(long long)(ya + 1) * n + k] = v.y;
        vmax = fmax(vmax, fmax(fabs(v.x), fabs(v.y)));
      }
    };
    if (cols == 0) {   // ring without lattice cells: its field is zero
      for (int k = t; k < n; k += geo.Tg) out(k, Cx<R>::mk(R(0), R(0)));
      continue;
    }
    for (int q = threadIdx.x; q < geo.G * L; q += blockDim.x) lds[q] = Cx<R>::mk(R(0), R(0));
    __syncthreads();
    // stage Z(., ya) + i Z(., ya + 1) over gx in [-H, H] (Z(-gx, y) = conj Z(gx, y))
    const int npair = min(geo.G, n / 2 - pair0);
    for (int q = threadIdx.x; q < npair * span; q += blockDim.x) {
      const int gg = q / span;
      const int gx = q - gg * span - H;
      const int y0 = 2 * (pair0 + gg);
      const int agx = gx < 0 ? -gx : gx;
      const T za = zs[(long long)y0 * cols + agx];
      const T zb = zs[(long long)(y0 + 1) * cols + agx];
      lds[gg * L + lpad(gx < 0 ? gx + n : gx)] =
          gx < 0 ? Cx<R>::mk(za.x + zb.y, -za.y + zb.x) : Cx<R>::mk(za.x - zb.y, za.y + zb.x);
    }
    __syncthreads();
    stockham_fft<R, U>(buf, n, log2n, t, geo.Tg, tw, out);
    __syncthreads();   // the staging area is refilled by the next iteration
  }
  if (fmax_bits) {
    float v = (float)vmax;
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    // non-negative floats order like their bit patterns
    if ((threadIdx.x & 63) == 0) atomicMax(&fmax_bits[(long long)set * nb + m], __float_as_uint(v));
  }
}

namespace {
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
constexpr int kRowIters = 4;
}  // namespace

int colpass_tile_columns(int n) { return fft_geom(n).G; }

template <typename R, bool DATA, typename GT>
hipError_t launch_colpass(const abs_plan_s* p, const GT* grids, const float* w, int w_batched,
                          int nsets, typename Cx<R>::T* Z, long long zset, const ColTile* tiles,
                          const typename Cx<R>::T* tw, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const dim3 grid((unsigned)p->tiles.size(), (unsigned)nsets);
  const FftGeom geo = fft_geom(p->n);
  const size_t lds = (size_t)geo.G * fft_lds_elems(p->n) * sizeof(typename Cx<R>::T);
  if (p->n > 4096) {
    auto k = colpass_kernel<R, 2, DATA, GT>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(grids, w, w_batched, p->wmode, p->n, p->log2n, tiles, bins, tw, Z, zset);
  } else {
    auto k = colpass_kernel<R, 1, DATA, GT>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(grids, w, w_batched, p->wmode, p->n, p->log2n, tiles, bins, tw, Z, zset);
  }
  return hipGetLastError();
}

hipError_t launch_colpass_data(const abs_plan_s* p, const void* grids, int dtype, const float* w,
                               int w_batched, int batch, float2* Z, long long zset, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const ColTile* tiles = reinterpret_cast<const ColTile*>(base + p->dl.tiles);
  const float2* tw = reinterpret_cast<const float2*>(base + p->dl.tw);
  if (dtype == ABS_C128)
    return launch_colpass<float, true, double2>(p, static_cast<const double2*>(grids), w, w_batched,
                                                batch, Z, zset, tiles, tw, st);
  return launch_colpass<float, true, float2>(p, static_cast<const float2*>(grids), w, w_batched,
                                             batch, Z, zset, tiles, tw, st);
}

hipError_t launch_colpass_weight(const abs_plan_s* p, const float* w, int w_batched, int nsets,
                                 double2* Z, long long zset, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const ColTile* tiles = reinterpret_cast<const ColTile*>(base + p->dl.tiles);
  const double2* tw = reinterpret_cast<const double2*>(base + p->dl.tw64);
  return launch_colpass<double, false, float2>(p, nullptr, w, w_batched, nsets, Z, zset, tiles, tw, st);
}

template <typename R>
hipError_t launch_rowpass(const abs_plan_s* p, int nsets, const typename Cx<R>::T* Z,
                          long long zset, R* F, long long fset, unsigned* fmax_bits, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const bool f64 = sizeof(R) == 8;
  const auto* tw = reinterpret_cast<const typename Cx<R>::T*>(base + (f64 ? p->dl.tw64 : p->dl.tw));
  const FftGeom geo = fft_geom(p->n);
  const int iters = std::max(1, std::min(kRowIters, p->n / 2 / geo.G));
  const int per_block = geo.G * iters;
  const int nrb = (p->n / 2 + per_block - 1) / per_block;
  const dim3 grid((unsigned)(p->nb * nrb), (unsigned)nsets);
  const size_t lds = (size_t)geo.G * fft_lds_elems(p->n) * sizeof(typename Cx<R>::T);
  if (p->n > 4096) {
    auto k = rowpass_kernel<R, 2>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(p->n, p->log2n, iters, bins, tw, Z, zset, F, fset, fmax_bits, p->nb);
  } else {
    auto k = rowpass_kernel<R, 1>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(p->n, p->log2n, iters, bins, tw, Z, zset, F, fset, fmax_bits, p->nb);
  }
  return hipGetLastError();
}

hipError_t launch_rowpass_f32(const abs_plan_s* p, int nsets, const float2* Z, long long zset,
                              float* F, long long fset, unsigned* fmax_bits, hipStream_t st) {
  return launch_rowpass<float>(p, nsets, Z, zset, F, fset, fmax_bits, st);
}
hipError_t launch_rowpass_f64(const abs_plan_s* p, int nsets, const double2* Z, long long zset,
                              double* F, long long fset, hipStream_t st) {
  return launch_rowpass<double>(p, nsets, Z, zset, F, fset, nullptr, st);
}

}  // namespace abs_impl
