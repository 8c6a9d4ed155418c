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
// Both passes stage a batch of sequences in LDS and run an in-place radix-4
// decimation-in-frequency FFT (one radix-2 step closes odd log2 n); results are
// read back through the digit-reversal map.
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

template <typename T>
__device__ __forceinline__ T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// Position of DFT output k after the in-place DIF stages (radix 4, then 2).
__device__ __forceinline__ int dr_pos(int k, int n) {
  int pos = 0;
  int m = n;
  while (m >= 4) {
    m >>= 2;
    pos += (k & 3) * m;
    k >>= 2;
  }
  return pos + k;  // m is 2 (k in {0, 1}) or 1 (k == 0)
}

// nseq sequences of length n at buf[s * n + idx]; forward sign; tw[k] = exp(-2 pi i k / n).
template <typename R>
__device__ void lds_fft(typename Cx<R>::T* buf, int n, int log2n, int nseq,
                        const typename Cx<R>::T* __restrict__ tw) {
  using T = typename Cx<R>::T;
  const int quarter_n = n >> 2;
  const int lq = log2n - 2;
  for (int len = n, llen = log2n; len >= 4; len >>= 2, llen -= 2) {
    const int q = len >> 2, lqq = llen - 2;
    const int stride = n >> llen;
    const int nbf = nseq * quarter_n;
    for (int t = threadIdx.x; t < nbf; t += blockDim.x) {
      const int s = t >> lq;
      const int r = t & (quarter_n - 1);
      const int j = r & (q - 1);
      const int grp = r >> lqq;
      T* b = buf + s * n + grp * len + j;
      const T a0 = b[0], a1 = b[q], a2 = b[2 * q], a3 = b[3 * q];
      const R s02x = a0.x + a2.x, s02y = a0.y + a2.y, d02x = a0.x - a2.x, d02y = a0.y - a2.y;
      const R s13x = a1.x + a3.x, s13y = a1.y + a3.y, d13x = a1.x - a3.x, d13y = a1.y - a3.y;
      // y_p = sum_q a_q (-i)^{q p}
      const T y0 = Cx<R>::mk(s02x + s13x, s02y + s13y);
      const T y2 = Cx<R>::mk(s02x - s13x, s02y - s13y);
      const T y1 = Cx<R>::mk(d02x + d13y, d02y - d13x);
      const T y3 = Cx<R>::mk(d02x - d13y, d02y + d13x);
      b[0] = y0;
      if (j == 0) {
        b[q] = y1;
        b[2 * q] = y2;
        b[3 * q] = y3;
      } else {
        const int e = j * stride;
        b[q] = cmul(y1, tw[e]);
        b[2 * q] = cmul(y2, tw[2 * e]);
        b[3 * q] = cmul(y3, tw[3 * e]);
      }
    }
    __syncthreads();
  }
  if (log2n & 1) {
    const int half = n >> 1;
    const int nbf = nseq * half;
    for (int t = threadIdx.x; t < nbf; t += blockDim.x) {
      const int s = t >> (log2n - 1);
      const int g = t & (half - 1);
      T* b = buf + s * n + 2 * g;
      const T a0 = b[0], a1 = b[1];
      b[0] = Cx<R>::mk(a0.x + a1.x, a0.y + a1.y);
      b[1] = Cx<R>::mk(a0.x - a1.x, a0.y - a1.y);
    }
    __syncthreads();
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

// Column pass.  blockIdx.x: column tile; blockIdx.y: set.  DATA: the set is grid
// `set` and the staged values are X = (W V(g) + conj(W V(-g)))/2 in FP32; otherwise
// the set is weight array `set` and the values are Y = (W(g) + W(-g))/2 in R.
template <typename R, bool DATA, typename GT>
__global__ void __launch_bounds__(kBlock)
colpass_kernel(const GT* __restrict__ grids, const float* __restrict__ w, int w_batched, int wmode,
               int n, int log2n, const ColTile* __restrict__ tiles, const BinDev* __restrict__ bins,
               const typename Cx<R>::T* __restrict__ tw, typename Cx<R>::T* __restrict__ Z,
               long long zset) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const ColTile tile = tiles[blockIdx.x];
  const int set = blockIdx.y;
  const long long nn = (long long)n * n;
  const float* __restrict__ ws = (w && w_batched) ? w + (long long)set * nn : w;
  const BinDev bin = bins[tile.m];
  const int nc = tile.ncols, H = bin.h;
  for (int t = threadIdx.x; t < nc * n; t += blockDim.x) lds[t] = Cx<R>::mk(R(0), R(0));
  __syncthreads();
  const int nrows = 2 * H + 1;
  for (int t = threadIdx.x; t < nrows * nc; t += blockDim.x) {
    const int r = t / nc, c = t - r * nc;
    const int gy = r - H, gx = tile.gx0 + c;
    const long long r2 = (long long)gx * gx + (long long)gy * gy;
    const double d2 = (double)r2;
    if (!(d2 >= bin.lo2 && d2 < bin.hi2)) continue;
    const int iy = gy < 0 ? gy + n : gy, ix = gx;  // gx >= 0
    const int my = gy > 0 ? n - gy : -gy, mx = gx > 0 ? n - gx : 0;
    const long long i0 = (long long)iy * n + ix, i1 = (long long)my * n + mx;
    const R w0 = weight_of<R>(ws, wmode, i0), w1 = weight_of<R>(ws, wmode, i1);
    T v;
    if constexpr (DATA) {
      const GT* __restrict__ gs = grids + (long long)set * nn;
      const float2 a = load_vis(gs, i0), b = load_vis(gs, i1);
      v = Cx<R>::mk(R(0.5) * (w0 * a.x + w1 * b.x), R(0.5) * (w0 * a.y - w1 * b.y));
    } else {
      v = Cx<R>::mk(R(0.5) * (w0 + w1), R(0));
    }
    lds[c * n + iy] = v;
  }
  __syncthreads();
  lds_fft<R>(lds, n, log2n, nc, tw);
  const int cols = bin.cols;
  T* __restrict__ zs = Z + (long long)set * zset + bin.zoff;
  for (int t = threadIdx.x; t < n * nc; t += blockDim.x) {
    const int y = t / nc, c = t - y * nc;
    zs[(long long)y * cols + tile.gx0 + c] = lds[c * n + dr_pos(y, n)];
  }
}

// Row pass.  blockIdx.x: ring m * (row-pair blocks per ring) + block; blockIdx.y: set.
template <typename R>
__global__ void __launch_bounds__(kBlock)
rowpass_kernel(int n, int log2n, int rb, const BinDev* __restrict__ bins,
               const typename Cx<R>::T* __restrict__ tw, const typename Cx<R>::T* __restrict__ Z,
               long long zset, R* __restrict__ F, long long fset) {
  using T = typename Cx<R>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int nrb = (n / 2 + rb - 1) / rb;
  const int m = blockIdx.x / nrb, blk = blockIdx.x - m * nrb;
  const int set = blockIdx.y;
  const BinDev bin = bins[m];
  const int H = bin.h, cols = bin.cols;
  const int pair0 = blk * rb;
  const int npair = min(rb, n / 2 - pair0);
  const long long nn = (long long)n * n;
  R* __restrict__ fs = F + (long long)set * fset + (long long)m * nn;
  if (cols == 0) {  // ring without lattice cells: its field is zero
    for (int t = threadIdx.x; t < npair * 2 * n; t += blockDim.x)
      fs[(long long)2 * pair0 * n + t] = R(0);
    return;
  }
  for (int t = threadIdx.x; t < npair * n; t += blockDim.x) lds[t] = Cx<R>::mk(R(0), R(0));
  __syncthreads();
  const T* __restrict__ zs = Z + (long long)set * zset + bin.zoff;
  const int span = 2 * H + 1;
  for (int t = threadIdx.x; t < npair * span; t += blockDim.x) {
    const int r = t / span;
    const int gx = t - r * span - H;
    const int ya = 2 * (pair0 + r);
    const int agx = gx < 0 ? -gx : gx;
    T za = zs[(long long)ya * cols + agx];
    T zb = zs[(long long)(ya + 1) * cols + agx];
    if (gx < 0) {
      za.y = -za.y;
      zb.y = -zb.y;
    }
    lds[r * n + (gx < 0 ? gx + n : gx)] = Cx<R>::mk(za.x - zb.y, za.y + zb.x);
  }
  __syncthreads();
  lds_fft<R>(lds, n, log2n, npair, tw);
  for (int t = threadIdx.x; t < npair * n; t += blockDim.x) {
    const int r = t / n, x = t - r * n;
    const T v = lds[r * n + dr_pos(x, n)];
    const long long y = 2 * (pair0 + r);
    fs[y * n + x] = v.x;
    fs[(y + 1) * n + x] = v.y;
  }
}

namespace {
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
}  // namespace

hipError_t launch_colpass_data(const abs_plan_s* p, const void* grids, int dtype, const float* w,
                               int w_batched, int batch, float2* Z, long long zset, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const ColTile* tiles = reinterpret_cast<const ColTile*>(base + p->dl.tiles);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const float2* tw = reinterpret_cast<const float2*>(base + p->dl.tw);
  const dim3 grid((unsigned)p->tiles.size(), (unsigned)batch);
  const size_t lds = (size_t)p->ct * p->n * sizeof(float2);
  if (dtype == ABS_C128) {
    auto k = colpass_kernel<float, true, double2>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(static_cast<const double2*>(grids), w, w_batched, p->wmode, p->n,
                                 p->log2n, tiles, bins, tw, Z, zset);
  } else {
    auto k = colpass_kernel<float, true, float2>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<grid, kBlock, lds, st>>>(static_cast<const float2*>(grids), w, w_batched, p->wmode, p->n,
                                 p->log2n, tiles, bins, tw, Z, zset);
  }
  return hipGetLastError();
}

hipError_t launch_colpass_weight(const abs_plan_s* p, const float* w, int w_batched, int nsets,
                                 double2* Z, long long zset, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const ColTile* tiles = reinterpret_cast<const ColTile*>(base + p->dl.tiles64);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const double2* tw = reinterpret_cast<const double2*>(base + p->dl.tw64);
  const dim3 grid((unsigned)p->tiles64.size(), (unsigned)nsets);
  const size_t lds = (size_t)p->ct64 * p->n * sizeof(double2);
  auto k = colpass_kernel<double, false, float2>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  k<<<grid, kBlock, lds, st>>>(nullptr, w, w_batched, p->wmode, p->n, p->log2n, tiles, bins, tw,
                               Z, zset);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_rowpass(const abs_plan_s* p, int nsets, const typename Cx<R>::T* Z,
                          long long zset, R* F, long long fset, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const BinDev* bins = reinterpret_cast<const BinDev*>(base + p->dl.bins);
  const bool f64 = sizeof(R) == 8;
  const auto* tw = reinterpret_cast<const typename Cx<R>::T*>(base + (f64 ? p->dl.tw64 : p->dl.tw));
  const int rb = f64 ? p->rb64 : p->rb;
  const int nrb = (p->n / 2 + rb - 1) / rb;
  const dim3 grid((unsigned)(p->nb * nrb), (unsigned)nsets);
  const size_t lds = (size_t)rb * p->n * sizeof(typename Cx<R>::T);
  auto k = rowpass_kernel<R>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  k<<<grid, kBlock, lds, st>>>(p->n, p->log2n, rb, bins, tw, Z, zset, F, fset);
  return hipGetLastError();
}

hipError_t launch_rowpass_f32(const abs_plan_s* p, int nsets, const float2* Z, long long zset,
                              float* F, long long fset, hipStream_t st) {
  return launch_rowpass<float>(p, nsets, Z, zset, F, fset, st);
}
hipError_t launch_rowpass_f64(const abs_plan_s* p, int nsets, const double2* Z, long long zset,
                              double* F, long long fset, hipStream_t st) {
  return launch_rowpass<double>(p, nsets, Z, zset, F, fset, st);
}

}  // namespace abs_impl
