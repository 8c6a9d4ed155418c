// Gridding of visibilities onto the uv grid, Eq. (9) of Gill et al. (2024).
//
// Each visibility V_i at baseline U_i adds w~ w_i V_i to the cells around g = rint(U_i / du)
// and, since the sky is real (V(-U) = conj V(U), Eq. 4), w~ w_i conj(V_i) to the mirrored
// cells -g; the weight sums N_g collect w~ w_i at both.  Sums are accumulated as 64-bit
// fixed-point integers with a power-of-two scale chosen from the largest |w_i V_i| (and
// w_i), so the result does not depend on the order in which the atomic adds land.
//
// Passes: (1) clear the accumulators and find the largest magnitudes, (2) scatter with
// integer atomics, (3) convert to FP32 and write the grid and the weight sums.
#include <algorithm>

#include "abs_internal.h"

namespace abs_impl {

struct GridScalars {
  unsigned int vmax_bits;   // largest |w V| component over all realisations (float bits)
  unsigned int wmax_bits;   // largest w
  unsigned long long dropped;
};

__global__ void __launch_bounds__(kBlock)
grid_clear_kernel(unsigned long long* __restrict__ acc, long long nacc, GridScalars* sc) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nacc; i += stride)
    acc[i] = 0ull;
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

__global__ void __launch_bounds__(kBlock)
grid_max_kernel(long long nvis, int batch, const float2* __restrict__ vis,
                const float* __restrict__ vw, GridScalars* sc) {
  float vm = 0.f, wm = 0.f;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const float wi = vw ? fabsf(vw[i]) : 1.0f;
    wm = fmaxf(wm, wi);
    for (int b = 0; b < batch; ++b) {
      const float2 v = vis[(long long)b * nvis + i];
      vm = fmaxf(vm, wi * fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  }
  vm = block_max(vm);
  wm = block_max(wm);
  if (threadIdx.x == 0) {
    // non-negative floats order like their bit patterns
    atomicMax(&sc->vmax_bits, __float_as_uint(vm));
    atomicMax(&sc->wmax_bits, __float_as_uint(wm));
  }
}

// Power-of-two scale E such that 2 * nvis * 49 contributions of magnitude <= max fit in
// 62 bits; returns 2^E as a double (E may be negative for huge inputs).
__device__ __forceinline__ double fixed_scale(float maxval, long long nvis) {
  if (!(maxval > 0.f)) return 1.0;
  int e;
  (void)frexpf(maxval, &e);               // maxval < 2^e
  int lg = 0;
  while ((1ll << lg) < 2 * 49 * (nvis > 0 ? nvis : 1)) ++lg;
  return ldexp(1.0, 61 - e - lg);
}

template <int KERNEL>
__global__ void __launch_bounds__(kBlock)
grid_scatter_kernel(int n, double du, double pit2, long long nvis, int batch,
                    const double2* __restrict__ uv, const float2* __restrict__ vis,
                    const float* __restrict__ vw, unsigned long long* __restrict__ acc,
                    unsigned long long* __restrict__ wacc, int integer_counts,
                    GridScalars* sc) {
  const double sv = fixed_scale(__uint_as_float(sc->vmax_bits), nvis);
  const double sw = integer_counts ? 1.0 : fixed_scale(__uint_as_float(sc->wmax_bits), nvis);
  const long long nn = (long long)n * n;
  const int half = n / 2;
  unsigned long long ndrop = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvis; i += stride) {
    const double2 U = uv[i];
    const double fx = U.x / du, fy = U.y / du;
    const long long gx = (long long)rint(fx), gy = (long long)rint(fy);
    if (!(gx > -half && gx < half && gy > -half && gy < half)) {  // NaN lands here too
      ++ndrop;
      continue;
    }
    const float wi = vw ? vw[i] : 1.0f;
    constexpr int R = KERNEL == ABS_GAUSS7 ? 3 : 0;
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const long long cx = gx + dx, cy = gy + dy;
        if (!(cx > -half && cx < half && cy > -half && cy < half)) continue;
        double kw = 1.0;
        if (KERNEL == ABS_GAUSS7) {
          const double ex = (double)cx * du - U.x, ey = (double)cy * du - U.y;
          kw = exp(-pit2 * (ex * ex + ey * ey));
        }
        const double c = kw * (double)wi;
        const long long i0 = (cy < 0 ? cy + n : cy) * n + (cx < 0 ? cx + n : cx);
        const long long i1 = (cy > 0 ? n - cy : -cy) * n + (cx > 0 ? n - cx : -cx);
        const unsigned long long qw = (unsigned long long)llrint(c * sw);
        atomicAdd(&wacc[i0], qw);
        atomicAdd(&wacc[i1], qw);
        for (int b = 0; b < batch; ++b) {
          const float2 v = vis[(long long)b * nvis + i];
          const unsigned long long qr = (unsigned long long)llrint(c * (double)v.x * sv);
          const unsigned long long qi = (unsigned long long)llrint(c * (double)v.y * sv);
          unsigned long long* a = acc + (long long)b * 2 * nn;
          atomicAdd(&a[2 * i0], qr);
          atomicAdd(&a[2 * i0 + 1], qi);
          atomicAdd(&a[2 * i1], qr);
          atomicAdd(&a[2 * i1 + 1], (unsigned long long)(-(long long)qi));
        }
      }
  }
  for (int o = 32; o > 0; o >>= 1) ndrop += __shfl_xor(ndrop, o);
  if ((threadIdx.x & 63) == 0 && ndrop) atomicAdd(&sc->dropped, ndrop);
}

__global__ void __launch_bounds__(kBlock)
grid_convert_kernel(int n, long long nvis, int batch, const unsigned long long* __restrict__ acc,
                    const unsigned long long* __restrict__ wacc, int integer_counts,
                    float2* __restrict__ grid, float* __restrict__ wsum,
                    long long* __restrict__ dropped, const GridScalars* sc) {
  const double sv = fixed_scale(__uint_as_float(sc->vmax_bits), nvis);
  const double sw = integer_counts ? 1.0 : fixed_scale(__uint_as_float(sc->wmax_bits), nvis);
  const double iv = 1.0 / sv, iw = 1.0 / sw;  // powers of two: exact
  const long long nn = (long long)n * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nn; c += stride) {
    for (int b = 0; b < batch; ++b) {
      const unsigned long long* a = acc + (long long)b * 2 * nn;
      grid[(long long)b * nn + c] = make_float2((float)((double)(long long)a[2 * c] * iv),
                                                (float)((double)(long long)a[2 * c + 1] * iv));
    }
    if (wsum) wsum[c] = (float)((double)(long long)wacc[c] * iw);
  }
  if (dropped && blockIdx.x == 0 && threadIdx.x == 0) *dropped = (long long)sc->dropped;
}

}  // namespace abs_impl

using namespace abs_impl;

extern "C" abs_status abs_grid(abs_plan_t p, int64_t nvis, int32_t batch, const double* uv,
                               const float* vis, const float* vis_w, int32_t kernel, void* work,
                               size_t work_bytes, float* grid, float* wsum, int64_t* dropped,
                               void* stream) {
  if (!p) return ABS_ERR_INVALID;
  if (!p->dev) return ABS_ERR_UNBOUND;
  if (nvis < 0 || batch < 1 || batch > p->max_batch) return ABS_ERR_INVALID;
  if (kernel != ABS_NEAREST && kernel != ABS_GAUSS7) return ABS_ERR_INVALID;
  if (!work || !grid || (nvis > 0 && (!uv || !vis))) return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(uv) | reinterpret_cast<uintptr_t>(vis) |
       reinterpret_cast<uintptr_t>(grid) | reinterpret_cast<uintptr_t>(work)) & 15)
    return ABS_ERR_INVALID;
  size_t need = 0;
  abs_grid_workspace(p, batch, &need);
  if (work_bytes < need) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long nn = (long long)p->n * p->n;
  GridScalars* sc = static_cast<GridScalars*>(work);
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(static_cast<char*>(work) + 256);
  unsigned long long* wacc = acc + (long long)2 * batch * nn;
  const long long nacc = (long long)(2 * batch + 1) * nn;
  const int integer_counts = (vis_w == nullptr && kernel == ABS_NEAREST) ? 1 : 0;
  const double pi = 3.14159265358979323846;
  const double pit2 = pi * pi * p->theta0 * p->theta0;
  (void)hipGetLastError();
  grid_clear_kernel<<<1024, kBlock, 0, st>>>(acc, nacc, sc);
  const unsigned gv = (unsigned)std::min<long long>(4096, std::max<long long>(1, (nvis + kBlock - 1) / kBlock));
  if (nvis > 0) {
    grid_max_kernel<<<gv, kBlock, 0, st>>>(nvis, batch, reinterpret_cast<const float2*>(vis), vis_w, sc);
    prof_begin(p, ABS_STAGE_GRID, st);
    if (kernel == ABS_GAUSS7)
      grid_scatter_kernel<ABS_GAUSS7><<<gv, kBlock, 0, st>>>(
          p->n, p->du, pit2, nvis, batch, reinterpret_cast<const double2*>(uv),
          reinterpret_cast<const float2*>(vis), vis_w, acc, wacc, integer_counts, sc);
    else
      grid_scatter_kernel<ABS_NEAREST><<<gv, kBlock, 0, st>>>(
          p->n, p->du, pit2, nvis, batch, reinterpret_cast<const double2*>(uv),
          reinterpret_cast<const float2*>(vis), vis_w, acc, wacc, integer_counts, sc);
    prof_end(p, ABS_STAGE_GRID, st);
  }
  grid_convert_kernel<<<2048, kBlock, 0, st>>>(p->n, nvis, batch, acc, wacc, integer_counts,
                                               reinterpret_cast<float2*>(grid), wsum,
                                               reinterpret_cast<long long*>(dropped), sc);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}
