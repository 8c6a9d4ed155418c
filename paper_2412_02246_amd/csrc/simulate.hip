// Visibilities of a flat-sky brightness field (Eq. 4 of Gill et al. 2024), the
// simulation step that precedes gridding in the paper's validation (Sec. 3: the sky is
// simulated on a flat grid, multiplied by the primary beam of Eq. 5 and transformed to
// the baselines by a DFT).
//
// For a sky of N x N pixels of side dtheta, pixel (a, b) (a: x / column, b: y / row) at
// theta = ((a - N/2) dtheta, (b - N/2) dtheta),
//   V(U) = q dtheta^2 sum_{a,b} A(theta_ab) T_ab exp(+2 pi i (u theta_x + v theta_y)),
// which is periodic in u and v with period 1/dtheta.  Direct summation costs N^2 per
// baseline; here it is a type-2 non-uniform FFT (Dutt & Rokhlin 1993; the
// "exponential of semicircle" kernel of Barnett, Magland & af Klinteberg 2019):
//   1. f_ab = q dtheta^2 A(theta_ab) T_ab / (c(a') c(b')), a' = a - N/2, with c the
//      kernel's Fourier transform on the pixel offsets (deconvolution);
//   2. G_j = sum_ab f_ab exp(+2 pi i (j_x a' + j_y b') / M) on the M = 2N grid (a
//      zero-padded 2-D FFT: M-point transforms of the N sky rows, a transpose, M-point
//      transforms of the M columns' N inputs);
//   3. V(U) = sum over the W x W grid points j nearest to x = U dtheta M of
//      phi(x_x - j_x) phi(x_y - j_y) G_j, phi(d) = exp(beta (sqrt(1 - (2d/W)^2) - 1)).
// With W = 8 and beta = 2.3 W on the twice-oversampled grid the kernel's error is about
// 1e-7 of the sum of |f|; the FP32 transforms add about 1e-6 of the visibilities' rms.
// Both beams of the paper are separable (Eq. 5: sinc^2 in theta_x times sinc^2 in
// theta_y; Eq. 6: a Gaussian), so step 1 multiplies each pixel by a row factor and a
// column factor from one table.
#include <cmath>

#include "fft_engine.h"

namespace abs_impl {
namespace {

constexpr int kSimW = 8;                  // kernel width in grid points
constexpr double kSimBeta = 2.3 * kSimW;  // kernel shape
constexpr int kQuad = 256;                // midpoint nodes for the kernel's transform

// Per-axis factor of pixel offset a' = a - N/2: the beam (one axis) over c(a'), where
// c(x) = (W/2) int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(pi W z x / M) dz (the
// kernel's Fourier transform, scaled as the spreading sum needs it); computed with
// z = sin s, a smooth periodic integrand, by the midpoint rule.  Also the twiddles
// exp(-2 pi i k / M) of the M-point transforms.  FP64.
__global__ void __launch_bounds__(kBlock)
sim_tables_kernel(int nsky, int msz, double dtheta, int beam, double bparam, float* __restrict__ axis,
                  float2* __restrict__ tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < msz) {
    double s, c;
    sincos(-2.0 * M_PI * (double)i / (double)msz, &s, &c);
    tw[i] = make_float2((float)c, (float)s);
  }
  if (i >= nsky) return;
  const double x = (double)(i - nsky / 2);
  double acc = 0.0;
  for (int q = 0; q < kQuad; ++q) {
    const double t = -0.5 * M_PI + M_PI * ((double)q + 0.5) / kQuad;
    double st, ct;
    sincos(t, &st, &ct);
    acc += exp(kSimBeta * (ct - 1.0)) * cos(M_PI * kSimW * st * x / (double)msz) * ct;
  }
  const double cx = 0.5 * kSimW * acc * (M_PI / kQuad);
  const double th = x * dtheta;
  double a = 1.0;
  if (beam == ABS_BEAM_MWA) {   // sinc^2(pi d theta / lambda), bparam = d / lambda
    const double y = M_PI * bparam * th;
    a = y == 0.0 ? 1.0 : (sin(y) / y) * (sin(y) / y);
  } else if (beam == ABS_BEAM_GAUSS) {   // exp(-theta^2 / theta0^2) per axis, bparam = theta0
    a = exp(-(th * th) / (bparam * bparam));
  }
  axis[i] = (float)(a / cx);
}

// Step 1 and the first half of step 2: for each sky row b (blockIdx.x * G + g), the
// M-point transform of the row's N deconvolved, beam-weighted, zero-padded values
// (input k holds pixel a' = k for k < N/2 and a' = k - M for k >= M - N/2), written to
// T[b][0 .. M).  The input slabs of the first pass that hold no pixel are not read.
template <int LOG2M>
__global__ void __launch_bounds__(kBlock)
sim_rows_kernel(const float* __restrict__ sky, int nsky, float scale, const float* __restrict__ axis,
                const float2* __restrict__ tw, float2* __restrict__ T) {
  using FF = Fft<LOG2M, kBlock>;
  constexpr int M = FF::N, S = M / 16;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int g = threadIdx.x / FF::TG, t = threadIdx.x - g * FF::TG;
  float2* buf = reinterpret_cast<float2*>(lds_raw) + g * FF::L;
  TwiddlesSplit<float, LOG2M, kBlock> twr;
  twr.stage(tw, reinterpret_cast<float2*>(lds_raw) + FF::G * FF::L, threadIdx.x, kBlock);
  __syncthreads();
  const int half = nsky / 2;
  const int b = blockIdx.x * FF::G + g;
  const bool active = b < nsky;
  const float* __restrict__ row = sky + (long long)(active ? b : 0) * nsky;
  const float rb = active ? scale * axis[b] : 0.0f;
  auto in = [&](int k, int, int r) -> float2 {
    float2 x = make_float2(0.0f, 0.0f);
    if (active && (r * S < half || (r + 1) * S > M - half)) {
      if (k < half) x.x = rb * axis[half + k] * row[half + k];
      else if (k >= M - half) x.x = rb * axis[k - (M - half)] * row[k - (M - half)];
    }
    return x;
  };
  float2* __restrict__ out_row = T + (long long)(active ? b : 0) * M;
  auto out = [&](int k, int, int, float2 v) {
    if (active) out_row[k] = v;
  };
  fft_passes<float, LOG2M, 0, kBlock>(buf, t, tw, twr, in, out);
}

// TT[x][y] = T[y][x] for an R x C complex matrix, through an LDS tile of 32 x 32.
__global__ void __launch_bounds__(kBlock)
sim_transpose_kernel(const float2* __restrict__ T, int R, int C, float2* __restrict__ TT) {
  __shared__ float2 tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += kBlock / 32) {
    const int r = r0 + y, c = c0 + tx;
    if (r < R && c < C) tile[y][tx] = T[(long long)r * C + c];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += kBlock / 32) {
    const int c = c0 + y, r = r0 + tx;
    if (r < R && c < C) TT[(long long)c * R + r] = tile[tx][y];
  }
}

// The second half of step 2: for each column j_x (a row of TT, N values over the sky
// rows), the M-point transform over b' (input k holds row b' = k for k < N/2 and
// b' = k - M for k >= M - N/2), written to G[j_x][0 .. M).
template <int LOG2M>
__global__ void __launch_bounds__(kBlock)
sim_cols_kernel(const float2* __restrict__ TT, int nsky, const float2* __restrict__ tw, float2* __restrict__ G) {
  using FF = Fft<LOG2M, kBlock>;
  constexpr int M = FF::N, S = M / 16;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int g = threadIdx.x / FF::TG, t = threadIdx.x - g * FF::TG;
  float2* buf = reinterpret_cast<float2*>(lds_raw) + g * FF::L;
  TwiddlesSplit<float, LOG2M, kBlock> twr;
  twr.stage(tw, reinterpret_cast<float2*>(lds_raw) + FF::G * FF::L, threadIdx.x, kBlock);
  __syncthreads();
  const int half = nsky / 2;
  const int jx = blockIdx.x * FF::G + g;
  const bool active = jx < M;   // small M: a block holds more transforms than there are rows
  const float2* __restrict__ col = TT + (long long)(active ? jx : 0) * nsky;
  auto in = [&](int k, int, int r) -> float2 {
    float2 x = make_float2(0.0f, 0.0f);
    if (active && (r * S < half || (r + 1) * S > M - half)) {
      if (k < half) x = col[half + k];
      else if (k >= M - half) x = col[k - (M - half)];
    }
    return x;
  };
  float2* __restrict__ out_row = G + (long long)(active ? jx : 0) * M;
  auto out = [&](int k, int, int, float2 v) {
    if (active) out_row[k] = v;
  };
  fft_passes<float, LOG2M, 0, kBlock>(buf, t, tw, twr, in, out);
}

// Step 3: one thread per baseline.  x = u dtheta M, y = v dtheta M in grid units (FP64);
// the W grid points j with |x - j| < W/2 on each axis (indices modulo M); weights
// phi(x - j) phi(y - k); G holds the forward transform, so the sum of exp(+...) terms is
// its complex conjugate (f is real).  vis[i] = (Re V, Im V).
__global__ void __launch_bounds__(kBlock)
sim_interp_kernel(const float2* __restrict__ G, int msz, double dtheta, long long nvis, const double* __restrict__ uv,
                  float2* __restrict__ vis) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvis) return;
  const double x = uv[2 * i] * dtheta * msz, y = uv[2 * i + 1] * dtheta * msz;
  const double jx0 = floor(x - 0.5 * kSimW) + 1.0, jy0 = floor(y - 0.5 * kSimW) + 1.0;
  const float fx = (float)(x - jx0), fy = (float)(y - jy0);   // in (W/2 - 1, W/2]
  float wx[kSimW], wy[kSimW];
#pragma unroll
  for (int q = 0; q < kSimW; ++q) {
    const float zx = (fx - (float)q) * (2.0f / kSimW), zy = (fy - (float)q) * (2.0f / kSimW);
    wx[q] = zx * zx < 1.0f ? expf((float)kSimBeta * (sqrtf(1.0f - zx * zx) - 1.0f)) : 0.0f;
    wy[q] = zy * zy < 1.0f ? expf((float)kSimBeta * (sqrtf(1.0f - zy * zy) - 1.0f)) : 0.0f;
  }
  const long long mm = msz;
  const long long bx = (((long long)jx0 % mm) + mm) % mm, by = (((long long)jy0 % mm) + mm) % mm;
  float re = 0.0f, im = 0.0f;
#pragma unroll
  for (int p = 0; p < kSimW; ++p) {
    long long rx = bx + p;
    if (rx >= mm) rx -= mm;
    const float2* __restrict__ grow = G + rx * mm;
    float sr = 0.0f, si = 0.0f;
#pragma unroll
    for (int q = 0; q < kSimW; ++q) {
      long long cy = by + q;
      if (cy >= mm) cy -= mm;
      const float2 v = grow[cy];
      sr = fmaf(wy[q], v.x, sr);
      si = fmaf(wy[q], v.y, si);
    }
    re = fmaf(wx[p], sr, re);
    im = fmaf(wx[p], si, im);
  }
  vis[i] = make_float2(re, -im);
}

struct SimWork {
  size_t axis, tw, T, TT, G, total;
};
SimWork sim_layout(int nsky) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t n = (size_t)nsky, m = 2 * n;
  SimWork w{};
  size_t off = 0;
  w.axis = off;
  off = al(off + n * 4);
  w.tw = off;
  off = al(off + m * 8);
  w.T = off;   // T (N x M) and later G (M x M) share the front of this region
  w.G = off;
  off = al(off + std::max(n * m, m * m) * 8);
  w.TT = off;
  off = al(off + m * n * 8);
  w.total = off;
  return w;
}

template <int LOG2M>
hipError_t launch_sim_ffts(const float* sky, int nsky, float scale, const float* axis, const float2* tw,
                           float2* T, float2* TT, float2* G, hipStream_t st) {
  using FF = Fft<LOG2M, kBlock>;
  constexpr int M = FF::N;
  const size_t lds = (size_t)(FF::G * FF::L + TwiddlesSplit<float, LOG2M, kBlock>::ENTRIES) * sizeof(float2);
  auto kr = sim_rows_kernel<LOG2M>;
  auto kc = sim_cols_kernel<LOG2M>;
  if (lds > 65536) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(kr), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(kc), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return hipErrorInvalidValue;
  }
  kr<<<(unsigned)((nsky + FF::G - 1) / FF::G), kBlock, lds, st>>>(sky, nsky, scale, axis, tw, T);
  sim_transpose_kernel<<<dim3((unsigned)(M / 32), (unsigned)((nsky + 31) / 32)), kBlock, 0, st>>>(T, nsky, M, TT);
  kc<<<(unsigned)((M + FF::G - 1) / FF::G), kBlock, lds, st>>>(TT, nsky, tw, G);
  return hipGetLastError();
}

}  // namespace
}  // namespace abs_impl

using namespace abs_impl;

extern "C" {

abs_status abs_simulate_workspace(int32_t nsky, size_t* bytes) {
  if (!bytes || nsky < 16 || nsky > kMaxN / 2 || (nsky & (nsky - 1))) return ABS_ERR_INVALID;
  *bytes = sim_layout(nsky).total;
  return ABS_OK;
}

abs_status abs_simulate(int32_t nsky, double dtheta, int32_t beam, double beam_param, double q, int32_t batch,
                        const float* sky, int64_t nvis, const double* uv, float* vis, void* work, size_t work_bytes,
                        void* stream) {
  if (nsky < 16 || nsky > kMaxN / 2 || (nsky & (nsky - 1))) return ABS_ERR_INVALID;
  if (!(dtheta > 0.0) || !std::isfinite(dtheta) || !std::isfinite(q)) return ABS_ERR_INVALID;
  if (beam < ABS_BEAM_NONE || beam > ABS_BEAM_GAUSS) return ABS_ERR_INVALID;
  if (beam != ABS_BEAM_NONE && !(beam_param > 0.0 && std::isfinite(beam_param))) return ABS_ERR_INVALID;
  if (batch < 1 || nvis < 0 || !sky || !work || (nvis > 0 && (!uv || !vis))) return ABS_ERR_INVALID;
  if ((reinterpret_cast<uintptr_t>(work) & 255) || (reinterpret_cast<uintptr_t>(sky) & 3)) return ABS_ERR_INVALID;
  const SimWork wl = sim_layout(nsky);
  if (work_bytes < wl.total) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wk = static_cast<char*>(work);
  float* axis = reinterpret_cast<float*>(wk + wl.axis);
  float2* tw = reinterpret_cast<float2*>(wk + wl.tw);
  float2* T = reinterpret_cast<float2*>(wk + wl.T);
  float2* TT = reinterpret_cast<float2*>(wk + wl.TT);
  float2* G = reinterpret_cast<float2*>(wk + wl.G);
  const int msz = 2 * nsky;
  (void)hipGetLastError();
  sim_tables_kernel<<<(unsigned)((msz + kBlock - 1) / kBlock), kBlock, 0, st>>>(nsky, msz, dtheta, beam, beam_param,
                                                                              axis, tw);
  const float scale = (float)(q * dtheta * dtheta);
  for (int b = 0; b < batch; ++b) {
    const float* s = sky + (long long)b * nsky * nsky;
    hipError_t e;
    switch (msz) {
#define ABS_SIM_CASE(L) \
  case 1 << L: e = launch_sim_ffts<L>(s, nsky, scale, axis, tw, T, TT, G, st); break;
      ABS_SIM_CASE(5) ABS_SIM_CASE(6) ABS_SIM_CASE(7) ABS_SIM_CASE(8) ABS_SIM_CASE(9)
      ABS_SIM_CASE(10) ABS_SIM_CASE(11) ABS_SIM_CASE(12) ABS_SIM_CASE(13)
#undef ABS_SIM_CASE
      default: return ABS_ERR_INVALID;
    }
    if (e != hipSuccess) return ABS_ERR_DEVICE;
    if (nvis > 0)
      sim_interp_kernel<<<(unsigned)((nvis + kBlock - 1) / kBlock), kBlock, 0, st>>>(
          G, msz, dtheta, nvis, uv, reinterpret_cast<float2*>(vis) + (long long)b * nvis);
  }
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

}  // extern "C"
