// After the estimator: the (ell1, mu, t) re-binning of the triplet estimates, ensemble
// statistics over realisations, and the local quadratic model's prediction averaged over
// the same lattice triangles ([B_Ana]_d), following Gill et al. (2024) Secs. 3 and 4.
//
// Re-binning (Sec. 3): ell1 in bins of equal logarithmic width, mu and t in equal linear
// bins of [0.5, 1]; a bin's value is the average of its triplets' B_t weighted by their
// triangle counts N_t, i.e. sum N_t B_t / sum N_t, which is Eq. (12) over the union of the
// bin's triangles.  Sums run over the triplets in index order (FP64), so results do not
// depend on the launch shape.
//
// Ensemble (Sec. 3): mean and sigma^2 = <X^2> - <X>^2 over the realisations, one thread
// per value, realisations added in order; Delta_B = |mean - model| / model and
// Delta_sigma = |mean - model| / sigma (Sec. 4).
//
// Model prediction (Eq. 14 averaged like Eq. 12): for triplet t the weighted sum
// T2_t = sum over closed triangles of Y1 Y2 Y3 (C1 C2 + C2 C3 + C3 C1).  The triangle sum
// F(Y) = sum Y1 Y2 Y3 is trilinear in the weights, so with Y' = Y (1 + s C / cmax),
// F(s) = N + s T1 / cmax + s^2 T2 / cmax^2 + s^3 T3 / cmax^3 and
// T2 = cmax^2 (F(+1) + F(-1) - 2 F(0)) / 2: three runs of the FP64 weight path (the same
// ring FFTs and contraction as N_t), combined as [B_Ana]_d,t = 2 f T2_t / N_t.
#include <cmath>

#include "abs_internal.h"

namespace abs_impl {

// One thread per (bin, grid): the bin's triplets in index order.
__global__ void __launch_bounds__(kBlock)
rebin_kernel(int ntrip, int nbins, const int* __restrict__ bin_of, const double* __restrict__ B,
             const double* __restrict__ N, double* __restrict__ Bbin, double* __restrict__ Nbin) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (k >= nbins) return;
  const double* Bg = B + (long long)g * ntrip;
  const double* Ng = N + (long long)g * ntrip;
  double num = 0.0, den = 0.0;
  for (int t = 0; t < ntrip; ++t) {
    if (bin_of[t] != k) continue;
    const double b = Bg[t];
    if (b != b) continue;   // empty triplet (NaN)
    num += Ng[t] * b;
    den += Ng[t];
  }
  Bbin[(long long)g * nbins + k] = den != 0.0 ? num / den : __builtin_nan("");
  Nbin[(long long)g * nbins + k] = den;
}

__global__ void __launch_bounds__(kBlock)
ensemble_kernel(int nreal, int nvals, const double* __restrict__ X, const double* __restrict__ model,
                double* __restrict__ mean, double* __restrict__ sigma, double* __restrict__ dB,
                double* __restrict__ dsig) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvals) return;
  double s = 0.0, s2 = 0.0;
  for (int r = 0; r < nreal; ++r) {
    const double x = X[(long long)r * nvals + v];
    s += x;
    s2 += x * x;
  }
  const double m = s / nreal;
  const double sg = sqrt(fmax(s2 / nreal - m * m, 0.0));
  mean[v] = m;
  sigma[v] = sg;
  if (model) {
    const double d = fabs(m - model[v]);
    if (dB) dB[v] = d / model[v];
    if (dsig) dsig[v] = d / sg;
  }
}

__global__ void zero_u32_kernel(unsigned* a) {
  if (threadIdx.x == 0) *a = 0u;
}

// Largest |(c(g) + c(-g)) / 2| over the cells of all rings (lo2 <= |g|^2 < hi2), as float
// bits (non-negative floats order like their bits).
__global__ void __launch_bounds__(kBlock)
cmax_kernel(const float* __restrict__ c, int n, int hm, double lo2, double hi2, unsigned* __restrict__ out) {
  const int side = 2 * hm + 1;
  float m = 0.f;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < (long long)side * side;
       e += (long long)gridDim.x * blockDim.x) {
    const int gy = (int)(e / side) - hm, gx = (int)(e % side) - hm;
    const double r2 = (double)((long long)gx * gx + (long long)gy * gy);
    if (!(r2 >= lo2 && r2 < hi2)) continue;
    const long long i0 = (long long)(gy < 0 ? gy + n : gy) * n + (gx < 0 ? gx + n : gx);
    const long long i1 = (long long)(gy > 0 ? n - gy : -gy) * n + (gx > 0 ? n - gx : -gx);
    m = fmaxf(m, fabsf(0.5f * (c[i0] + c[i1])));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void __launch_bounds__(kBlock)
model_combine_kernel(int ntrip, const double* __restrict__ Fp, const double* __restrict__ Fm,
                     const double* __restrict__ F0, const unsigned* __restrict__ cmax_bits,
                     const unsigned long long* __restrict__ wmin_bits, double f, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntrip) return;
  const double cm = (double)__uint_as_float(*cmax_bits);
  const double t2 = 0.5 * cm * cm * (Fp[t] + Fm[t] - 2.0 * F0[t]);
  const double wm = __longlong_as_double((long long)*wmin_bits);
  out[t] = F0[t] < 0.5 * wm * wm * wm ? __builtin_nan("") : 2.0 * f * t2 / F0[t];
}

// Workspace of abs_model_discrete: the counts workspace, then three count vectors and the
// largest |C|.
struct ModelWork {
  size_t counts, fp, fm, f0, cmax, total;
};
ModelWork model_layout(const abs_plan_s* p) {
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  ModelWork m{};
  size_t off = 0;
  m.counts = off;
  off = al(off + work_layout(p, 0, 0, 0).total);
  m.fp = off;
  off = al(off + (size_t)p->ntrip * 8);
  m.fm = off;
  off = al(off + (size_t)p->ntrip * 8);
  m.f0 = off;
  off = al(off + (size_t)p->ntrip * 8);
  m.cmax = off;
  off = al(off + 4);
  m.total = off;
  return m;
}

}  // namespace abs_impl

using namespace abs_impl;

extern "C" {

abs_status abs_rebin_table(abs_plan_t p, int32_t nl1, const double* l1_edges, int32_t nmu, int32_t nt,
                           int32_t* bin_of_triplet) {
  if (!p || nl1 < 1 || !l1_edges || nmu < 1 || nt < 1 || !bin_of_triplet) return ABS_ERR_INVALID;
  if ((int64_t)nl1 * nmu * nt > 0x7fffffffLL) return ABS_ERR_INVALID;
  for (int b = 0; b < nl1; ++b)
    if (!(l1_edges[b + 1] > l1_edges[b])) return ABS_ERR_INVALID;
  for (int64_t t = 0; t < p->ntrip; ++t) {
    const double* L = &p->labels[5 * t];
    const double l1 = L[0], mu = L[3], tt = L[4];
    int lb = -1;
    for (int b = 0; b < nl1; ++b)
      if (l1 >= l1_edges[b] && l1 < l1_edges[b + 1]) {
        lb = b;
        break;
      }
    if (lb < 0) {
      bin_of_triplet[t] = -1;
      continue;
    }
    // inner edges 0.5 + 0.5 m / nbins in FP64; the bin counts the edges at or below the label
    int mb = 0, tb = 0;
    for (int m = 1; m < nmu; ++m) mb += mu >= 0.5 + 0.5 * m / nmu;
    for (int m = 1; m < nt; ++m) tb += tt >= 0.5 + 0.5 * m / nt;
    bin_of_triplet[t] = (lb * nmu + mb) * nt + tb;
  }
  return ABS_OK;
}

abs_status abs_rebin(abs_plan_t p, int32_t nbins, const int32_t* bin_of_triplet, int32_t batch,
                     const double* B, const double* N, double* Bbin, double* Nbin, void* stream) {
  if (!p || nbins < 1 || !bin_of_triplet || batch < 1 || !B || !N || !Bbin || !Nbin) return ABS_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const dim3 g((unsigned)((nbins + kBlock - 1) / kBlock), (unsigned)batch);
  rebin_kernel<<<g, kBlock, 0, st>>>((int)p->ntrip, nbins, bin_of_triplet, B, N, Bbin, Nbin);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

abs_status abs_ensemble(int32_t nreal, int32_t nvals, const double* X, const double* model, double* mean,
                        double* sigma, double* dB, double* dsigma, void* stream) {
  if (nreal < 1 || nvals < 1 || !X || !mean || !sigma) return ABS_ERR_INVALID;
  if ((dB || dsigma) && !model) return ABS_ERR_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  ensemble_kernel<<<(unsigned)((nvals + kBlock - 1) / kBlock), kBlock, 0, st>>>(nreal, nvals, X, model, mean,
                                                                                sigma, dB, dsigma);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

abs_status abs_model_workspace(abs_plan_t p, size_t* bytes) {
  if (!p || !bytes) return ABS_ERR_INVALID;
  *bytes = model_layout(p).total;
  return ABS_OK;
}

abs_status abs_model_discrete(abs_plan_t p, const float* w, const float* c, double f, void* work,
                              size_t work_bytes, double* out, void* stream) {
  if (!p) return ABS_ERR_INVALID;
  abs_status s = ensure_device(p);
  if (s != ABS_OK) return s;
  if (!c || !work || !out || (!w && p->wmode != ABS_W_UNIT)) return ABS_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(work) & 255) return ABS_ERR_INVALID;
  if (p->nchan > 1) return ABS_ERR_INVALID;   // the model of Eq. (14) is a single-frequency one
  const ModelWork ml = model_layout(p);
  if (work_bytes < ml.total) return ABS_ERR_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wk = static_cast<char*>(work);
  unsigned* cmax = reinterpret_cast<unsigned*>(wk + ml.cmax);
  (void)hipGetLastError();
  zero_u32_kernel<<<1, 64, 0, st>>>(cmax);
  cmax_kernel<<<256, kBlock, 0, st>>>(c, p->n, p->hmax, p->lo2[0], p->hi2[p->nb - 1], cmax);
  if (hipGetLastError() != hipSuccess) return ABS_ERR_DEVICE;
  double* F[3] = {reinterpret_cast<double*>(wk + ml.fp), reinterpret_cast<double*>(wk + ml.fm),
                  reinterpret_cast<double*>(wk + ml.f0)};
  const double sgn[3] = {1.0, -1.0, 0.0};
  const WorkLayout cl = work_layout(p, 0, 0, 0);
  for (int r = 0; r < 3; ++r) {
    WeightMod mod;
    mod.c = c;
    mod.cmax_bits = cmax;
    mod.sgn = sgn[r];
    if ((s = counts_into(p, w, wk + ml.counts, r < 2 ? &mod : nullptr, F[r], st)) != ABS_OK) return s;
  }
  // the unmodulated run (last) left its smallest ring-cell weight in the counts workspace
  const unsigned long long* wmin = reinterpret_cast<const unsigned long long*>(wk + ml.counts + cl.wmin);
  model_combine_kernel<<<(unsigned)((p->ntrip + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      (int)p->ntrip, F[0], F[1], F[2], cmax, wmin, f, out);
  return hipGetLastError() == hipSuccess ? ABS_OK : ABS_ERR_DEVICE;
}

}  // extern "C"
