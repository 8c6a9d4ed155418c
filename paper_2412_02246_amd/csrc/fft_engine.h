// Compile-time-length complex FFT engine shared by the ring-field passes (fft.hip) and
// the sky-to-visibility transform (simulate.hip): self-sorting Stockham passes of
// radix 16 (then one radix-2, 4 or 8 pass), n/16 threads a transform (two butterflies a
// thread when n/16 exceeds the workgroup), exchanging data through a padded LDS buffer.
// The sign is the forward one, exp(-2 pi i j k / n).  Callers supply the first pass's
// inputs (in) and take the last pass's outputs (out), so loads and stores can be fused
// with whatever the caller does around the transform.
#pragma once

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

// ---------------------------------------------------------------------------------
// Compile-time-length engine (used by the row pass).  With n fixed every LDS address is
// the thread's base plus a constant, each thread's twiddles are fixed for the kernel's
// lifetime (kept in registers when they are few) and the first pass reads its inputs
// straight from global memory, skipping all-zero slabs of the pruned input.
template <int LOG2N, int BLOCK = kBlock>
struct Fft {
  static constexpr int N = 1 << LOG2N;
  static constexpr int U = N / 16 > BLOCK ? 2 : 1;            // radix-16 butterflies per thread
  static constexpr int TG = N / 16 / U < BLOCK ? N / 16 / U : BLOCK;   // threads per transform
  static constexpr int G = BLOCK / TG;                        // transforms per block
  static constexpr int NP16 = LOG2N / 4, LREST = LOG2N % 4;
  static constexpr int NPASS = NP16 + (LREST ? 1 : 0);
  static constexpr int L = N + N / 16;                        // padded LDS elements
  static constexpr bool WAVE = TG <= 64;                      // one wave holds whole transforms
  static constexpr int lrp(int p) { return p < NP16 ? 4 : LREST; }
  static constexpr int nb(int p) { return 16 * U / (1 << lrp(p)); }
  // twiddles of passes 1 .. p - 1 (pass 0 has none)
  static constexpr int tw_before(int p) {
    int c = 0;
    for (int q = 1; q < p; ++q) c += nb(q) * ((1 << lrp(q)) - 1);
    return c;
  }
  static constexpr int NTW = tw_before(NPASS);
};

// Orders a transform's LDS traffic between passes: a wave-level fence when one wave
// holds whole transforms (LDS serves one wave's operations in order), else a barrier.
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Per-thread twiddles held in registers (REG = true, the only form defined here), loaded
// once per block; transforms that need more take TwiddlesSplit below.
template <typename R, int LOG2N, bool REG, int BLOCK = kBlock>
struct Twiddles;
template <typename R, int LOG2N, int BLOCK>
struct Twiddles<R, LOG2N, true, BLOCK> {
  using T = typename Cx<R>::T;
  using F = Fft<LOG2N, BLOCK>;
  T w[F::NTW > 0 ? F::NTW : 1];
  __device__ __forceinline__ void load(const T* __restrict__ tw, int t) {
    load_from<1>(tw, t);
  }
  template <int P>
  __device__ __forceinline__ void load_from(const T* __restrict__ tw, int t) {
    if constexpr (P < F::NPASS) {
      constexpr int LRP = F::lrp(P), RP = 1 << LRP, LNS = 4 * P, SH = LOG2N - LNS - LRP;
#pragma unroll
      for (int j = 0; j < F::nb(P); ++j) {
        const int m = (t + F::TG * j) & ((1 << LNS) - 1);
#pragma unroll
        for (int r = 1; r < RP; ++r) w[F::tw_before(P) + j * (RP - 1) + r - 1] = tw[(r * m) << SH];
      }
      load_from<P + 1>(tw, t);
    }
  }
  template <int P>
  __device__ __forceinline__ T get(const T* __restrict__, int, int j, int r) const {
    return w[F::tw_before(P) + j * ((1 << F::lrp(P)) - 1) + r - 1];
  }
};

// Twiddles from LDS tables (row passes, and column passes whose threads need more twiddles
// than registers hold).  Pass 1, when it is radix 16, reads its twiddles straight from a
// 16 x 15 table: thread t's butterflies there have m = t mod 16, so entry [m][r - 1] is
// w^(r m 2^SH1) and the 15 reads of a butterfly take one base address and immediate
// offsets, with no index arithmetic or product.  Pass 2, when it is radix 16 too and a
// transform has a multiple of 256 threads, has m = t mod 256 = m0 + 16 m1, and its twiddle
// w^(r m 2^SH2) (SH2 = SH1 - 4) is the product of w^(r m0 2^SH2), from a second 16 x 15
// table, and w^(r m1 2^SH1), from the first.  (These tables take an 8192-point row transform
// from 1362 to 1180 VALU instructions, the FFT passes being bound by VALU issue.)  Later
// passes use a two-level table:
// w^a = hi[a / LO] lo[a % LO] with lo[c] = w^c (c < LO = min(64, N)) and hi[b] = w^(LO b)
// (b < N / LO), so one complex product (about one rounding more than the table entry)
// replaces a load from memory.  All tables are copied from the plan's natural-order table.
template <typename R, int LOG2N, int BLOCK = kBlock>
struct TwiddlesSplit {
  using T = typename Cx<R>::T;
  using F = Fft<LOG2N, BLOCK>;
  static constexpr int LLO = LOG2N < 6 ? LOG2N : 6, LO = 1 << LLO;
  // pass 1 direct: radix 16 there, and m = (t + TG j) mod 16 = t mod 16 (TG a multiple of 16)
  static constexpr bool P1 = F::NPASS > 1 && F::lrp(1) == 4 && F::TG % 16 == 0;
  static constexpr bool P2 = P1 && F::NPASS > 2 && F::lrp(2) == 4 && F::TG % 256 == 0;
  static constexpr int SH1 = LOG2N - 8;
  static constexpr int N1 = P1 ? 16 * 15 : 0, N2 = P2 ? 16 * 15 : 0;
  static constexpr int T1 = LO + F::N / LO, T2 = T1 + N1;   // offsets of the two tables
  static constexpr int ENTRIES = T2 + N2;
  const T* lo;   // LDS: lo[LO], hi[N / LO], then the pass-1 and pass-2 tables
  // Copies the tables from the natural-order table tw (N entries) into LDS at dst; the
  // caller synchronises the block before the first get.
  __device__ __forceinline__ void stage(const T* __restrict__ tw, T* dst, int tid, int nthreads) {
    for (int e = tid; e < ENTRIES; e += nthreads) {
      int src;
      if (e < LO) {
        src = e;
      } else if (e < T1) {
        src = (e - LO) * LO;
      } else {
        const int b = e < T2 ? T1 : T2;   // pass-1 table: 2^SH1 steps; pass-2 table: 2^(SH1 - 4)
        const int m = (e - b) / 15, r = (e - b) - 15 * m + 1;
        src = e < T2 ? (r * m) << (P1 ? SH1 : 0) : (r * m) << (P2 ? SH1 - 4 : 0);
      }
      dst[e] = tw[src];
    }
    lo = dst;
  }
  template <int P>
  __device__ __forceinline__ T get(const T* __restrict__, int t, int j, int r) const {
    constexpr int LRP = F::lrp(P), LNS = 4 * P, SH = LOG2N - LNS - LRP;
    if constexpr (P == 1 && P1) {
      return lo[T1 + 15 * (t & 15) + r - 1];
    } else if constexpr (P == 2 && P2) {
      return cmul(lo[T2 + 15 * (t & 15) + r - 1], lo[T1 + 15 * ((t >> 4) & 15) + r - 1]);
    } else {
      const int m = (t + F::TG * j) & ((1 << LNS) - 1);
      const int a = (r * m) << SH;   // < N
      return cmul(lo[LO + (a >> LLO)], lo[a & (LO - 1)]);
    }
  }
};

// Pass P of the length-2^LOG2N transform held by thread t of its TG threads.  Pass 0
// takes its inputs from in(k) (natural order, any memory); the last pass hands its
// outputs to out(k, value); passes in between read and write the padded LDS buffer.
template <typename R, int LOG2N, int P, int BLOCK, class TW, class In, class Out>
__device__ __forceinline__ void fft_pass(typename Cx<R>::T* buf, int t, const typename Cx<R>::T* __restrict__ tw,
                                         const TW& twr, In& in, Out& out) {
  using T = typename Cx<R>::T;
  using F = Fft<LOG2N, BLOCK>;
  constexpr int LRP = F::lrp(P), RP = 1 << LRP, NB = F::nb(P);
  constexpr int LNS = 4 * P, NS = 1 << LNS, STRIDE = F::N / RP;
  constexpr bool FIRST = P == 0, LAST = P == F::NPASS - 1;
  T v[NB][RP];
  if constexpr (FIRST) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < RP; ++r) v[j][r] = in(t + F::TG * j + r * STRIDE, j, r);
  } else {
    static_assert(STRIDE % 16 == 0, "padded reads need a stride that is a multiple of 16");
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int lb = lpad(t + F::TG * j);
#pragma unroll
      for (int r = 0; r < RP; ++r) v[j][r] = buf[lb + r * (STRIDE + STRIDE / 16)];
    }
    if constexpr (!LAST) fft_sync<F::WAVE>();   // every read of this pass precedes every write
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if constexpr (!FIRST) {
#pragma unroll
      for (int r = 1; r < RP; ++r) v[j][r] = cmul(v[j][r], twr.template get<P>(tw, t, j, r));
    }
    dft<R, RP>(v[j]);
    const int b = t + F::TG * j;
    const int idxD = ((b >> LNS) << (LNS + LRP)) + (b & (NS - 1));
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RP; ++q) out(idxD + q * NS, j, q, v[j][q]);
    } else if constexpr (FIRST) {
      // k = 16 b + q: lpad(k) = 17 b + q
#pragma unroll
      for (int q = 0; q < RP; ++q) buf[17 * b + q] = v[j][q];
    } else {
      const int lb = lpad(idxD);
#pragma unroll
      for (int q = 0; q < RP; ++q) buf[lb + q * (NS + NS / 16)] = v[j][q];
    }
  }
  if constexpr (!LAST) fft_sync<F::WAVE>();
}

template <typename R, int LOG2N, int P, int BLOCK, class TW, class In, class Out>
__device__ __forceinline__ void fft_passes(typename Cx<R>::T* buf, int t, const typename Cx<R>::T* __restrict__ tw,
                                           const TW& twr, In& in, Out& out) {
  fft_pass<R, LOG2N, P, BLOCK>(buf, t, tw, twr, in, out);
  if constexpr (P + 1 < Fft<LOG2N, BLOCK>::NPASS) fft_passes<R, LOG2N, P + 1, BLOCK>(buf, t, tw, twr, in, out);
}

}  // namespace abs_impl
