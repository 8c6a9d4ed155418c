// Precision form of the triplet contraction (Eq. 12 numerator) on the gfx950 matrix cores.
//
// For a chunk of K pixels the sums S_(ij)k = sum_theta P_ij(theta) D_k(theta), with pair
// products P_ij = D_i D_j, form a (pairs x K) by (K x rings) matrix product.  Both
// operands are split into two 16-bit halves, x = hi + lo (BF16, or FP16 after scaling every
// ring by a power of two so that its largest |value| lies in [64, 128)), and each 16 x 16 output tile
// accumulates hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_{bf16,f16} in FP32; the lo*lo term
// is below the split's own rounding.  Each chunk's products start from zero and are then
// added to the tile's running FP32 sum (long FP32 accumulation chains, not the split,
// otherwise dominate the error); tile sums over a workgroup's pixels are written as FP64
// partials per triplet, in the same layout as the FP32 path, so the FP64 finaliser is
// shared.
//
// Tiles are block-sparse: each triplet i <= j <= k is the pair product D_j D_k of its two
// largest rings times its smallest ring D_i; pairs ordered by (j, k) are cut into row
// tiles of 16, and each row tile only multiplies against the rings i that close a triangle
// with one of its pairs (16 columns per MFMA tile; absent rows / columns point at a zero
// row of LDS).  Output entries that are not plan triplets are computed and dropped.
//
// Workgroup: 8 waves; blockIdx.x = pixel block, blockIdx.y = set, blockIdx.z = wave
// group.  Per chunk of kChunk pixels the workgroup stages the rings' FP32 values and their
// hi/lo halves in LDS; each wave then evaluates its MFMA tiles (at most TPW,
// accumulators in registers across the whole pixel block).  Variants: TPW = kTilesPerWave
// with DEPTH chunks of loads in flight (4 for up to 32 rings, 1 above), and for small
// plans TPW = kSmallTilesPerWave, whose 128 registers a lane let two workgroups share a
// CU, so one workgroup's staging and barriers overlap the other's matrix work.  The A
// operand (the row tile's pair products, split) is formed once per chunk and kept for the
// wave's consecutive tiles of that row tile; the B operand likewise while the columns stay
// the same.
#include "abs_internal.h"

namespace abs_impl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaThreads = 512;
constexpr int kChunk = 128;                 // pixels staged per step (4 MFMA k-steps of 32)
// Padded LDS row lengths (elements).  Half-precision rows of 144 (288 bytes) read with
// fewer bank conflicts than rows of 136 in the column operand's loads (8192^2 x 16 BF16x3:
// 89.4 against 91.1 ms; 4096^2: 7.37 against 7.60 ms); FP32 rows of 136 or 140 gain nothing.
constexpr int kRow32 = kChunk + 4;
constexpr int kRow16 = kChunk + 16;
// FP16 scaling: every ring is scaled by a power of two to a largest |value| in
// [2^(kF16Exp-1), 2^kF16Exp); pair products then stay below 2^14 < 65504 and their low
// halves stay clear of the FP16 subnormal range for all but negligible terms.
constexpr int kF16Exp = 7;

template <bool F16> struct Half;
template <> struct Half<false> {
  using T = __bf16;
  using V = bf16x8;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Half<true> {
  using T = _Float16;
  using V = f16x8;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Pair products p = a[q] b[q] of 8 pixels split into p ~ hi + lo, both 16-bit.  BF16: hi
// is p truncated to its upper 16 bits (the two halves of two products packed by one byte
// permute), lo = a b - hi (fused, exact up to one rounding) rounded to BF16: about four
// VALU operations a product.  FP16: hi = fl16(a b) and lo = fl16(a b - hi), each one
// mixed-precision FMA: two operations a product.
template <bool F16>
__device__ __forceinline__ void split8(const float* a, const float* b, typename Half<F16>::V& hi,
                                       typename Half<F16>::V& lo) {
  const f32x4 a0 = *reinterpret_cast<const f32x4*>(a), a1 = *reinterpret_cast<const f32x4*>(a + 4);
  const f32x4 b0 = *reinterpret_cast<const f32x4*>(b), b1 = *reinterpret_cast<const f32x4*>(b + 4);
  const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
  if constexpr (!F16) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    u32x4 hw, lw;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float p0 = av[2 * q] * bv[2 * q], p1 = av[2 * q + 1] * bv[2 * q + 1];
      const unsigned u0 = __float_as_uint(p0), u1 = __float_as_uint(p1);
      hw[q] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);   // upper halves of p1 : p0
      const float l0 = __builtin_fmaf(av[2 * q], bv[2 * q], -__uint_as_float(u0 & 0xffff0000u));
      const float l1 = __builtin_fmaf(av[2 * q + 1], bv[2 * q + 1], -__uint_as_float(u1 & 0xffff0000u));
      typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
      const bf16x2 lp = {(__bf16)l0, (__bf16)l1};
      lw[q] = __builtin_bit_cast(unsigned, lp);
    }
    hi = __builtin_bit_cast(typename Half<F16>::V, hw);
    lo = __builtin_bit_cast(typename Half<F16>::V, lw);
  } else {
    // two products a packed register: hi = fl16(a b) and lo = fl16(a b - hi), each one
    // mixed-precision FMA writing one half; the second product's lo reads its hi from the
    // upper half (op_sel), so no separate copy of it is made.  One block for all eight
    // products: the compiler's hazard tracking does not see into it, so it ends with the
    // two wait states a matrix instruction needs before reading a VGPR that a VALU
    // operation has just written.
    unsigned h0, h1, h2, h3, l0, l1, l2, l3;
#define ABS_MIX2(H, L, A0, B0, A1, B1)                                            \
  "v_fma_mixlo_f16 " H ", " A0 ", " B0 ", 0\n\t"                                  \
  "v_fma_mixhi_f16 " H ", " A1 ", " B1 ", 0\n\t"                                  \
  "v_fma_mixlo_f16 " L ", " A0 ", " B0 ", -" H " op_sel_hi:[0,0,1]\n\t"           \
  "v_fma_mixhi_f16 " L ", " A1 ", " B1 ", -" H " op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
    asm(ABS_MIX2("%0", "%4", "%8", "%9", "%10", "%11")
        ABS_MIX2("%1", "%5", "%12", "%13", "%14", "%15")
        ABS_MIX2("%2", "%6", "%16", "%17", "%18", "%19")
        ABS_MIX2("%3", "%7", "%20", "%21", "%22", "%23")
        "s_nop 1"
        : "=&v"(h0), "=&v"(h1), "=&v"(h2), "=&v"(h3), "=&v"(l0), "=&v"(l1), "=&v"(l2), "=&v"(l3)
        : "v"(av[0]), "v"(bv[0]), "v"(av[1]), "v"(bv[1]), "v"(av[2]), "v"(bv[2]),
          "v"(av[3]), "v"(bv[3]), "v"(av[4]), "v"(bv[4]), "v"(av[5]), "v"(bv[5]),
          "v"(av[6]), "v"(bv[6]), "v"(av[7]), "v"(bv[7]));
#undef ABS_MIX2
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 hw = {h0, h1, h2, h3}, lw = {l0, l1, l2, l3};
    hi = __builtin_bit_cast(typename Half<F16>::V, hw);
    lo = __builtin_bit_cast(typename Half<F16>::V, lw);
  }
}

size_t mfma_lds_bytes(int nb) {
  return (size_t)(nb + 1) * (kRow32 * 4 + 2 * kRow16 * 2);
}

template <bool F16, int NBMAX, int DEPTH, int TPW>
__global__ void __launch_bounds__(kMfmaThreads, TPW <= 2 ? 4 : 2)
mfma_contract_kernel(const float* __restrict__ F, long long set_stride, long long npix, int ppb,
                     double* __restrict__ part, int nblk, int ntrip, int nb,
                     const int2* __restrict__ pt_pairs, const int* __restrict__ mt_ptile,
                     const int* __restrict__ mt_bins, const int* __restrict__ mt_trip,
                     const int2* __restrict__ wave_tiles, const unsigned* __restrict__ fmax_bits) {
  using H = Half<F16>;
  using HT = typename H::T;
  using HV = typename H::V;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* d32 = reinterpret_cast<float*>(lds_raw);
  HT* dhi = reinterpret_cast<HT*>(lds_raw + (size_t)(nb + 1) * kRow32 * 4);
  HT* dlo = dhi + (size_t)(nb + 1) * kRow16;

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 15, quad = lane >> 4;
  const long long set = blockIdx.y;
  const float* __restrict__ Fs = F + set * set_stride;
  const long long p0 = (long long)blockIdx.x * ppb;
  const long long p1 = (p0 + ppb < npix) ? p0 + ppb : npix;
  const int2 wr = wave_tiles[blockIdx.z * (kMfmaThreads / 64) + wave];

  // power-of-two scale per ring (FP16 only), from max |F_m| recorded by the row pass:
  // sexp[m] = e with max |F_m| < 2^e (0 for an all-zero ring)
  __shared__ int sexp[kMaxBins + 1];
  const bool scaled = F16 && fmax_bits != nullptr;
  if (threadIdx.x <= nb) {
    int e = 0;
    if (scaled && threadIdx.x < nb) {
      const unsigned b = fmax_bits[set * nb + threadIdx.x];
      e = b ? (int)((b >> 23) & 0xffu) - 126 : 0;
    }
    sexp[threadIdx.x] = e;
  }

  // the zero row
  for (int q = threadIdx.x; q < kRow32; q += blockDim.x) d32[nb * kRow32 + q] = 0.f;
  for (int q = threadIdx.x; q < kRow16; q += blockDim.x) {
    dhi[nb * kRow16 + q] = (HT)0.f;
    dlo[nb * kRow16 + q] = (HT)0.f;
  }
  // sexp (written by the first nb + 1 threads, all in wave 0) is read by every wave while
  // it stages the first chunk, before the chunk loop's first barrier: publish it here
  __syncthreads();

  f32x4 acc[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this lane's row of each tile, packed j | k << 8 | column ring << 16 (rings <= kMaxBins,
  // the zero row included), read once: no global load inside the chunk loop, whose
  // in-order completion count would otherwise also wait for the next chunk's prefetch
  unsigned meta[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    meta[s] = 0;
    if (s < wr.y) {
      const int tile = wr.x + s;
      const int2 ij = pt_pairs[mt_ptile[tile] * 16 + row];
      meta[s] = (unsigned)ij.x | ((unsigned)ij.y << 8) | ((unsigned)mt_bins[tile * 16 + row] << 16);
    }
  }

  // The chunk's global loads are issued DEPTH chunks ahead into registers (DEPTH buffers,
  // used in turn), so that several chunks' loads are in flight while the matrix work runs:
  // with few rings a chunk's work is short and one chunk ahead leaves the memory latency
  // exposed.  Thread q stages the pixel pairs
  // (m, x / 2) = divmod(threadIdx.x + kMfmaThreads * u, kChunk / 2), u < kStage: 8-byte
  // loads, and whole-word LDS stores of the two pixels' values and halves.
  constexpr int kStage = (NBMAX * kChunk / 2) / kMfmaThreads;
  const int nstage = (nb * kChunk / 2 + kMfmaThreads - 1) / kMfmaThreads;
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef HT h16x2 __attribute__((ext_vector_type(2)));
  f32x2 pre[DEPTH][kStage];
  auto load_chunk = [&](f32x2 (&buf)[kStage], long long c0) {
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int q = threadIdx.x + kMfmaThreads * u;
      const int m = q / (kChunk / 2), x = 2 * (q - m * (kChunk / 2));
      // Unconditional loads from clamped addresses: entries past the last ring or past the
      // block end (prefetch beyond the last chunk) are never staged, and loads that are all
      // issued let the compiler wait for one buffer without waiting for the others.
      // Blocks hold whole chunks (p0, p1 multiples of kChunk), p1 - 2 >= p0.
      const int mc = m < nb ? m : nb - 1;
      const long long p = c0 + x;
      const long long pc = p < p1 ? p : p1 - 2;
      buf[u] = *reinterpret_cast<const f32x2*>(Fs + (long long)mc * npix + pc);
    }
  };
#pragma unroll
  for (int b = 0; b < DEPTH; ++b) load_chunk(pre[b], p0 + (long long)b * kChunk);
  for (long long cb = p0; cb < p1; cb += (long long)DEPTH * kChunk) {
#pragma unroll
  for (int b = 0; b < DEPTH; ++b) {
    // Every phase runs, also past the block end (only blocks shorter than DEPTH chunks
    // have such phases; they stage zeros, which add nothing): no path skips a phase's
    // loads, so the compiler can wait for one buffer while the later ones stay in flight.
    const long long c0 = cb + (long long)b * kChunk;
    const bool live = c0 < p1;
    // stage the chunk: FP32 values (scaled for FP16) and their hi / lo halves
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int q = threadIdx.x + kMfmaThreads * u;
      const int m = q / (kChunk / 2), x = 2 * (q - m * (kChunk / 2));
      if (u < nstage && m < nb) {
        f32x2 v = live ? pre[b][u] : f32x2{0.f, 0.f};
        if (scaled) {
          v.x = ldexpf(v.x, kF16Exp - sexp[m]);
          v.y = ldexpf(v.y, kF16Exp - sexp[m]);
        }
        const h16x2 h = {(HT)v.x, (HT)v.y};
        const h16x2 l = {(HT)(v.x - (float)h.x), (HT)(v.y - (float)h.y)};
        *reinterpret_cast<f32x2*>(d32 + m * kRow32 + x) = v;
        *reinterpret_cast<h16x2*>(dhi + m * kRow16 + x) = h;
        *reinterpret_cast<h16x2*>(dlo + m * kRow16 + x) = l;
      }
    }
    __syncthreads();
    // the buffer is free again: load the chunk DEPTH ahead into it (masked off past p1)
    load_chunk(pre[b], c0 + (long long)DEPTH * kChunk);
    // A operand (the row tile's pair products, split) and B operand (the tile's ring
    // columns, split) for the chunk's kChunk/32 k-steps, each kept while consecutive tiles
    // of the wave use the same rows / columns
    HV ah[kChunk / 32], al[kChunk / 32], bh[kChunk / 32], bl[kChunk / 32];
    unsigned held_rows = ~0u;   // pair (j | k << 8) held by this lane (none yet)
    int held = -1;              // column ring held by this lane (-1: none yet)
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      if (s < wr.y) {
        // opaque copy: keeps the compiler from hoisting the decoded addresses of every
        // tile out of the chunk loop (three live registers a tile instead of one)
        unsigned m = meta[s];
        asm volatile("" : "+v"(m));
        const unsigned rows = m & 0xffffu;
        const int bin = (int)(m >> 16);
        if (__builtin_amdgcn_ballot_w64(rows != held_rows)) {
          const float* dj = d32 + (rows & 0xffu) * kRow32;
          const float* dk = d32 + (rows >> 8) * kRow32;
#pragma unroll
          for (int ks = 0; ks < kChunk / 32; ++ks) {
            const int x0 = ks * 32 + quad * 8;
            split8<F16>(dj + x0, dk + x0, ah[ks], al[ks]);
          }
          held_rows = rows;
        }
        if (__builtin_amdgcn_ballot_w64(bin != held)) {
#pragma unroll
          for (int ks = 0; ks < kChunk / 32; ++ks) {
            const int x0 = ks * 32 + quad * 8;
            bh[ks] = *reinterpret_cast<const HV*>(dhi + bin * kRow16 + x0);
            bl[ks] = *reinterpret_cast<const HV*>(dlo + bin * kRow16 + x0);
          }
          held = bin;
        }
        // the chunk's three split products summed from zero (a chain of 3 kChunk/32
        // MFMA steps), then one FP32 add into the tile's running sum: every FP32
        // accumulation chain stays short
        f32x4 cs = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kChunk / 32; ++ks) {
          cs = H::mma(ah[ks], bh[ks], cs);
          cs = H::mma(ah[ks], bl[ks], cs);
          cs = H::mma(al[ks], bh[ks], cs);
        }
        acc[s] += cs;
      }
    }
    __syncthreads();
  }
  }

  // lane holds C[4 * quad + q][row] of each of its tiles
  double* __restrict__ out = part + (set * nblk + blockIdx.x) * (long long)ntrip;
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    if (s < wr.y) {
      const int tile = wr.x + s;
      const int pt = mt_ptile[tile];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * quad + q;
        const int t = mt_trip[tile * 256 + r * 16 + row];
        if (t >= 0) {
          double v = (double)acc[s][q];
          if (scaled) {
            const int2 ij = pt_pairs[pt * 16 + r];
            const int k = mt_bins[tile * 16 + row];
            v = ldexp(v, sexp[ij.x] + sexp[ij.y] + sexp[k] - 3 * kF16Exp);
          }
          out[t] = v;
        }
      }
    }
  }
}

hipError_t launch_mfma_contract(const abs_plan_s* p, const float* F, long long fset, int nsets,
                                double* part, const unsigned* fmax_bits, hipStream_t st) {
  const char* base = static_cast<const char*>(p->dev);
  const int2* pt_pairs = reinterpret_cast<const int2*>(base + p->dl.pt_pairs);
  const int* mt_ptile = reinterpret_cast<const int*>(base + p->dl.mt_ptile);
  const int* mt_bins = reinterpret_cast<const int*>(base + p->dl.mt_bins);
  const int* mt_trip = reinterpret_cast<const int*>(base + p->dl.mt_trip);
  const int2* wave_tiles = reinterpret_cast<const int2*>(base + p->dl.wave_tiles);
  const size_t lds = mfma_lds_bytes(p->nbc);   // every contraction bin of a set is staged
  const dim3 grid((unsigned)p->nblk, (unsigned)nsets, (unsigned)p->mfma_groups);
  const long long npix = (long long)p->n * p->n;
  // the variant the plan chose (mfma_tpw, mfma_depth): small plans two tiles a wave; up
  // to 32 rings four chunks in flight; larger plans one
  const bool f16 = p->precision == ABS_FP16X3;
  const bool small = p->mfma_tpw == kSmallTilesPerWave, deep = p->mfma_depth == 4;
  if (!small && p->nbc > 32 && deep) return hipErrorInvalidValue;
  auto k = f16 ? (small  ? mfma_contract_kernel<true, 32, 1, kSmallTilesPerWave>
                  : deep ? mfma_contract_kernel<true, 32, 4, kTilesPerWave>
                         : mfma_contract_kernel<true, kMaxBins, 1, kTilesPerWave>)
               : (small  ? mfma_contract_kernel<false, 32, 1, kSmallTilesPerWave>
                  : deep ? mfma_contract_kernel<false, 32, 4, kTilesPerWave>
                         : mfma_contract_kernel<false, kMaxBins, 1, kTilesPerWave>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k<<<grid, kMfmaThreads, lds, st>>>(F, fset, npix, p->pix_per_block, part, p->nblk, (int)p->ntrip, p->nbc,
                                     pt_pairs, mt_ptile, mt_bins, mt_trip, wave_tiles,
                                     f16 ? fmax_bits : nullptr);
  return hipGetLastError();
}

}  // namespace abs_impl
