// Internal state of an abs plan and the launch helpers shared by the HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/abs.h"

namespace abs_impl {

constexpr int kBlock = 256;          // threads per workgroup for most kernels here

// Workgroup i of a launch runs on XCD i % 8 (each XCD has its own L2).  xcd_block maps
// it to a logical block so that every XCD takes runs of kXcdRun consecutive logical
// blocks, interleaved with the other XCDs' runs: neighbouring blocks that write parts of
// the same cache lines then do so through one L2.  The grid is padded to a multiple of
// 8 kXcdRun blocks (xcd_grid); logical blocks past the real count return at once.
constexpr unsigned kXcds = 8, kXcdRun = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned bid) {
  const unsigned grp = bid / (kXcds * kXcdRun), r = bid - grp * (kXcds * kXcdRun);
  return grp * (kXcds * kXcdRun) + (r % kXcds) * kXcdRun + r / kXcds;
}
inline unsigned xcd_grid(long long nblk) {
  const long long g = (long long)kXcds * kXcdRun;
  return (unsigned)((nblk + g - 1) / g * g);
}
// Threads per column-pass workgroup (f32: FP32 data fields, else FP64 weight fields) and
// the FFT engine's block, from which the threads per transform follow (Fft<n, engine>):
// 4096-point columns run two 256-thread transforms in a 512-thread workgroup, so that a
// tile's outputs leave in 64-byte runs instead of 32 (4.7 -> 2.6 ms at 4096^2 x 16; four
// transforms in 1024 threads measured slower, 1.39 against 1.08 ms at 4096^2 x 16), and so
// do FP32 8192-point columns, two transforms in 141 KB of LDS (8.7 -> 5.6 ms at 8192^2 x 8;
// one transform a workgroup, 32-byte runs: 7.6 ms).  8192-point transforms take 512 threads
// (one butterfly each): their LDS leaves one workgroup per CU, so this doubles its waves
// (FP32, 1024 threads: 5.22 -> 4.90 ms at 8192^2 x 8; FP64, one transform in 512 threads:
// 1.29 -> 1.12 ms).  Others kBlock (four 2048-point transforms in 512 threads: no gain).
// The host's column tiles hold as many columns as one workgroup transforms at once.
constexpr int col_block(int log2n, bool f32) { return log2n == 13 && f32 ? 1024 : log2n == 12 || log2n == 13 ? 512 : kBlock; }
constexpr int col_engine(int log2n, bool f32) { (void)f32; return log2n == 12 || log2n == 13 ? 512 : kBlock; }
constexpr int kMaxBins = 64;
constexpr int kTilesPerWave = 12;    // MFMA output tiles owned by one wave (precision form)
constexpr int kSmallTilesPerWave = 2;   // the same for small plans (kernel variant)
constexpr int kMaxN = 8192;

// One contiguous run of uv columns gx0 .. gx0 + ncols - 1 of ring m, transformed
// together by one workgroup of the column pass.
struct ColTile {
  int32_t m, gx0, ncols, pad;
};

// Per-ring constants on the device.
struct BinDev {
  int32_t d2lo, d2hi; // a cell is in the ring when d2lo <= |g|^2 < d2hi (the squared edges
                      // lo2 <= |g|^2 < hi2 rounded up: |g|^2 is an integer)
  int32_t h;          // largest |gx| of any cell of the ring (columns 0..h are used)
  int32_t cols;       // h + 1, or 0 for a ring without lattice cells
  int64_t zoff;       // offset (complex elements) of the ring's column-pass output in one set
};

// Offsets (bytes) of the tables inside the caller's plan memory.
struct DevLayout {
  size_t tw, tw64, bins, tiles, tiles64;
  size_t pt_pairs, mt_ptile, mt_bins, mt_trip, wave_tiles;   // precision-form tables
  size_t pos32, pos64;   // position of each triplet in the FP32 / FP64 kernel's partials
  size_t tmap;           // level plans: index of each of their triplets in the parent's list
  size_t total;
};

// Offsets (bytes) of the buffers inside the abs_estimate workspace.
// One separately compiled piece of the contraction: a run of slices of one kernel kind.
struct JitPart {
  int kind = 0;                  // 0: FP32 data fields, 1: FP64 weight fields
  int z0 = 0, z1 = 0;            // slices [z0, z1) of that kind
  std::string src;               // generated source
  std::vector<char> code;        // code object
  bool compiled = false;
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
};

struct WorkLayout {
  int nsets;          // D sets followed by I sets
  int ndsets;         // D sets (spg per grid)
  int nisets;
  int npsets;         // contraction partial sets of the data (ndsets / nchan)
  int nipsets;        // and of the weights (nisets / nchan)
  size_t zd, zi, fd, fi, part, part64, fmax, wmin, xc, total;
  int64_t zset;       // complex elements per set of column-pass output
  int64_t fset;       // values per set of data fields (nbins * n * n)
  int64_t fset64;     // values per set of weight fields (nbins * npix64)
  int64_t partset;    // doubles per data set of contraction partials (nblk * ntrip)
  int64_t partset64;  // doubles per weight set (nblk64 * ntrip)
  // plans with resolution levels: each level's own layout (its xc and wmin unused) and
  // its offset in the workspace; xc and wmin above are the parent's
  std::vector<WorkLayout> lv;
  std::vector<size_t> lvbase;
};

}  // namespace abs_impl

struct abs_plan_s {
  // descriptor
  int n = 0, nb = 0, log2n = 0;
  // Multi-frequency plans: nchan channels of the same rings; every data set of a call is
  // one channel of one multi-frequency grid (channel-major), the FFT passes transform each
  // channel's nb rings, and the contraction runs over nbc = nchan * nb "channel rings"
  // s = c * nb + r (ring r of channel c), which are contiguous in memory because the
  // channels' fields are consecutive sets.  Single-frequency plans have nchan = 1.
  int nchan = 1, nbc = 0;
  double du = 1.0, norm = 0.0, theta0 = 0.0;
  int precision = 0, wmode = 0, max_batch = 1;
  uint32_t flags = 0;
  std::vector<double> edges, lo2, hi2;
  // rings
  std::vector<int> h, cols;
  int hmax = 0;                  // largest h over the rings (extent of the Hermitian part)
  std::vector<int64_t> zoff;     // complex elements, per ring, within one set
  int64_t ncols = 0;             // sum of cols
  std::vector<double> radius;    // mean |g| per ring
  // triplets, ascending (i, j, k)
  std::vector<int32_t> trips;    // 3 * ntrip
  std::vector<double> labels;    // 5 * ntrip
  int64_t ntrip = 0, npairs = 0;
  // FFT tiling
  int ct = 0, ct64 = 0;          // columns per column-pass block (FP32 data, FP64 weights)
  std::vector<abs_impl::ColTile> tiles, tiles64;
  // precision form: 16-pair row tiles, 16 x 16 MFMA tiles and their owner waves
  std::vector<int> pt_pairs;     // 2 * 16 per row tile: (j, k), padding rows (nb, nb)
  std::vector<int> mt_ptile;     // row tile of each MFMA tile
  std::vector<int> mt_bins;      // 16 ring columns per MFMA tile, padding nb
  std::vector<int> mt_trip;      // 256 per MFMA tile: triplet index or -1
  std::vector<int> wave_tiles;   // 2 per wave: first tile, count
  int mfma_groups = 0;           // workgroups (of 8 waves) per pixel block and set
  int mfma_tpw = 0;              // tiles per wave of the kernel variant the plan uses
  int mfma_depth = 1;            // chunks of loads in flight in that variant
  // precision forms: whether this plan's data contraction runs on the matrix units; a plan
  // (or level) whose triplets fill few tiles is cheaper in the FP32 VALU kernel, which is
  // also more accurate, so it takes that one (see use_mfma_for)
  bool use_mfma = false;
  // contraction kernel (compiled at run time for this triplet list)
  int ngroups = 0;               // wave groups of the FP32 kernel; one wave per group
  int ngroups64 = 0;             // wave groups of the FP64 kernel (weight fields)
  int waves = 4, waves64 = 4;    // waves (groups) per workgroup of the two kernels
  bool jk32 = false, jk64 = false;   // triplets formed as (D_j D_k) D_i (else (D_i D_j) D_k)
  int block32 = 0, block64 = 0;      // triplet order in blocks of this many j (0: none)
  std::vector<int> pos32, pos64; // position of each triplet in the kernels' triplet orders
  int pix_per_block = 0;         // pixels per contraction workgroup (data sets)
  int nblk = 0;                  // contraction pixel blocks per data set
  int pix_per_block64 = 0;       // the same for the FP64 weight sets (fewer sets: smaller blocks)
  int nblk64 = 0;
  // Weight fields are even (I(-x, -y) = I(x, y): the weights are real and symmetric), so
  // only rows 0 .. n/2 are formed, per ring in npix64 values: block 0 holds rows 0 and
  // n/2 (then zeros), blocks 1 .. nblk64 - 1 rows 1 .. n/2 - 1 (then zeros); the sum over
  // all pixels is block 0 plus twice the others.
  int64_t npix64 = 0;
  std::vector<abs_impl::JitPart> parts;   // contraction code, compiled per part
  // Resolution levels.  A triplet i <= j <= k with h_i + h_j + h_k < m and 2 h_k < m (h:
  // a ring's largest |g_x|) closes exactly the same triangles on an m x m periodic grid
  // as on the n x n one (a sum of three of its cells is zero modulo m only if it is zero),
  // and its ring fields on the m grid are those on the n grid sampled every n/m pixels.
  // Such a plan runs its triplets in level plans (`lv`, largest m first), each over m^2
  // pixels with the rings ring0 .. ring0 + nb - 1 its triplets use (renumbered from 0);
  // the parent forms the Hermitian part once (its hmax covers every level) and the
  // smallest ring weight over all rings (for the empty-triplet rule), and owns no kernel
  // code of its own.
  int max_ratio = 1;                     // largest n / m allowed for a level
  bool is_level = false;                 // a level plan of some parent
  int ring0 = 0;                         // level plan: the parent's index of its ring 0
  std::vector<abs_plan_s*> lv;           // level plans (empty: the plan runs at n itself)
  std::vector<int32_t> tmap;             // level plan: parent index of each of its triplets
  int xc_hm = 0;                         // half extent of the Hermitian part its column pass reads
  size_t dev_off = 0;                    // level plan: offset of its tables in the parent's memory
  // device binding
  abs_impl::DevLayout dl{};
  void* dev = nullptr;
  int device = -1;
  // A second stream (default priority, created by abs_plan_bind on the plan's device) and
  // two events: an estimate's weight sets run there beside its data sets, forked after
  // the call's first launch on the caller's stream and joined before its normalisation.
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  int aux_device = -1;
  // timing hook: events recorded around one stage's launches (see abs_profile)
  hipEvent_t prof[4][2] = {};
};

namespace abs_impl {
// A modulation of the weights for the model's discrete prediction: every weight-set cell's
// Y(g) becomes Y(g) (1 + sgn Cs(g) / cmax), Cs(g) = (c(g) + c(-g)) / 2, cmax = the float
// whose bits *cmax_bits holds (on the device).
struct WeightMod {
  const float* c = nullptr;
  const unsigned* cmax_bits = nullptr;
  double sgn = 0.0;
};
// plan.cpp
bool build_jit_source(abs_plan_s* p);
abs_status compile_jit(abs_plan_s* p, int part);
uint64_t jit_key(const abs_plan_s* p, int part);
// The plans that run kernels: the level plans, or the plan itself.
inline std::vector<abs_plan_s*> run_plans(abs_plan_s* p) {
  return p->lv.empty() ? std::vector<abs_plan_s*>{p} : p->lv;
}
inline std::vector<const abs_plan_s*> run_plans(const abs_plan_s* p) {
  if (p->lv.empty()) return {p};
  return std::vector<const abs_plan_s*>(p->lv.begin(), p->lv.end());
}
// Part `k` of the plan's code counted over its run plans: the owning plan and the index
// there (nullptr when out of range).
abs_plan_s* part_owner(abs_plan_s* p, int k, int* local);
void destroy_plan(abs_plan_s* p);
// Destroys the plan's second stream and its events (on the device they belong to).
void release_aux(abs_plan_s* p);
WorkLayout work_layout(const abs_plan_s* p, int grids, int w_batched, int have_counts, int spg = 1);
void build_mfma_tables(abs_plan_s* p);
// estimate.hip
abs_status ensure_device(abs_plan_s* p);
abs_status counts_into(abs_plan_s* p, const float* w, char* wk, const WeightMod* mod, double* N,
                       hipStream_t st);
inline void prof_begin(const abs_plan_s* p, int stage, hipStream_t st) {
  if (p->prof[stage][0]) (void)hipEventRecord(p->prof[stage][0], st);
}
inline void prof_end(const abs_plan_s* p, int stage, hipStream_t st) {
  if (p->prof[stage][1]) (void)hipEventRecord(p->prof[stage][1], st);
}
}  // namespace abs_impl
