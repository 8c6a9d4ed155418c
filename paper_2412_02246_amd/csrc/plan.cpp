// Host side of an abs plan: rings, the exact lattice test for ring triplets, labels,
// FFT tiling, the run-time generated contraction kernel and workspace layouts.
//
// Rings and triplets follow Gill et al. (2024): Sec. 2 divides the uv plane into
// annular rings a_m; Sec. 3 evaluates Eq. (12) for every combination of three rings,
// each estimate averaging all closed triangles with one vertex per ring.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <set>
#include <tuple>

#include "abs_internal.h"

using namespace abs_impl;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Ring membership: lo2 <= r2 < hi2 with r2 the exact integer |g|^2 (as a double,
// exact below 2^53) and lo2, hi2 the FP64 squares of the edges.
inline bool in_ring(long long r2, double lo2, double hi2) {
  const double d = static_cast<double>(r2);
  return d >= lo2 && d < hi2;
}

// For column offset x (any sign), the non-negative y with lo2 <= x^2 + y^2 < hi2
// form the integer range [ya, yb] (empty when ya > yb).
void y_range(long long x, double lo2, double hi2, long long& ya, long long& yb) {
  const long long x2 = x * x;
  const double t = hi2 - static_cast<double>(x2);
  ya = 1;
  yb = 0;
  if (t <= 0.0) return;
  long long y = static_cast<long long>(std::floor(std::sqrt(t)));
  while (y >= 0 && !(static_cast<double>(x2 + y * y) < hi2)) --y;
  while (static_cast<double>(x2 + (y + 1) * (y + 1)) < hi2) ++y;
  if (y < 0) return;
  const double u = lo2 - static_cast<double>(x2);
  long long z = u <= 0.0 ? 0 : static_cast<long long>(std::ceil(std::sqrt(u)));
  while (z > 0 && static_cast<double>(x2 + (z - 1) * (z - 1)) >= lo2) --z;
  while (z <= y && static_cast<double>(x2 + z * z) < lo2) ++z;
  ya = z;
  yb = y;
}

struct RingRows {
  long long H = -1;                 // largest |x| holding a cell
  std::vector<long long> ya, yb;    // indexed by |x|, 0..H
};

RingRows ring_rows(double lo2, double hi2) {
  RingRows r;
  long long X = static_cast<long long>(std::floor(std::sqrt(std::max(hi2, 0.0)))) + 1;
  r.ya.resize(X + 1);
  r.yb.resize(X + 1);
  for (long long x = 0; x <= X; ++x) {
    y_range(x, lo2, hi2, r.ya[x], r.yb[x]);
    if (r.ya[x] <= r.yb[x]) r.H = x;
  }
  r.ya.resize(r.H + 1);
  r.yb.resize(r.H + 1);
  return r;
}

inline bool intervals_meet(long long a0, long long a1, long long b0, long long b1) {
  return std::max(a0, b0) <= std::min(a1, b1);
}

// Does the planar lattice hold g1 in ring i, g2 in ring j with g1 + g2 in ring k?
// (Then g3 = -(g1 + g2) lies in ring k as well, the rings being symmetric.)
// The configuration is invariant under the 8 symmetries of the square lattice, so g1
// is restricted to 0 <= y1 <= x1; each candidate g2 column x2 is tested in O(1)
// against the two annulus constraints written as intervals in y2.
bool has_planar_triangle(const RingRows& Ri, const RingRows& Rj, const RingRows& Rk,
                         double lok, double hij) {
  if (Ri.H < 0 || Rj.H < 0 || Rk.H < 0) return false;
  // |g1| must exceed lo_k - hi_j, since |g1 + g2| < |g1| + hi_j.
  const double need = lok - hij;
  const double need2 = need > 0 ? need * need : -1.0;
  for (long long x1 = Ri.H; x1 >= 0; --x1) {
    const long long ya = Ri.ya[x1], yb = std::min(Ri.yb[x1], x1);
    for (long long y1 = yb; y1 >= ya; --y1) {
      if (need2 > 0 && static_cast<double>(x1 * x1 + y1 * y1) <= need2) continue;
      for (long long x2 = -Rj.H; x2 <= Rj.H; ++x2) {
        const long long ax2 = x2 < 0 ? -x2 : x2;
        const long long s = x1 + x2, as = s < 0 ? -s : s;
        if (as > Rk.H) continue;
        const long long ja = Rj.ya[ax2], jb = Rj.yb[ax2];
        const long long ka = Rk.ya[as], kb = Rk.yb[as];
        if (ja > jb || ka > kb) continue;
        // y2 in [-jb, -ja] u [ja, jb]  and  y1 + y2 in [-kb, -ka] u [ka, kb]
        const long long J[2][2] = {{-jb, -ja}, {ja, jb}};
        const long long K[2][2] = {{-kb - y1, -ka - y1}, {ka - y1, kb - y1}};
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            if (intervals_meet(J[a][0], J[a][1], K[b][0], K[b][1])) return true;
      }
    }
  }
  return false;
}

// Cyclic closure (modulo n), by direct search; used only for ABS_ALLOW_WRAP plans.
bool has_cyclic_triangle(int n, const std::vector<std::pair<int, int>>& ci,
                         const std::vector<std::pair<int, int>>& cj, double lo2k, double hi2k) {
  auto wrap = [n](long long v) {
    long long r = ((v % n) + n) % n;
    return r < n / 2 ? r : r - n;
  };
  for (auto& a : ci)
    for (auto& b : cj) {
      const long long x = wrap(-(long long)a.first - b.first);
      const long long y = wrap(-(long long)a.second - b.second);
      if (in_ring(x * x + y * y, lo2k, hi2k)) return true;
    }
  return false;
}

std::vector<std::pair<int, int>> cells_of(const RingRows& R) {
  std::vector<std::pair<int, int>> c;
  for (long long x = -R.H; x <= R.H; ++x) {
    const long long ax = x < 0 ? -x : x;
    for (long long y = R.ya[ax]; y <= R.yb[ax]; ++y) {
      c.emplace_back((int)x, (int)y);
      if (y != 0) c.emplace_back((int)x, (int)-y);
    }
  }
  return c;
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

namespace abs_impl {

WorkLayout work_layout(const abs_plan_s* p, int grids, int w_batched, int have_counts, int spg) {
  if (!p->lv.empty()) {
    // the parent's Hermitian part and wmin slots, then each level's buffers
    WorkLayout w{};
    w.nisets = have_counts ? 0 : ((w_batched && p->wmode != ABS_W_UNIT) ? grids : 1) * p->nchan;
    const int batch = grids * spg * p->nchan;
    w.ndsets = batch;
    w.nsets = batch + w.nisets;
    w.npsets = batch / p->nchan;
    w.nipsets = w.nisets / p->nchan;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    w.wmin = off;
    off = al(off + (size_t)(batch + w.nisets) * 8);
    w.xc = off;
    off = al(off + (size_t)(batch + w.nisets) * (size_t)(p->hmax + 1) * (size_t)(2 * p->hmax + 1) * 8);
    for (const abs_plan_s* q : p->lv) {
      w.lv.push_back(work_layout(q, grids, w_batched, have_counts, spg));
      w.lvbase.push_back(off);
      off = al(off + w.lv.back().total);
    }
    w.total = off;
    return w;
  }
  WorkLayout w{};
  // spg data sets per grid (4 for complex input: see abs_estimate_complex), one weight set
  // per grid with batched weights, else one (none with cached counts)
  // multi-frequency: nchan data sets a grid and one weight set per channel
  w.nisets = have_counts ? 0 : ((w_batched && p->wmode != ABS_W_UNIT) ? grids : 1) * p->nchan;
  const int batch = grids * spg * p->nchan;
  w.ndsets = batch;
  w.nsets = batch + w.nisets;
  w.npsets = batch / p->nchan;
  w.nipsets = w.nisets / p->nchan;
  const int64_t n = p->n;
  w.zset = n * p->ncols;
  w.fset = (int64_t)p->nb * n * n;
  w.fset64 = (int64_t)p->nb * p->npix64;
  w.partset = (int64_t)p->nblk * p->ntrip;
  w.partset64 = (int64_t)p->nblk64 * p->ntrip;
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 0;
  w.zd = off;
  off = al(off + (size_t)batch * w.zset * 8);
  w.zi = off;
  off = al(off + (size_t)w.nisets * w.zset * 16);
  w.fd = off;
  off = al(off + (size_t)batch * w.fset * 4);
  w.fi = off;
  off = al(off + (size_t)w.nisets * w.fset64 * 8);
  w.part = off;
  off = al(off + (size_t)w.npsets * w.partset * 8);
  w.part64 = off;
  off = al(off + (size_t)w.nipsets * w.partset64 * 8);
  w.fmax = off;
  off = al(off + (size_t)batch * p->nb * 4);
  // smallest non-zero ring-cell weight per data set, then per weight set (FP64 bits)
  // (a level plan uses its parent's wmin and Hermitian part)
  const bool level = p->is_level;
  w.wmin = off;
  if (!level) off = al(off + (size_t)(batch + w.nisets) * 8);
  // column-major Hermitian part for the column pass: 8 bytes per cell (FP32 complex for
  // the data sets, FP64 real for the weight sets, which follow the data sets: the two run
  // concurrently)
  w.xc = off;
  if (!level)
    off = al(off + (size_t)(batch + w.nisets) * (size_t)(p->hmax + 1) * (size_t)(2 * p->hmax + 1) * 8);
  w.total = off;
  return w;
}

// The triplet contraction sum_theta F_i F_j F_k (Eq. 12: the numerator with the data
// fields, the denominator with the weight fields) specialised to this plan's triplet
// list: every wave owns a fixed group of triplets, holds one accumulator per triplet
// in registers, and walks its workgroup's pixels with one pixel per lane; the field
// values of a pixel are loaded once (coalesced across lanes, prefetched one
// iteration ahead) and every pair product (F_i F_j, or F_j F_k when the plan's
// triplets are grouped by their two largest rings) is formed once per pixel.
// Accumulators are summed across the wave through LDS in FP64 and written per
// workgroup; the finaliser adds workgroups in a fixed order.
// Two kernels are emitted: abs_contract (FP32 fields, FP32 accumulators) and
// abs_contract64 (FP64 fields and accumulators, for the weight fields).
namespace {

// Split the ordered triplet list (ord[0 .. ntrip)) into G contiguous groups whose
// register estimate, rw * (slots + bins used), stays within kBudget, and with the pair
// products the group forms (the compiler may keep them all live at once to overlap them)
// within kBudgetPairs: above it the generated kernels spill (measured: groups of
// rw * (slots + bins + pairs) up to 246 compile without spills, 258 and 262 spill 53 and
// 12 VGPRs).  G is a multiple of the waves per workgroup (*waves): 4, or 8 when more than
// 4 groups are needed (fewer slices re-read the fields).
std::vector<int> split_groups(const abs_plan_s* p, const std::vector<int>& ord, int rw, bool jk, int* waves) {
  const int T = (int)p->ntrip;
  const int kBudget = rw == 1 ? 200 : 184, kBudgetPairs = rw == 1 ? 232 : 208;
  auto cost_ok = [&](int t0, int t1) {
    std::set<int> bins;
    int pairs = 0, pa = -1, pb = -1;
    for (int t = t0; t < t1; ++t) {
      const int* x = &p->trips[3 * ord[t]];
      for (int q = 0; q < 3; ++q) bins.insert(x[q]);
      const int a = jk ? x[1] : x[0], b = jk ? x[2] : x[1];
      if (a != pa || b != pb) ++pairs;
      pa = a;
      pb = b;
    }
    const int regs = rw * ((t1 - t0) + (int)bins.size());
    return regs <= kBudget && regs + rw * pairs <= kBudgetPairs;
  };
  auto even = [&](int G) {
    std::vector<int> start(G + 1);
    for (int g = 0; g <= G; ++g) start[g] = (int)((int64_t)T * g / G);
    return start;
  };
  for (int G = 4; G <= 16384; G += 4) {
    std::vector<int> start = even(G);
    bool ok = true;
    for (int g = 0; g < G && ok; ++g) ok = cost_ok(start[g], start[g + 1]);
    if (!ok) continue;
    if (G == 4) {
      *waves = 4;
      return start;
    }
    *waves = 8;
    return even((G + 7) / 8 * 8);   // more, smaller groups still fit the budget
  }
  return {};
}

// Rings a kernel's slices stage, summed over the slices: the fields it reads per pixel.
int64_t staged_rings(const abs_plan_s* p, const std::vector<int>& ord, const std::vector<int>& start, int W) {
  const int G = (int)start.size() - 1;
  int64_t sum = 0;
  for (int z = 0; z < G / W; ++z) {
    std::set<int> b;
    for (int t = start[W * z]; t < start[W * z + W]; ++t)
      for (int q = 0; q < 3; ++q) b.insert(p->trips[3 * ord[t] + q]);
    sum += (int64_t)b.size();
  }
  return sum;
}

// Pair products a kernel's groups form per pixel: one per run of triplets with the same
// pair inside a group.
int64_t pairs_formed(const abs_plan_s* p, const std::vector<int>& ord, const std::vector<int>& start,
                     bool jk) {
  int64_t n = 0;
  for (size_t g = 0; g + 1 < start.size(); ++g) {
    int pa = -1, pb = -1;
    for (int t = start[g]; t < start[g + 1]; ++t) {
      const int* x = &p->trips[3 * ord[t]];
      const int a = jk ? x[1] : x[0], b = jk ? x[2] : x[1];
      if (a != pa || b != pb) ++n;
      pa = a;
      pb = b;
    }
  }
  return n;
}

// Triplet order of one kernel.  Each triplet i <= j <= k is formed as a pair product
// times a single ring: (D_i D_j) D_k, or (D_j D_k) D_i, whose pairs are fewer (a pair of
// large rings closes triangles with a run of small ones) but whose groups may span more
// rings.  Base order (i, j, k) or (j, k, i), then optionally blocks of B consecutive j;
// pairs stay contiguous, so each pair product is formed once per group.  The cost of an
// order is the VALU work per pixel (pair products formed + one FMA per triplet) plus the
// rings its slices stage, each weighed as kStagedRingCost operations (a field value read
// from memory and stored to LDS).
struct KernelOrder {
  std::vector<int> ord, start;
  int waves = 4;
  bool jk = false;
  int block = 0;    // blocks of this many consecutive j (0: none)
};
constexpr int64_t kStagedRingCost = 16;
KernelOrder choose_order(const abs_plan_s* p, int rw) {
  const int T = (int)p->ntrip;
  KernelOrder best;
  int64_t best_cost = -1;
  for (bool jk : {false, true}) {
    std::vector<int> base(T);
    for (int t = 0; t < T; ++t) base[t] = t;
    if (jk)
      std::stable_sort(base.begin(), base.end(), [&](int a, int b) {
        const int* x = &p->trips[3 * a];
        const int* y = &p->trips[3 * b];
        return std::make_tuple(x[1], x[2], x[0]) < std::make_tuple(y[1], y[2], y[0]);
      });
    for (int B : {0, 4, 8, 16}) {
      KernelOrder o;
      o.jk = jk;
      o.block = B;
      o.ord = base;
      if (B > 0)
        std::stable_sort(o.ord.begin(), o.ord.end(),
                         [&](int a, int b) { return p->trips[3 * a + 1] / B < p->trips[3 * b + 1] / B; });
      o.start = split_groups(p, o.ord, rw, jk, &o.waves);
      if (o.start.empty()) continue;
      const int64_t cost = kStagedRingCost * staged_rings(p, o.ord, o.start, o.waves) +
                           pairs_formed(p, o.ord, o.start, jk) + T;
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        best = std::move(o);
      }
    }
  }
  return best;
}

// Kernel layout.  A workgroup is W waves (W consecutive triplet groups, "slice" z) on
// one pixel block of one set.  The pixels are walked in chunks of 64 (one per lane);
// the rings the slice uses (its union U_z) are staged chunk by chunk in LDS, each wave
// loading every W-th of them, so every field value is read from memory once per
// workgroup.  A wave's loads for chunk c + 1 are issued two chunks ahead and stored to
// the LDS stage that chunk c - 1 occupied, after the one barrier per chunk that also
// publishes chunk c.  Workgroups are numbered so that the slices of one pixel block
// run on one XCD (blocks are dealt to the 8 XCDs round robin), where they share L2.
void emit_kernel(const abs_plan_s* p, const std::vector<int>& ord, const std::vector<int>& start, int W,
                 bool jk, int z0, int z1, const char* name, const char* R, std::string& s) {
  char buf[1024];
  const int G = (int)start.size() - 1;   // a multiple of W
  const int GZ = G / W;
  const int PZ = z1 - z0;                 // slices of this part
  const bool dbl = std::strcmp(R, "double") == 0;
  const int kRed = dbl ? 16 : 32;
  std::vector<std::vector<int>> gbins(G), U(GZ);
  for (int g = 0; g < G; ++g) {
    std::set<int> b;
    for (int t = start[g]; t < start[g + 1]; ++t)
      for (int q = 0; q < 3; ++q) b.insert(p->trips[3 * ord[t] + q]);
    gbins[g].assign(b.begin(), b.end());
  }
  int NU = 1;
  for (int z = z0; z < z1; ++z) {
    std::set<int> b;
    for (int g = W * z; g < W * z + W; ++g) b.insert(gbins[g].begin(), gbins[g].end());
    U[z].assign(b.begin(), b.end());
    NU = std::max(NU, (int)U[z].size());
  }
  std::snprintf(buf, sizeof buf,
                "extern \"C\" __global__ void __launch_bounds__(%d) %s(\n"
                "    const %s* __restrict__ F, long long set_stride, long long npix, int ppb,\n"
                "    double* __restrict__ part, int nblk, int ntrip) {\n", 64 * W, name, R);
  s += buf;
  // LDS: the staging area during the pixel walk, the reduction rows afterwards
  const size_t esz = dbl ? 8 : 4;
  const size_t lds = std::max((size_t)2 * NU * 64 * esz, (size_t)W * kRed * 65 * esz);
  std::snprintf(buf, sizeof buf,
                "  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;\n"
                "  const int xcd = blockIdx.x & 7, kx = blockIdx.x >> 3;\n"
                "  const int blk = xcd + 8 * (kx / %d), z = %d + kx %% %d;\n"
                "  if (blk >= nblk) return;\n"
                "  const int grp = z * %d + wave;\n"
                "  const long long set = blockIdx.y;\n"
                "  const long long p0 = (long long)blk * ppb;\n"
                "  const long long p1 = (p0 + ppb < npix) ? p0 + ppb : npix;\n"
                "  const int nch = (int)((p1 - p0) / 64);\n"
                "  const %s* __restrict__ Fs = F + set * set_stride + p0;\n"
                "  double* __restrict__ out = part + (set * nblk + blk) * (long long)ntrip;\n"
                "  __shared__ %s lds_all[%zu];\n"
                "  %s (*stg)[%d][64] = reinterpret_cast<%s (*)[%d][64]>(lds_all);\n"
                "  %s* red = lds_all + wave * %d * 65;\n"
                "  switch (grp) {\n", PZ, z0, PZ, W, R, R, lds / esz, R, NU, R, NU, R, kRed);
  s += buf;
  for (int g = W * z0; g < W * z1; ++g) {
    const int z = g / W, w = g % W;
    const int t0 = start[g], t1 = start[g + 1];
    const std::vector<int>& Uz = U[z];
    auto slot = [&](int m) { return (int)(std::lower_bound(Uz.begin(), Uz.end(), m) - Uz.begin()); };
    std::vector<int> mine;   // rings this wave stages
    for (int k = w; k < (int)Uz.size(); k += W) mine.push_back(Uz[k]);
    std::snprintf(buf, sizeof buf, "  case %d: {\n", g);
    s += buf;
    for (int t = t0; t < t1; ++t) {
      std::snprintf(buf, sizeof buf, "    %s a%d = 0;\n", R, t - t0);
      s += buf;
    }
    for (size_t k = 0; k < mine.size(); ++k) {
      std::snprintf(buf, sizeof buf,
                    "    const %s* __restrict__ L%zu = Fs + %dLL * npix;\n    %s e%zu, o%zu;\n", R, k,
                    mine[k], R, k, k);
      s += buf;
    }
    // prologue: chunk 0 to stage 0, chunk 1 in flight (odd set), chunk 2 in flight (even
    // set).  nch is even (pixel blocks are multiples of 128 pixels); loads past the last
    // chunk re-read it, which keeps every load unconditional.
    auto loads = [&](const char* set, const char* chunk) {
      std::string r;
      for (size_t k = 0; k < mine.size(); ++k) {
        std::snprintf(buf, sizeof buf, "    %s%zu = L%zu[(unsigned)(64 * min(%s, nch - 1) + lane)];\n", set,
                      k, k, chunk);
        r += buf;
      }
      return r;
    };
    auto stores = [&](const char* set, const char* stage) {
      std::string r;
      for (size_t k = 0; k < mine.size(); ++k) {
        std::snprintf(buf, sizeof buf, "    stg[%s][%d][lane] = %s%zu;\n", stage, slot(mine[k]), set, k);
        r += buf;
      }
      return r;
    };
    auto compute = [&](const char* stage) {
      std::string r;
      for (int m : gbins[g]) {
        std::snprintf(buf, sizeof buf, "    const %s d%d_%s = stg[%s][%d][lane];\n", R, m, stage, stage,
                      slot(m));
        r += buf;
      }
      std::snprintf(buf, sizeof buf, "    {\n    %s t;\n", R);
      r += buf;
      // pair (a, b) and single ring c of each triplet: (i, j) and k, or (j, k) and i
      int pa = -1, pb = -1;
      for (int t = t0; t < t1; ++t) {
        const int* x = &p->trips[3 * ord[t]];
        const int a = jk ? x[1] : x[0], b = jk ? x[2] : x[1], c = jk ? x[0] : x[2];
        if (a != pa || b != pb) {
          std::snprintf(buf, sizeof buf, "    t = d%d_%s * d%d_%s;\n", a, stage, b, stage);
          r += buf;
          pa = a;
          pb = b;
        }
        std::snprintf(buf, sizeof buf, "    a%d = abs_fma(t, d%d_%s, a%d);\n", t - t0, c, stage, t - t0);
        r += buf;
      }
      r += "    }\n";
      return r;
    };
    s += loads("e", "0");
    s += stores("e", "0");
    s += loads("o", "1");
    s += loads("e", "2");
    // chunk c even: publish stage 0 (chunk c), store chunk c + 1 (odd set) to stage 1,
    // load chunk c + 3 into the odd set, compute chunk c; then the same for c + 1.  The
    // loads of a chunk are issued two chunks before it is stored.
    s += "    for (int c = 0; c < nch; c += 2) {\n    __syncthreads();\n";
    s += stores("o", "1");
    s += loads("o", "c + 3");
    s += compute("0");
    s += "    __syncthreads();\n";
    s += stores("e", "0");
    s += loads("e", "c + 4");
    s += compute("1");
    s += "    }\n";
    // the reduction rows overlay the staging area: every wave has finished reading it
    s += "    __syncthreads();\n";
    // Cross-lane sums through LDS, kRed accumulators at a time: every lane stores its
    // values as one row per accumulator, then lane l < kRed adds row l in FP64.  One
    // store per accumulator keeps the generated code (and its compile time) small.
    for (int c0 = t0; c0 < t1; c0 += kRed) {
      const int c1 = std::min(t1, c0 + kRed);
      for (int t = c0; t < c1; ++t) {
        std::snprintf(buf, sizeof buf, "    red[%d * 65 + lane] = a%d;\n", t - c0, t - t0);
        s += buf;
      }
      std::snprintf(buf, sizeof buf,
                    "    abs_wave_sync();\n"
                    "    if (lane < %d) {\n"
                    "      double v = 0.0;\n"
                    "      for (int q = 0; q < 64; ++q) v += (double)red[lane * 65 + q];\n"
                    "      out[%d + lane] = v;\n"
                    "    }\n"
                    "    abs_wave_sync();\n", c1 - c0, c0);
      s += buf;
    }
    s += "  } break;\n";
  }
  s += "  default: break;\n  }\n}\n";
}

}  // namespace

// Slices per separately compiled part: bounds the size (and compile time) of one
// generated module, so that large plans compile as several parts in parallel processes.
// Fewer, larger parts run faster (8192^2 / 64 rings: FP32 contraction 155 ms in parts of 4
// slices, 140 ms in parts of 12; FP64 123 and 109 ms) and take longer to compile (a
// 12-slice part about 8 s).
constexpr int kSlicesPerPart = 12;
// Default bound of n / m for resolution levels (abs_plan_desc.levels = 0): 4, and 2 for the
// BF16 split form, whose per-product error (about 2^-16) is the largest; with ratio 4 its
// worst triplet error against the FP64 oracle reached 8.8e-5 on a 512^2 / 24-ring plan
// (FP16 split 4.4e-6, FP32 3.9e-6).
constexpr int kDefaultLevelRatio = 4, kDefaultLevelRatioBf16 = 2;

bool build_jit_source(abs_plan_s* p) {
  const KernelOrder o32 = choose_order(p, 1), o64 = choose_order(p, 2);
  if (o32.start.empty() || o64.start.empty()) return false;
  const std::vector<int>& g32 = o32.start;
  const std::vector<int>& g64 = o64.start;
  const int w32 = o32.waves, w64 = o64.waves;
  p->ngroups = (int)g32.size() - 1;
  p->ngroups64 = (int)g64.size() - 1;
  p->waves = w32;
  p->waves64 = w64;
  p->jk32 = o32.jk;
  p->jk64 = o64.jk;
  p->block32 = o32.block;
  p->block64 = o64.block;
  // partial sums are written in kernel order: position of every triplet in each order
  p->pos32.assign(p->ntrip, 0);
  p->pos64.assign(p->ntrip, 0);
  for (int t = 0; t < (int)p->ntrip; ++t) {
    p->pos32[o32.ord[t]] = t;
    p->pos64[o64.ord[t]] = t;
  }
  const std::string head =
      "// generated: triplet contraction for one ring-triplet list\n"
      "__device__ __forceinline__ float abs_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }\n"
      "__device__ __forceinline__ double abs_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }\n"
      "// orders a wave's LDS stores before its loads from other lanes\n"
      "__device__ __forceinline__ void abs_wave_sync() {\n"
      "  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, \"wavefront\");\n"
      "  __builtin_amdgcn_wave_barrier();\n}\n";
  p->parts.clear();
  auto add = [&](int kind, const std::vector<int>& ord, const std::vector<int>& start, int W,
                 bool jk, const char* R) {
    const int GZ = ((int)start.size() - 1) / W;
    // parts of up to kSlicesPerPart slices: the slices of one launch run together and
    // share their field reads through L2, which separate launches cannot
    const int per = kSlicesPerPart;
    for (int z0 = 0; z0 < GZ; z0 += per) {
      JitPart part;
      part.kind = kind;
      part.z0 = z0;
      part.z1 = std::min(GZ, z0 + per);
      part.src = head;
      emit_kernel(p, ord, start, W, jk, part.z0, part.z1, "abs_contract", R, part.src);
      p->parts.push_back(std::move(part));
    }
  };
  // the FP32 kernel serves the FP32 data path; the weight fields always use FP64
  if (!p->use_mfma) add(0, o32.ord, g32, w32, o32.jk, "float");
  add(1, o64.ord, g64, w64, o64.jk, "double");
  return true;
}

// FNV-1a of a part's generated source and the compile options: identifies a code object.
uint64_t jit_key(const abs_plan_s* p, int part) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const char* d, size_t n) {
    for (size_t i = 0; i < n; ++i) {
      h ^= (unsigned char)d[i];
      h *= 1099511628211ull;
    }
  };
  const std::string& src = p->parts[part].src;
  mix(src.data(), src.size());
  const char tag[] = "gfx950 -O3 -packed-fp32-ops";
  mix(tag, sizeof tag);
  return h;
}

abs_status compile_jit(abs_plan_s* p, int part) {
  JitPart& q = p->parts[part];
  if (q.compiled) return ABS_OK;
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, q.src.c_str(), "abs_contract.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return ABS_ERR_JIT;
  // Packed FP32 instructions are disabled for every kernel of this library.
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, 6, opts);
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return ABS_ERR_JIT;
  }
  size_t sz = 0;
  if (hiprtcGetCodeSize(prog, &sz) != HIPRTC_SUCCESS || sz == 0) {
    hiprtcDestroyProgram(&prog);
    return ABS_ERR_JIT;
  }
  q.code.resize(sz);
  const bool ok = hiprtcGetCode(prog, q.code.data()) == HIPRTC_SUCCESS;
  hiprtcDestroyProgram(&prog);
  if (!ok) return ABS_ERR_JIT;
  // ABS_JIT_DUMP=<directory>: keep the generated source and code object for inspection.
  if (const char* dir = std::getenv("ABS_JIT_DUMP")) {
    const std::string base = std::string(dir) + "/abs_contract_n" + std::to_string(p->n) + "_t" +
                             std::to_string(p->ntrip) + "_p" + std::to_string(part);
    if (FILE* f = std::fopen((base + ".hip").c_str(), "wb")) {
      std::fwrite(q.src.data(), 1, q.src.size(), f);
      std::fclose(f);
    }
    if (FILE* f = std::fopen((base + ".co").c_str(), "wb")) {
      std::fwrite(q.code.data(), 1, q.code.size(), f);
      std::fclose(f);
    }
  }
  q.compiled = true;
  return ABS_OK;
}

// Row order inside a row tile.  A lane of row r reads 16 bytes of ring j_r and of ring
// k_r at the same pixel offset; with LDS rows of 132 words, ring m starts in bank group
// m mod 8 (of 32 banks) or m mod 16 (of 64), so two rows of one access group reading
// different rings of the same group conflict.  Local search over row swaps minimises such
// clashes within groups of 8 and of 16 consecutive rows (the pair list is unchanged).
void order_rows(std::vector<std::pair<int, int>>& rows) {
  const int R = (int)rows.size();
  auto clash = [](int a, int b, int mod) { return a != b && a % mod == b % mod; };
  auto cost = [&]() {
    int c = 0;
    for (int a = 0; a < R; ++a)
      for (int b = a + 1; b < R; ++b) {
        const bool same8 = a / 8 == b / 8;
        c += clash(rows[a].second, rows[b].second, 16) + clash(rows[a].first, rows[b].first, 16);
        if (same8) c += clash(rows[a].second, rows[b].second, 8) + clash(rows[a].first, rows[b].first, 8);
      }
    return c;
  };
  int best = cost();
  for (bool improved = true; improved && best > 0;) {
    improved = false;
    for (int a = 0; a < R; ++a)
      for (int b = a + 1; b < R; ++b) {
        std::swap(rows[a], rows[b]);
        const int c = cost();
        if (c < best) {
          best = c;
          improved = true;
        } else {
          std::swap(rows[a], rows[b]);
        }
      }
  }
}

// Precision-form tiling.  Each triplet i <= j <= k is split as the pair product of its two
// largest rings, D_j D_k, times the smallest ring D_i (a pair (j, k) closes triangles with
// a run of small rings i, which gives far fewer distinct pairs than (i, j) pairs with their
// k: 228 against 528 at 32 rings, 855 against 2080 at 64).  Pairs ordered by (j, k) are cut
// into row tiles of 16; each row tile multiplies against the union of its rings i, 16 per
// MFMA tile, and all column tiles of a row tile share it (the kernel forms its operand once
// and keeps it while the wave's consecutive tiles use the same rows).
void build_mfma_tables(abs_plan_s* p) {
  const int nb = p->nbc;   // contraction bins: the rings, or the channel rings of a multi-frequency plan
  std::vector<std::vector<int>> cset(nb * nb);
  std::vector<int> tindex(nb * nb * nb, -1);     // [(j * nb + k) * nb + i]
  for (int64_t t = 0; t < p->ntrip; ++t) {
    const int i = p->trips[3 * t], j = p->trips[3 * t + 1], k = p->trips[3 * t + 2];
    cset[j * nb + k].push_back(i);
    tindex[(j * nb + k) * nb + i] = (int)t;
  }
  std::vector<std::pair<int, int>> pairs;   // (j, k)
  for (int j = 0; j < nb; ++j)
    for (int k = j; k < nb; ++k)
      if (!cset[j * nb + k].empty()) pairs.push_back({j, k});
  p->pt_pairs.clear();
  p->mt_ptile.clear();
  p->mt_bins.clear();
  p->mt_trip.clear();
  const int npt = (int)((pairs.size() + 15) / 16);
  std::vector<std::vector<std::vector<int>>> ctiles(npt);   // column tiles of each row tile
  int T = 0;
  for (int pt = 0; pt < npt; ++pt) {
    std::set<int> cs;
    std::vector<std::pair<int, int>> rows(16, {nb, nb});
    for (int r = 0; r < 16; ++r) {
      const size_t q = (size_t)pt * 16 + r;
      if (q < pairs.size()) {
        rows[r] = pairs[q];
        for (int i : cset[pairs[q].first * nb + pairs[q].second]) cs.insert(i);
      }
    }
    order_rows(rows);
    for (const auto& jk : rows) {
      p->pt_pairs.push_back(jk.first);
      p->pt_pairs.push_back(jk.second);
    }
    const std::vector<int> cv(cs.begin(), cs.end());
    for (size_t c0 = 0; c0 < cv.size(); c0 += 16) {
      std::vector<int> cols(16);
      for (int c = 0; c < 16; ++c) cols[c] = c0 + c < cv.size() ? cv[c0 + c] : nb;
      ctiles[pt].push_back(cols);
      ++T;
    }
  }
  // Row tiles (with all their column tiles) are dealt to waves longest first, each to the
  // least loaded wave with room (longest-processing-time rule); a wave's cost counts 2
  // per tile (its matrix work and column operand) and 5 per row tile (forming and
  // splitting the pair products, the larger part).  Early row tiles (small rings) have
  // one column tile, late ones up to four, so equal tile counts would be unequal work.
  auto cost = [&](int pt) { return 5 + 2 * (int)ctiles[pt].size(); };
  std::vector<int> order(npt);
  for (int pt = 0; pt < npt; ++pt) order[pt] = pt;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  // Deal the row tiles to `waves` waves of at most `cap` tiles each; false if one does
  // not fit.
  std::vector<std::vector<int>> assign;
  auto deal = [&](int waves, int cap) {
    std::vector<int> load(waves, 0), cnt(waves, 0);
    assign.assign(waves, {});
    for (int pt : order) {
      int best = -1;
      for (int w = 0; w < waves; ++w)
        if (cnt[w] + (int)ctiles[pt].size() <= cap && (best < 0 || load[w] < load[best])) best = w;
      if (best < 0) return false;
      assign[best].push_back(pt);
      load[best] += cost(pt);
      cnt[best] += (int)ctiles[pt].size();
    }
    return true;
  };
  // Small plans (at most 32 rings, 8 waves of at most kSmallTilesPerWave tiles) use the
  // kernel variant with few accumulators, whose registers allow two workgroups per CU;
  // others the one with kTilesPerWave, in as many 8-wave groups as needed.
  int waves = 8;
  if (nb <= 32 && deal(8, kSmallTilesPerWave)) {
    p->mfma_tpw = kSmallTilesPerWave;
    p->mfma_depth = 1;
  } else {
    p->mfma_tpw = kTilesPerWave;
    // plans of at most 32 rings keep four chunks of loads in flight (their work per chunk
    // is short); larger plans one, which keeps the registers for the tiles
    p->mfma_depth = nb <= 32 ? 4 : 1;
    waves = std::max(8, (T + kTilesPerWave - 1) / kTilesPerWave);
    waves = (waves + 7) / 8 * 8;
    while (!deal(waves, kTilesPerWave)) waves += 8;
  }
  p->mfma_groups = waves / 8;
  p->wave_tiles.assign(2 * waves, 0);
  int tile = 0;
  for (int w = 0; w < waves; ++w) {
    std::sort(assign[w].begin(), assign[w].end());
    p->wave_tiles[2 * w] = tile;
    for (int pt : assign[w])
      for (const std::vector<int>& cols : ctiles[pt]) {
        p->mt_ptile.push_back(pt);
        for (int c = 0; c < 16; ++c) p->mt_bins.push_back(cols[c]);
        for (int r = 0; r < 16; ++r) {
          const int j = p->pt_pairs[2 * (pt * 16 + r)], k = p->pt_pairs[2 * (pt * 16 + r) + 1];
          for (int c = 0; c < 16; ++c) {
            const int i = cols[c];
            p->mt_trip.push_back(j < nb && i < nb ? tindex[(j * nb + k) * nb + i] : -1);
          }
        }
        ++tile;
      }
    p->wave_tiles[2 * w + 1] = tile - p->wave_tiles[2 * w];
  }
}


// Rings of a plan: per ring the largest |g_x| (h), the half-plane columns 0 .. h its
// column pass transforms, their offset in a set of column-pass output (n per column), the
// mean radius; also hmax and the total column count.  Returns each ring's rows of cells.
std::vector<RingRows> setup_rings(abs_plan_s* p) {
  const int nb = p->nb;
  std::vector<RingRows> rows(nb);
  p->h.assign(nb, 0);
  p->cols.assign(nb, 0);
  p->zoff.assign(nb, 0);
  p->radius.assign(nb, 0.0);
  int64_t acc = 0;
  for (int m = 0; m < nb; ++m) {
    rows[m] = ring_rows(p->lo2[m], p->hi2[m]);
    p->h[m] = (int)rows[m].H;
    p->cols[m] = rows[m].H >= 0 ? (int)rows[m].H + 1 : 0;
    p->zoff[m] = acc * p->n;
    acc += p->cols[m];
    double sr = 0.0;
    long long cnt = 0;
    for (long long x = -rows[m].H; x <= rows[m].H; ++x) {
      const long long ax = x < 0 ? -x : x;
      for (long long y = rows[m].ya[ax]; y <= rows[m].yb[ax]; ++y) {
        const double r = std::sqrt((double)(x * x + y * y));
        sr += (y == 0) ? r : 2.0 * r;
        cnt += (y == 0) ? 1 : 2;
      }
    }
    p->radius[m] = cnt ? sr / (double)cnt : std::nan("");
  }
  p->ncols = acc;
  p->hmax = 0;
  for (int m = 0; m < nb; ++m) p->hmax = std::max(p->hmax, p->h[m]);
  p->nbc = p->nchan * nb;
  return rows;
}

int64_t count_pairs(const std::vector<int32_t>& trips) {
  std::set<std::pair<int, int>> pairs;
  for (size_t t = 0; t + 2 < trips.size(); t += 3) pairs.insert({trips[t], trips[t + 1]});
  return (int64_t)pairs.size();
}

// Precision forms: run the data contraction on the matrix units only where that is
// estimated to be faster than the FP32 VALU kernel.  Per pixel and set, modelled on the
// 8192^2, 4096^2 and 1024^2 workloads' level kernels (one MI355X): the VALU kernel about
// 4 + 0.45 bins + 0.015 (pairs + 2 triplets) ps, the MFMA kernel about 8 + 0.64 bins +
// 2.13 tiles ps (each 16 x 16 tile three split products per chunk, operands staged for
// every bin).  With few triplets per tile (the top levels, small plans) the VALU kernel
// wins.  ABS_ALL_MFMA keeps every contraction on the matrix units.
bool use_mfma_for(const abs_plan_s* p) {
  if (p->precision == ABS_FP32) return false;
  if (p->flags & ABS_ALL_MFMA) return true;
  std::set<std::pair<int, int>> ij, jk;
  for (int64_t t = 0; t < p->ntrip; ++t) {
    ij.insert({p->trips[3 * t], p->trips[3 * t + 1]});
    jk.insert({p->trips[3 * t + 1], p->trips[3 * t + 2]});
  }
  const double flops = (double)std::min(ij.size(), jk.size()) + 2.0 * (double)p->ntrip;
  const double t32 = 4.0 + 0.45 * p->nbc + 0.015 * flops;
  const double t16 = 8.0 + 0.64 * p->nbc + 2.13 * (double)p->mt_ptile.size();
  return t16 < t32;
}

// FFT tiling, contraction pixel blocks, the device layout of the tables, the precision
// form's tables and the contraction code of a plan whose rings and triplets are set.
bool setup_kernels(abs_plan_s* p) {
  const int n = p->n, nb = p->nb;
  // FFT tiling: a column-pass workgroup of col_block(log2 n) threads transforms ct columns
  // of one ring at once, one transform per TG threads (n/16, or n/32 when n/16 exceeds the
  // engine's block: two butterflies a thread)
  {
    const int n16 = std::max(1, n / 16);
    auto tg = [&](bool f32) {
      const int eb = col_engine(p->log2n, f32);
      return std::min(n16 > eb ? n16 / 2 : n16, eb);
    };
    p->ct = col_block(p->log2n, true) / tg(true);
    p->ct64 = col_block(p->log2n, false) / tg(false);
  }
  p->tiles.clear();
  p->tiles64.clear();
  for (int m = 0; m < nb; ++m) {
    for (int g0 = 0; g0 < p->cols[m]; g0 += p->ct)
      p->tiles.push_back({m, g0, std::min(p->ct, p->cols[m] - g0), 0});
    for (int g0 = 0; g0 < p->cols[m]; g0 += p->ct64)
      p->tiles64.push_back({m, g0, std::min(p->ct64, p->cols[m] - g0), 0});
  }
  const int64_t npix = (int64_t)n * n;
  p->pix_per_block = (int)std::min<int64_t>(16384, std::max<int64_t>(1024, npix / 64));
  p->nblk = (int)((npix + p->pix_per_block - 1) / p->pix_per_block);
  // one weight set per call as a rule: smaller blocks keep the GPU busy
  // weight fields: half plane, block 0 = rows 0 and n/2 (so at least 2n pixels a block);
  // at most 256 blocks of the half plane, so that the slices of the weight kernel, one
  // 8-wave workgroup per CU, fill whole rounds of the 256 CUs rather than leaving a round
  // with a few workgroups.  Blocks are multiples of 128 pixels: the contraction walks
  // them in pairs of 64-pixel chunks.
  {
    const int64_t rows_b = (int64_t)(p->n / 2 - 1) * p->n;
    const int64_t want = std::max<int64_t>(std::max<int64_t>(1024, 2 * (int64_t)p->n), (rows_b + 254) / 255);
    p->pix_per_block64 = (int)((want + 127) / 128 * 128);
    const int64_t b = p->pix_per_block64;
    p->nblk64 = 1 + (int)((rows_b + b - 1) / b);
    p->npix64 = (int64_t)p->nblk64 * b;
  }

  // device layout of the plan tables
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 0;
  p->dl.tw = off;
  off = al(off + (size_t)n * 8);
  p->dl.tw64 = off;
  off = al(off + (size_t)n * 16);
  p->dl.bins = off;
  off = al(off + (size_t)nb * sizeof(BinDev));
  p->dl.tiles = off;
  off = al(off + p->tiles.size() * sizeof(ColTile));
  p->dl.tiles64 = off;
  off = al(off + p->tiles64.size() * sizeof(ColTile));
  build_mfma_tables(p);
  p->dl.pt_pairs = off;
  off = al(off + p->pt_pairs.size() * 4);
  p->dl.mt_ptile = off;
  off = al(off + p->mt_ptile.size() * 4);
  p->dl.mt_bins = off;
  off = al(off + p->mt_bins.size() * 4);
  p->dl.mt_trip = off;
  off = al(off + p->mt_trip.size() * 4);
  p->dl.wave_tiles = off;
  off = al(off + p->wave_tiles.size() * 4);
  p->dl.pos32 = off;
  off = al(off + (size_t)p->ntrip * 4);
  p->dl.pos64 = off;
  off = al(off + (size_t)p->ntrip * 4);
  p->dl.tmap = off;
  off = al(off + p->tmap.size() * 4);
  p->dl.total = off;
  p->use_mfma = use_mfma_for(p);
  return build_jit_source(p);
}

// Resolution levels of a plan.  A triplet i <= j <= k fits a level of size m when
// h_i + h_j + h_k < m and 2 h_k < m (h: a ring's largest |g_x|, which is also its largest
// |g_y|): the x and y components of the sum of three of its cells then lie in (-m, m), so
// the sum vanishes modulo m only where it vanishes, and no two cells of a ring share a
// column or row of the m x m transform.  It runs in the smallest chosen level that fits it
// (the level at n, always available, takes the rest, wrapped plans' cyclic triplets
// included; a level left without triplets is dropped), and a level transforms only the
// rings from its smallest i to its largest k.  The sets of levels drawn from n/2, n/4, ...,
// n / max_ratio (at least 16) are compared by a cost per call, in units of one
// contraction flop on one set: per level, its FFT passes (each of its rings over m^2
// pixels, about kFftCost flops a pixel and ring), its contraction (pair products and two
// flops per triplet, per pixel), both over max_batch data sets and one weight set, and a
// fixed cost for its launches (kLevelCost, about 40 us).  The ratio is bounded because the
// sum over m^2 pixels averages the fields' rounding errors over fewer terms (the FP32
// error of a level's sums grows about as n / m against the FP64 random-error scale of the
// full-grid sum).  ABS_EVERY_LEVEL takes every candidate level.
void choose_levels(const abs_plan_s* p, std::vector<int>& sizes, std::vector<int>& level_of) {
  constexpr double kFftCost = 72.0, kLevelCost = 2.4e9;
  const int T = (int)p->ntrip, n = p->n;
  std::vector<int> need(T);
  for (int t = 0; t < T; ++t) {
    const int* x = &p->trips[3 * t];
    const int h0 = p->h[x[0] % p->nb], h1 = p->h[x[1] % p->nb], h2 = p->h[x[2] % p->nb];
    const int hs = h0 + h1 + h2, hm = std::max(h0, std::max(h1, h2));
    int m = 16;
    while ((hs >= m || 2 * hm >= m) && m <= n) m *= 2;
    need[t] = m;
  }
  std::vector<int> cand;
  for (int m = n / 2; m >= 16 && (int64_t)m * p->max_ratio >= n; m /= 2) cand.push_back(m);
  const double sets = (double)p->max_batch + 1.0;
  double best = -1.0;
  const int all = (1 << cand.size()) - 1;
  for (int mask = (p->flags & ABS_EVERY_LEVEL) ? all : 0; mask <= all; ++mask) {
    std::vector<int> lv = {n};
    for (int c = 0; c < (int)cand.size(); ++c)
      if (mask >> c & 1) lv.push_back(cand[c]);
    std::vector<int> lof(T);
    for (int t = 0; t < T; ++t) {
      int L = 0;
      for (int q = 1; q < (int)lv.size(); ++q)
        if (lv[q] >= need[t]) L = q;   // lv is descending: the last that fits is the smallest
      lof[t] = L;
    }
    double cost = 0.0;
    std::vector<int> keep, remap(lv.size(), -1);
    for (int L = 0; L < (int)lv.size(); ++L) {
      int64_t cnt = 0;
      int K0 = p->nb, K1 = 0;
      std::set<std::pair<int, int>> ij, jk;
      for (int t = 0; t < T; ++t) {
        if (lof[t] != L) continue;
        const int* x = &p->trips[3 * t];
        ++cnt;
        for (int q = 0; q < 3; ++q) {
          K0 = std::min(K0, x[q] % p->nb);
          K1 = std::max(K1, x[q] % p->nb + 1);
        }
        ij.insert({x[0], x[1]});
        jk.insert({x[1], x[2]});
      }
      if (cnt == 0) continue;   // a level without triplets is left out
      remap[L] = (int)keep.size();
      keep.push_back(lv[L]);
      const double m2 = (double)lv[L] * lv[L];
      cost += sets * m2 * (kFftCost * p->nchan * (K1 - K0) + (double)std::min(ij.size(), jk.size()) + 2.0 * cnt) +
              kLevelCost;
    }
    if (best < 0.0 || cost < best) {
      best = cost;
      sizes = keep;
      level_of.resize(T);
      for (int t = 0; t < T; ++t) level_of[t] = remap[lof[t]];
    }
  }
}

// A level plan of size m: the parent's rings K0 .. K1-1 (from the smallest i to the
// largest k of its triplets), renumbered from 0; the given triplets of the parent (tidx,
// ascending) in that numbering; its own FFT tiling, tables and contraction code.  Its
// column pass reads the parent's Hermitian part.
abs_plan_s* make_level(const abs_plan_s* p, int m, const std::vector<int32_t>& tidx) {
  abs_plan_s* q = new (std::nothrow) abs_plan_s;
  if (!q) return nullptr;
  q->is_level = true;
  int K0 = p->nb, K1 = 0;
  for (int32_t t : tidx)
    for (int c = 0; c < 3; ++c) {
      K0 = std::min(K0, p->trips[3 * t + c] % p->nb);
      K1 = std::max(K1, p->trips[3 * t + c] % p->nb + 1);
    }
  q->n = m;
  q->nb = K1 - K0;
  q->nchan = p->nchan;
  q->ring0 = K0;
  q->log2n = ilog2(m);
  q->du = p->du;
  q->theta0 = p->theta0;
  q->norm = p->norm;
  q->precision = p->precision;
  q->wmode = p->wmode;
  q->max_batch = p->max_batch;
  q->flags = p->flags;
  q->edges.assign(p->edges.begin() + K0, p->edges.begin() + K1 + 1);
  q->lo2.assign(p->lo2.begin() + K0, p->lo2.begin() + K1);
  q->hi2.assign(p->hi2.begin() + K0, p->hi2.begin() + K1);
  setup_rings(q);
  q->xc_hm = p->hmax;
  q->tmap = tidx;
  // channel ring s = c nb + r of the parent is c nb' + (r - K0) here (the order is kept)
  for (int32_t t : tidx)
    for (int c = 0; c < 3; ++c) {
      const int sidx = p->trips[3 * t + c];
      q->trips.push_back((sidx / p->nb) * q->nb + (sidx % p->nb - K0));
    }
  q->ntrip = (int64_t)tidx.size();
  q->npairs = count_pairs(q->trips);
  if (!setup_kernels(q)) {
    delete q;
    return nullptr;
  }
  return q;
}

abs_plan_s* part_owner(abs_plan_s* p, int k, int* local) {
  if (k < 0) return nullptr;
  for (abs_plan_s* q : run_plans(p)) {
    if (k < (int)q->parts.size()) {
      *local = k;
      return q;
    }
    k -= (int)q->parts.size();
  }
  return nullptr;
}

void release_aux(abs_plan_s* p) {
  if (!p->aux && !p->fork && !p->join) return;
  int cur = -1;
  const bool other = hipGetDevice(&cur) == hipSuccess && p->aux_device >= 0 && cur != p->aux_device;
  if (other) (void)hipSetDevice(p->aux_device);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->join) (void)hipEventDestroy(p->join);
  if (other) (void)hipSetDevice(cur);
  p->aux = nullptr;
  p->fork = p->join = nullptr;
  p->aux_device = -1;
}

void destroy_plan(abs_plan_s* p) {
  if (!p) return;
  bool loaded = false;
  for (abs_plan_s* q : run_plans(p))
    for (const JitPart& c : q->parts) loaded = loaded || c.module;
  if (loaded) {
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && p->device >= 0 && cur != p->device;
    if (other) (void)hipSetDevice(p->device);
    for (abs_plan_s* q : run_plans(p))
      for (JitPart& c : q->parts)
        if (c.module) (void)hipModuleUnload(c.module);
    if (other) (void)hipSetDevice(cur);
  }
  release_aux(p);
  for (abs_plan_s* q : p->lv) delete q;
  delete p;
}

}  // namespace abs_impl

extern "C" {

const char* abs_status_str(abs_status s) {
  switch (s) {
    case ABS_OK: return "ok";
    case ABS_ERR_INVALID: return "invalid argument";
    case ABS_ERR_ALIAS: return "rings reach beyond n/3 (triangles would wrap); set ABS_ALLOW_WRAP";
    case ABS_ERR_UNBOUND: return "plan is not bound to device memory";
    case ABS_ERR_DEVICE: return "HIP runtime or kernel error";
    case ABS_ERR_JIT: return "run-time compilation of the contraction kernel failed";
    case ABS_ERR_NOMEM: return "out of host memory or caller buffer too small";
    case ABS_ERR_EMPTY: return "no ring triplet contains a closed lattice triangle";
    case ABS_ERR_SCRATCH:
      return "the estimate needs more workspace than the 256 MiB static scratch of abs_estimate_noalloc";
  }
  return "unknown status";
}

abs_status abs_plan(const abs_plan_desc* d, abs_plan_t* out) {
  if (!d || !out) return ABS_ERR_INVALID;
  *out = nullptr;
  const int n = d->n, nb = d->nbins;
  if (n < 16 || n > kMaxN || (n & (n - 1))) return ABS_ERR_INVALID;
  if (nb < 1 || nb > kMaxBins || !d->edges) return ABS_ERR_INVALID;
  if (d->max_batch < 1 || d->max_batch > 65535) return ABS_ERR_INVALID;
  if (d->wmode < ABS_W_UNIT || d->wmode > ABS_W_GIVEN) return ABS_ERR_INVALID;
  if (d->precision < ABS_FP32 || d->precision > ABS_FP16X3) return ABS_ERR_INVALID;
  if (!(d->du > 0.0) || !std::isfinite(d->du)) return ABS_ERR_INVALID;
  if (d->levels < 0 || d->levels > n || (d->levels & (d->levels - 1))) return ABS_ERR_INVALID;
  const int nchan = d->nchan < 1 ? 1 : d->nchan;
  if (nchan * nb > kMaxBins) return ABS_ERR_INVALID;
  for (int m = 0; m <= nb; ++m)
    if (!std::isfinite(d->edges[m]) || d->edges[m] < 0.0) return ABS_ERR_INVALID;
  for (int m = 0; m < nb; ++m)
    if (!(d->edges[m + 1] > d->edges[m])) return ABS_ERR_INVALID;
  if (d->edges[0] == 0.0 && !(d->flags & ABS_ALLOW_DC)) return ABS_ERR_INVALID;
  if (d->edges[nb] > 0.5 * n) return ABS_ERR_ALIAS;
  if (d->edges[nb] > n / 3.0 && !(d->flags & ABS_ALLOW_WRAP)) return ABS_ERR_ALIAS;

  abs_plan_s* p = new (std::nothrow) abs_plan_s;
  if (!p) return ABS_ERR_NOMEM;
  p->n = n;
  p->nb = nb;
  p->log2n = ilog2(n);
  p->du = d->du;
  p->theta0 = d->theta0 > 0 ? d->theta0 : 0.6 * 24.68 * kPi / 180.0;
  p->norm = d->norm > 0 ? d->norm : kPi * p->theta0 * p->theta0 / 3.0;
  p->precision = d->precision;
  p->wmode = d->wmode;
  p->max_batch = d->max_batch;
  p->flags = d->flags;
  p->nchan = nchan;
  p->max_ratio = d->levels != 0 ? d->levels
                 : d->precision == ABS_BF16X3 ? kDefaultLevelRatioBf16 : kDefaultLevelRatio;
  p->edges.assign(d->edges, d->edges + nb + 1);
  for (int m = 0; m < nb; ++m) {
    p->lo2.push_back(p->edges[m] * p->edges[m]);
    p->hi2.push_back(p->edges[m + 1] * p->edges[m + 1]);
  }
  const std::vector<RingRows> rows = setup_rings(p);
  p->xc_hm = p->hmax;

  // triplets i <= j <= k with at least one closed lattice triangle
  const bool wrap = (p->flags & ABS_ALLOW_WRAP) && p->edges[nb] > n / 3.0;
  std::vector<std::vector<std::pair<int, int>>> cells;
  if (wrap) {
    cells.resize(nb);
    for (int m = 0; m < nb; ++m) cells[m] = cells_of(rows[m]);
  }
  for (int i = 0; i < nb; ++i)
    for (int j = i; j < nb; ++j)
      for (int k = j; k < nb; ++k) {
        bool ok;
        if (wrap) {
          ok = has_cyclic_triangle(n, cells[i], cells[j], p->lo2[k], p->hi2[k]);
        } else {
          if (!(p->edges[k] < p->edges[i + 1] + p->edges[j + 1])) continue;  // triangle inequality
          ok = has_planar_triangle(rows[i], rows[j], rows[k], p->edges[k], p->edges[j + 1]);
        }
        if (!ok) continue;
        p->trips.push_back(i);
        p->trips.push_back(j);
        p->trips.push_back(k);
      }
  // Multi-frequency plans: every non-decreasing triple of channel rings s = c nb + r whose
  // rings, sorted, form a plan triplet (the estimator of Eq. 12 with the three fields taken
  // at three channels, each unordered combination of (ring, channel) pairs once).
  if (p->nchan > 1) {
    std::set<std::tuple<int, int, int>> ok;
    for (size_t t = 0; t + 2 < p->trips.size(); t += 3) ok.insert({p->trips[t], p->trips[t + 1], p->trips[t + 2]});
    std::vector<int32_t> st;
    const int B = p->nbc;
    for (int s1 = 0; s1 < B; ++s1)
      for (int s2 = s1; s2 < B; ++s2)
        for (int s3 = s2; s3 < B; ++s3) {
          int r[3] = {s1 % nb, s2 % nb, s3 % nb};
          std::sort(r, r + 3);
          if (!ok.count({r[0], r[1], r[2]})) continue;
          st.push_back(s1);
          st.push_back(s2);
          st.push_back(s3);
        }
    p->trips.swap(st);
  }
  p->ntrip = (int64_t)p->trips.size() / 3;
  if (p->ntrip == 0) {
    delete p;
    return ABS_ERR_EMPTY;
  }
  p->npairs = count_pairs(p->trips);
  p->labels.resize(5 * p->ntrip);
  for (int64_t t = 0; t < p->ntrip; ++t) {
    int r[3] = {p->trips[3 * t] % nb, p->trips[3 * t + 1] % nb, p->trips[3 * t + 2] % nb};
    std::sort(r, r + 3);
    const double l3 = 2 * kPi * p->du * p->radius[r[0]];
    const double l2 = 2 * kPi * p->du * p->radius[r[1]];
    const double l1 = 2 * kPi * p->du * p->radius[r[2]];
    double* L = &p->labels[5 * t];
    L[0] = l1;
    L[1] = l2;
    L[2] = l3;
    L[3] = (l1 * l1 + l2 * l2 - l3 * l3) / (2.0 * l1 * l2);
    L[4] = l2 / l1;
  }

  // resolution levels, when the cost model finds more than one worth running
  std::vector<int> sizes, level_of;
  choose_levels(p, sizes, level_of);
  if (sizes.size() > 1 || sizes[0] != n) {
    size_t off = 0;
    for (int L = 0; L < (int)sizes.size(); ++L) {
      std::vector<int32_t> tidx;
      for (int64_t t = 0; t < p->ntrip; ++t)
        if (level_of[t] == L) tidx.push_back((int32_t)t);
      abs_plan_s* q = make_level(p, sizes[L], tidx);
      if (!q) {
        destroy_plan(p);
        return ABS_ERR_JIT;
      }
      q->dev_off = off;
      off = (off + q->dl.total + 255) & ~(size_t)255;
      p->lv.push_back(q);
    }
    p->dl = DevLayout{};
    p->dl.total = off;
  } else if (!setup_kernels(p)) {
    delete p;
    return ABS_ERR_JIT;
  }
  *out = p;
  return ABS_OK;
}

namespace {
void fill_info(const abs_plan_s* p, abs_plan_info* o) {
  o->n = p->n;
  o->nbins = p->nb;
  o->ntrip = p->ntrip;
  o->npairs = p->npairs;
  o->ncols = p->ncols;
  o->plan_bytes = (int64_t)p->dl.total;
  o->norm = p->norm;
  o->mfma_tiles = (int64_t)p->mt_ptile.size();
  o->jit_parts = (int32_t)p->parts.size();
  o->contract_parts = o->weight_parts = 0;
  for (const JitPart& q : p->parts) ++(q.kind == 0 ? o->contract_parts : o->weight_parts);
  o->contract_jk = p->jk32 ? 1 : 0;
  o->contract_block = p->block32;
  o->contract_waves = p->waves;
  o->weight_jk = p->jk64 ? 1 : 0;
  o->weight_block = p->block64;
  o->weight_waves = p->waves64;
  o->mfma_tiles_per_wave = p->mfma_tpw;
  o->mfma_depth = p->mfma_depth;
  o->nlevels = 1;
  o->ring0 = p->ring0;
  o->nchan = p->nchan;
}
}  // namespace

abs_status abs_plan_info_get(abs_plan_t p, abs_plan_info* o) {
  if (!p || !o) return ABS_ERR_INVALID;
  if (p->lv.empty()) {
    fill_info(p, o);
    return ABS_OK;
  }
  // the code variants reported are the top level's; counts are summed over the levels
  fill_info(p->lv[0], o);
  o->n = p->n;
  o->nbins = p->nb;
  o->ntrip = p->ntrip;
  o->npairs = p->npairs;
  o->ncols = p->ncols;
  o->plan_bytes = (int64_t)p->dl.total;
  o->mfma_tiles = o->jit_parts = o->contract_parts = o->weight_parts = 0;
  for (const abs_plan_s* q : p->lv) {
    abs_plan_info qi;
    fill_info(q, &qi);
    o->mfma_tiles += qi.mfma_tiles;
    o->jit_parts += qi.jit_parts;
    o->contract_parts += qi.contract_parts;
    o->weight_parts += qi.weight_parts;
  }
  o->nlevels = (int32_t)p->lv.size();
  return ABS_OK;
}

abs_status abs_plan_level_info(abs_plan_t p, int32_t level, abs_plan_info* o, int32_t* tmap) {
  if (!p || !o || level < 0) return ABS_ERR_INVALID;
  if (p->lv.empty()) {
    if (level != 0) return ABS_ERR_INVALID;
    fill_info(p, o);
    if (tmap)
      for (int64_t t = 0; t < p->ntrip; ++t) tmap[t] = (int32_t)t;
    return ABS_OK;
  }
  if (level >= (int)p->lv.size()) return ABS_ERR_INVALID;
  const abs_plan_s* q = p->lv[level];
  fill_info(q, o);
  o->plan_bytes = 0;   // part of the parent's
  if (tmap) std::memcpy(tmap, q->tmap.data(), q->tmap.size() * sizeof(int32_t));
  return ABS_OK;
}

abs_status abs_plan_triplets(abs_plan_t p, int32_t* ijk, double* labels, double* radius) {
  if (!p) return ABS_ERR_INVALID;
  if (ijk) std::memcpy(ijk, p->trips.data(), p->trips.size() * sizeof(int32_t));
  if (labels) std::memcpy(labels, p->labels.data(), p->labels.size() * sizeof(double));
  if (radius) std::memcpy(radius, p->radius.data(), p->radius.size() * sizeof(double));
  return ABS_OK;
}

abs_status abs_plan_compile(abs_plan_t p) {
  if (!p) return ABS_ERR_INVALID;
  for (abs_plan_s* q : run_plans(p))
    for (int k = 0; k < (int)q->parts.size(); ++k) {
      const abs_status s = compile_jit(q, k);
      if (s != ABS_OK) return s;
    }
  return ABS_OK;
}

abs_status abs_plan_compile_part(abs_plan_t p, int32_t part) {
  int k = 0;
  abs_plan_s* q = p ? part_owner(p, part, &k) : nullptr;
  if (!q) return ABS_ERR_INVALID;
  return compile_jit(q, k);
}

abs_status abs_plan_code(abs_plan_t p, int32_t part, uint64_t* key, void* dst, size_t* bytes) {
  int k = 0;
  abs_plan_s* q = p ? part_owner(p, part, &k) : nullptr;
  if (!q || !bytes) return ABS_ERR_INVALID;
  JitPart& c = q->parts[k];
  if (key) *key = jit_key(q, k);
  if (!dst) {
    if (!c.compiled) {
      const abs_status s = compile_jit(q, k);
      if (s != ABS_OK) return s;
    }
    *bytes = c.code.size();
    return ABS_OK;
  }
  if (!c.compiled) return ABS_ERR_INVALID;
  if (*bytes < c.code.size()) return ABS_ERR_NOMEM;
  std::memcpy(dst, c.code.data(), c.code.size());
  *bytes = c.code.size();
  return ABS_OK;
}

abs_status abs_plan_set_code(abs_plan_t p, int32_t part, uint64_t key, const void* src, size_t bytes) {
  int k = 0;
  abs_plan_s* q = p ? part_owner(p, part, &k) : nullptr;
  if (!q || !src || bytes == 0) return ABS_ERR_INVALID;
  if (key != jit_key(q, k)) return ABS_ERR_INVALID;   // compiled for another triplet list
  JitPart& c = q->parts[k];
  c.code.assign(static_cast<const char*>(src), static_cast<const char*>(src) + bytes);
  c.compiled = true;
  return ABS_OK;
}

abs_status abs_estimate_workspace(abs_plan_t p, int32_t batch, int32_t w_batched,
                                  int32_t have_counts, size_t* bytes) {
  if (!p || !bytes || batch < 0 || batch > p->max_batch) return ABS_ERR_INVALID;
  *bytes = work_layout(p, batch, w_batched, have_counts).total;
  return ABS_OK;
}

abs_status abs_destroy(abs_plan_t p) {
  destroy_plan(p);
  return ABS_OK;
}

}  // extern "C"
