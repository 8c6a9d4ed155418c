/*
 * abs.h -- C ABI of the MI355X (gfx950) FFT binned angular bispectrum library.
 *
 * The estimator is the one of Gill, Bharadwaj, Ali & Elahi (2024), "A visibility-based
 * angular bispectrum estimator for radio-interferometric data":
 *   - visibilities are gridded onto a uv grid of spacing dU_g (Sec. 2, Eq. 9);
 *   - the grid is cut into annular rings a_m (Sec. 2, the ring construction);
 *   - per ring, the data field D_m (Eq. 10) and the weight field I_m (Eq. 11) are
 *     inverse Fourier transforms of the ring-restricted W V and W;
 *   - for every ring triplet, B-hat = (1/A) sum_theta D1 D2 D3 / sum_theta I1 I2 I3 (Eq. 12),
 *     the weighted average over all closed triangles with one vertex per ring.
 *
 * Conventions shared by every call:
 *   - grids are n x n, row-major, row index = v cell, column index = u cell, DC at
 *     [0][0]; index i stands for the signed cell i < n/2 ? i : i - n;
 *   - a cell g belongs to ring m iff edges[m]^2 <= |g|^2 < edges[m+1]^2, compared as
 *     the exact integer |g|^2 against the FP64 squares of the edges;
 *   - the input is defined through its Hermitian part X(g) = (W V(g) + conj(W V(-g)))/2
 *     and Y(g) = (W(g) + W(-g))/2, so every field is real;
 *   - triplets are stored i <= j <= k (ascending ring index), so ell1 = ell_k,
 *     ell2 = ell_j, ell3 = ell_i; a triplet is kept when its rings contain at least
 *     one closed lattice triangle (decided exactly on the host);
 *   - reported sums are per triangle: S_t = (1/n^2) sum_theta D_i D_j D_k equals the sum
 *     of X(g1) X(g2) X(g3) over closed triangles, N_t likewise with Y, and
 *     B_t = S_t / (A N_t);
 *   - empty triplets (Eq. 12 has no weighted triangle to average): weights are taken to
 *     be non-negative, so every closed triangle whose three cells carry weight adds at
 *     least w_min^3 to N_t, w_min being the smallest non-zero Y over the cells of all
 *     rings (1 for unit weights); where N_t < w_min^3 / 2 the triplet has no weighted
 *     triangle, its N_t is rounding noise of an exact zero, and B_t is NaN (N_t is still
 *     reported);
 *   - device pointers are caller-owned and must stay valid until the stream work that
 *     uses them has finished; the library never allocates device memory (the one static
 *     array it holds is the scratch of abs_estimate_noalloc);
 *   - every function returns a status code; none aborts or prints.  Launch or device
 *     errors surface as ABS_ERR_DEVICE from the call that saw them or from abs_sync;
 *   - `stream` arguments are hipStream_t values passed as void* (NULL = default stream).
 */
#ifndef ABS_H_
#define ABS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum abs_status {
  ABS_OK = 0,
  ABS_ERR_INVALID = 1,  /* bad argument: null pointer, size, mode, alignment, batch */
  ABS_ERR_ALIAS = 2,    /* rings reach |g| > n/3, where triangles wrap, without ABS_ALLOW_WRAP */
  ABS_ERR_UNBOUND = 3,  /* the plan has no device memory yet (see abs_plan_bind) */
  ABS_ERR_DEVICE = 4,   /* a HIP runtime call or kernel launch failed */
  ABS_ERR_JIT = 5,      /* run-time compilation of the plan's contraction kernel failed */
  ABS_ERR_NOMEM = 6,    /* host allocation failed, or a caller buffer is too small */
  ABS_ERR_EMPTY = 7,    /* no ring triplet contains a closed lattice triangle */
  ABS_ERR_SCRATCH = 8   /* abs_estimate_noalloc: the call needs more than its static scratch */
} abs_status;

/* precision of the triplet contraction (the ring FFTs are always FP32); the split forms run
 * on the matrix units wherever the plan's cost model expects that to be faster than the
 * FP32 kernel (see ABS_ALL_MFMA) */
enum { ABS_FP32 = 0, ABS_BF16X3 = 1, ABS_FP16X3 = 2 };
/* weight modes (Sec. 2, the paragraph after Eq. 10) */
enum { ABS_W_UNIT = 0,      /* W = 1 on every ring cell                                */
       ABS_W_INV_COUNT = 1, /* w holds gridded counts N_g: W = 1/N_g if N_g >= 0.5 else 0 */
       ABS_W_GIVEN = 2 };   /* w holds W itself (must be symmetric, W(-g) = W(g))      */
/* element type of the gridded visibilities passed to abs_estimate */
enum { ABS_C64 = 0, ABS_C128 = 1 };
/* gridding kernels (Eq. 9) */
enum { ABS_NEAREST = 0, ABS_GAUSS7 = 1 };
/* plan flags */
#define ABS_ALLOW_WRAP 1u /* accept rings beyond n/3: triangles then close modulo n */
#define ABS_ALLOW_DC 2u   /* accept edges[0] == 0, i.e. a ring holding g = 0 (tests) */
#define ABS_EVERY_LEVEL 4u /* run every resolution level n/2 .. n/levels that holds a    */
                           /* triplet, instead of the set the cost model picks (tests) */
#define ABS_ALL_MFMA 8u    /* precision forms: contract every level on the matrix units; */
                           /* without it a level whose triplets fill few 16 x 16 tiles  */
                           /* is contracted by the FP32 kernel (faster there, and more  */
                           /* accurate)                                                 */

typedef struct abs_plan_s* abs_plan_t;

typedef struct abs_plan_desc {
  int32_t n;            /* grid side, power of two, 16 <= n <= 8192                    */
  int32_t nbins;        /* number of rings, 1 <= nbins <= 64                          */
  const double* edges;  /* host, nbins + 1 strictly increasing radii in grid cells;   */
                        /* copied by abs_plan                                         */
  double du;            /* grid spacing dU_g in wavelengths (Eq. 9, Sec. 3); labels   */
                        /* use ell = 2 pi du |g| and gridding uses g = rint(U / du)    */
  double norm;          /* the A of Eq. (12); <= 0 selects pi theta0^2 / 3             */
  double theta0;        /* Gaussian beam width of Eq. (6) in radians, for ABS_GAUSS7   */
                        /* and the default norm; <= 0 selects 0.6 x 24.68 deg          */
  int32_t precision;    /* ABS_FP32, ABS_BF16X3 or ABS_FP16X3                          */
  int32_t wmode;        /* ABS_W_UNIT, ABS_W_INV_COUNT or ABS_W_GIVEN                  */
  int32_t max_batch;    /* largest batch abs_estimate / abs_grid will be given (>= 1) */
  uint32_t flags;       /* ABS_ALLOW_WRAP | ABS_ALLOW_DC | ABS_EVERY_LEVEL | ABS_ALL_MFMA */
  int32_t levels;       /* largest n / m of a resolution level: a power of two; 1 runs */
                        /* every triplet at n; 0 selects 4 (2 for ABS_BF16X3).  A     */
                        /* triplet i <= j <= k with h_i + h_j + h_k < m and 2 h_k < m  */
                        /* (h: a ring's largest |g_x|) closes exactly the same         */
                        /* triangles on an m x m grid (Eqs. 10-12 summed over m^2      */
                        /* pixels), so it may be evaluated there; the plan picks its   */
                        /* levels by a cost model.  Larger ratios save more work but   */
                        /* average rounding errors over fewer pixels (a level's error  */
                        /* grows about as n / m)                                       */
  int32_t nchan;        /* channels of a multi-frequency plan (0 or 1: one channel).   */
                        /* With nchan = C > 1 (C x nbins <= 64) the plan estimates the */
                        /* multi-frequency angular bispectrum, Eq. (12) with the three  */
                        /* fields taken at channels a, b, c (Sec. 1 names the multi-   */
                        /* frequency and 3-D bispectrum as the next step): triplets run */
                        /* over channel rings s = c nbins + r, every non-decreasing     */
                        /* (s1, s2, s3) whose rings, sorted, form a plan triplet; each  */
                        /* grid of a call is C consecutive channel grids               */
} abs_plan_desc;

typedef struct abs_plan_info {
  int32_t n, nbins;
  int64_t ntrip;        /* number of ring triplets the plan evaluates                  */
  int64_t npairs;       /* distinct (i, j) ring pairs among them                      */
  int64_t ncols;        /* half-plane uv columns the ring FFTs touch, summed over rings */
  int64_t plan_bytes;   /* device bytes abs_plan_bind needs                           */
  double norm;          /* the A actually used                                        */
  int64_t mfma_tiles;   /* 16 x 16 output tiles of the precision-form contraction     */
  int32_t jit_parts;    /* separately compiled pieces of the contraction code         */
  /* code variants the plan selected (reported for tests and tuning):                  */
  int32_t contract_parts;  /* code parts of the FP32 data kernel (0: precision form)   */
  int32_t contract_jk;     /* 1: triplets formed as (D_j D_k) D_i, 0: as (D_i D_j) D_k */
  int32_t contract_block;  /* triplet order in blocks of this many j (0: none)         */
  int32_t contract_waves;  /* waves per workgroup (triplet groups of one slice)        */
  int32_t weight_parts, weight_jk, weight_block, weight_waves;  /* same, FP64 kernel  */
  int32_t mfma_tiles_per_wave;  /* precision form: output tiles a wave owns (2 or 12)  */
  int32_t mfma_depth;           /* precision form: chunks of loads in flight (1 or 4)  */
  int32_t nlevels;              /* resolution levels the plan runs (1: none below n);  */
                                /* with several, the variants above are the first     */
                                /* (largest) level's and the counts are summed        */
  int32_t ring0;                /* abs_plan_level_info: the level's first ring (its   */
                                /* nbins rings are ring0 .. ring0 + nbins - 1); 0 here */
  int32_t nchan;                /* channels (1 unless a multi-frequency plan)          */
} abs_plan_info;

/* Build a plan on the host: rings (Sec. 2), the triplet list with an exact lattice
 * test (Sec. 3: all ring triplets, each kept when its rings hold a closed lattice
 * triangle), per-triplet labels and the device tables.  No HIP call is made.
 * Errors: ABS_ERR_INVALID (n not a power of two in [16, 8192], nbins out of range,
 * edges not strictly increasing or negative, edges[0] == 0 without ABS_ALLOW_DC,
 * bad mode, max_batch < 1, levels not 0 or a power of two <= n), ABS_ERR_ALIAS (edges[nbins] > n/3 without ABS_ALLOW_WRAP,
 * or any ring reaching |g| >= n/2), ABS_ERR_EMPTY, ABS_ERR_NOMEM. */
abs_status abs_plan(const abs_plan_desc* desc, abs_plan_t* out);

/* Sizes and counts of a plan (host only). */
abs_status abs_plan_info_get(abs_plan_t plan, abs_plan_info* out);

/* One resolution level of a plan (host only), 0 <= level < nlevels, largest first: its
 * grid side m (info->n), the rings ring0 .. ring0 + nbins - 1 it transforms, its
 * triplets (ntrip, npairs) and code variants; plan_bytes is 0 (the tables live in the
 * parent's memory).  tmap:
 * host int32 [info->ntrip], the index in the plan's triplet list of each of the level's
 * triplets (ascending), or NULL.  A plan without levels reports itself as level 0.
 * Errors: ABS_ERR_INVALID. */
abs_status abs_plan_level_info(abs_plan_t plan, int32_t level, abs_plan_info* info, int32_t* tmap);

/* Host copies of the triplet list, labels and ring radii; any pointer may be NULL.
 *   ijk      int32  [ntrip][3]  ring indices i <= j <= k (multi-frequency plans: channel
 *                               rings s = c nbins + r, s1 <= s2 <= s3; labels then come
 *                               from the rings sorted by size)
 *   labels   double [ntrip][5]  (ell1, ell2, ell3, mu, t) from the rings' mean radii,
 *                               ell = 2 pi du <|g|>, mu = (l1^2 + l2^2 - l3^2) / (2 l1 l2),
 *                               t = l2 / l1 (Sec. 2, below Eq. 3 and after Eq. 12)
 *   radius   double [nbins]     unweighted mean |g| of each ring's lattice cells */
abs_status abs_plan_triplets(abs_plan_t plan, int32_t* ijk, double* labels, double* radius);

/* Compile the plan's contraction code for gfx950 (host only, no device needed): every
 * part in turn.  The code is generated per triplet list and cut into jit_parts pieces
 * (runs of triplet groups) that compile independently.  abs_plan_bind compiles what has
 * not been compiled or installed.  Errors: ABS_ERR_JIT. */
abs_status abs_plan_compile(abs_plan_t plan);

/* Compile one part, 0 <= part < jit_parts.  Errors: ABS_ERR_INVALID, ABS_ERR_JIT. */
abs_status abs_plan_compile_part(abs_plan_t plan, int32_t part);

/* A part's compiled code object, for caching or for compiling the parts of one or many
 * plans in several processes (run-time compilation is serialised within one process).
 *   part   0 <= part < jit_parts
 *   key    out: identifies the part's generated source and compile options (may be NULL)
 *   dst    NULL: compile the part if needed and return the size in *bytes; otherwise
 *          copy the code object into dst (host, *bytes long) and set *bytes to its size
 * Errors: ABS_ERR_INVALID (bad part, dst given before compilation), ABS_ERR_NOMEM
 * (*bytes too small), ABS_ERR_JIT. */
abs_status abs_plan_code(abs_plan_t plan, int32_t part, uint64_t* key, void* dst, size_t* bytes);

/* Install a part's code object obtained from abs_plan_code of an identical plan (same
 * key); abs_plan_bind then loads it instead of compiling.  The bytes are copied.
 * Errors: ABS_ERR_INVALID (null, empty, bad part or key mismatch). */
abs_status abs_plan_set_code(abs_plan_t plan, int32_t part, uint64_t key, const void* src,
                             size_t bytes);

/* Attach caller-owned device memory of at least plan_bytes bytes (256-byte aligned)
 * to the plan, upload its tables on `stream` and load the compiled kernel on the
 * current device; also create, on that device, the plan's second stream (non-blocking,
 * default priority) and two events, which abs_destroy releases.  The memory must outlive
 * the plan's use.  Errors: ABS_ERR_INVALID, ABS_ERR_NOMEM (bytes too small), ABS_ERR_JIT,
 * ABS_ERR_DEVICE. */
abs_status abs_plan_bind(abs_plan_t plan, void* plan_mem, size_t bytes, void* stream);

/* Device workspace needed by abs_estimate for `batch` grids, when the weights are
 * per grid (w_batched = 1), shared (0), or replaced by cached counts (n_given != NULL,
 * pass have_counts = 1). */
abs_status abs_estimate_workspace(abs_plan_t plan, int32_t batch, int32_t w_batched,
                                  int32_t have_counts, size_t* bytes);

/* Device workspace needed by abs_grid for `nvis` baselines and `batch` realisations
 * (nvis < 2^31). */
abs_status abs_grid_workspace(abs_plan_t plan, int64_t nvis, int32_t batch, size_t* bytes);

/* Gridding, Eq. (9): each visibility goes to the cell g = rint(U / du) (round half to
 * even, FP64) and, because the sky is real (Eq. 4), its conjugate goes to -g.
 * Visibilities with any |g| component >= n/2 are dropped and counted.
 *   nvis     number of visibilities (baselines), >= 0
 *   batch    realisations sharing the baselines, 1 <= batch <= max_batch (max_batch x
 *            nchan for a multi-frequency plan: one per channel grid)
 *   uv       device double [nvis][2]  (u, v) in wavelengths
 *   vis      device float  [batch][nvis][2]  (re, im)
 *   vis_w    device float  [nvis] per-visibility weights, or NULL for 1
 *   kernel   ABS_NEAREST (w~ = 1 at the nearest cell) or ABS_GAUSS7
 *            (w~ = exp(-pi^2 theta0^2 |U_g - U|^2) on the 7 x 7 cells around it)
 *   work     device workspace of abs_grid_workspace bytes
 *   grid     device float  [batch][n][n][2]  V_g, overwritten
 *   wsum     device float  [n][n]  N_g = sum of w~ x vis_w, overwritten; may be NULL
 *   dropped  device int64  [1]  number of dropped visibilities, overwritten; may be NULL
 * The visibilities are sorted by nearest cell and every cell gathers its own sum in
 * 64-bit fixed point, so results are bitwise reproducible.  Errors: ABS_ERR_INVALID,
 * ABS_ERR_UNBOUND, ABS_ERR_NOMEM, ABS_ERR_DEVICE. */
abs_status abs_grid(abs_plan_t plan, int64_t nvis, int32_t batch, const double* uv,
                    const float* vis, const float* vis_w, int32_t kernel, void* work,
                    size_t work_bytes, float* grid, float* wsum, int64_t* dropped,
                    void* stream);

/* Gridding of many batches of visibilities on one baseline set (the paper's simulations
 * draw every realisation on one baseline distribution, Sec. 3), Eq. (9) with the nearest
 * cell and unit weights: the baselines are sorted once (abs_grid_sort), the caller keeps
 * its visibilities in the sorted slot order as records of the batch's values (slot-major),
 * and every later gridding (abs_grid_sorted) reads each record once and writes each cell
 * once.
 *
 * Slot order: the mirror pairs of cells (g, -g) in the order of their representative cell
 * (rows 0 .. n/2 of the grid, row-major; in rows 0 and n/2 columns 0 .. n/2 only), and in
 * each pair the visibilities whose nearest cell is g before those nearest to -g.  Within
 * one cell the order is unspecified and may differ between sorts of the same baselines;
 * the grids do not depend on it.
 *
 * Sizes for a plan (its n) and nvis baselines (nvis < 2^31): the baseline set, kept while
 * it is used ((n/2 + 1) n x 8 + 4 bytes), and the scratch abs_grid_sort uses.  Either
 * output pointer may be NULL.  Errors: ABS_ERR_INVALID. */
abs_status abs_grid_sort_workspace(abs_plan_t plan, int64_t nvis, size_t* set_bytes, size_t* work_bytes);

/* Sort nvis baselines (Eq. 9's nearest cell, as abs_grid: round half to even in FP64;
 * baselines with any |g| component >= n/2 are dropped).
 *   uv      device double [nvis][2]  (u, v) in wavelengths
 *   set     device buffer of set_bytes: receives the run table of the set (int32 [(n/2 + 1)
 *           n x 2 + 1]: entry 2 lc is where pair lc's slots start, 2 lc + 1 where its -g
 *           slots start; the last entry is the number kept); owned by the caller
 *   work    device scratch of work_bytes, free again once the call's work has run
 *   perm    device int32 [nvis]: perm[k] = the index (into uv) of the baseline in slot k
 *           for k < kept, -1 from kept on
 *   wsum    device float [n][n]: N_g, the number of visibilities at g plus those at -g
 *           (unit weights); may be NULL
 *   kept    device int64 [1]: number of baselines kept (nvis minus those dropped); may be NULL
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID, ABS_ERR_UNBOUND, ABS_ERR_NOMEM,
 * ABS_ERR_DEVICE. */
abs_status abs_grid_sort(abs_plan_t plan, int64_t nvis, const double* uv, void* set, size_t set_bytes,
                         void* work, size_t work_bytes, int32_t* perm, float* wsum, int64_t* kept,
                         void* stream);

/* Reorder visibilities into slot-order records once: out[k][b] = vis[b][perm[k]] for
 * k < ld (0 where perm[k] is -1).
 *   vis   device float [batch][nvis][2];  out  device float [ld][batch][2], ld <= nvis
 *   perm  as abs_grid_sort returned it
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID, ABS_ERR_DEVICE. */
abs_status abs_grid_permute(abs_plan_t plan, int64_t nvis, int32_t batch, const int32_t* perm, int64_t ld,
                            const float* vis, float* out, void* stream);

/* Eq. (9) on a sorted baseline set: the same grids abs_grid gives for the nearest cell
 * and unit weights, bit for bit (both sum each pair of cells (g, -g) exactly, in FP64, or in
 * 64-bit fixed point with a scale from that pair's own values when their magnitudes span
 * too wide a range for that; neither depends on the order of the visibilities).
 *   set     the set from abs_grid_sort (any plan of the same n may use it)
 *   batch   1 <= batch <= max_batch (x nchan)
 *   ld      slots (records) in vis; slots from ld on are not read (give at least the kept
 *           count, or their visibilities are left out)
 *   vis     device float [ld][batch][2]: the batch's values of each slot, in slot order
 *           (abs_grid_permute, or produced so)
 *   grid    device float [batch][n][n][2]  V_g, overwritten
 *   wsum    device float [n][n]  N_g of the slots read, overwritten; may be NULL
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID, ABS_ERR_UNBOUND, ABS_ERR_NOMEM,
 * ABS_ERR_DEVICE. */
abs_status abs_grid_sorted(abs_plan_t plan, const void* set, size_t set_bytes, int32_t batch, int64_t ld,
                           const float* vis, float* grid, float* wsum, void* stream);

/* The estimator, Eqs. (10)-(12), for `batch` gridded-visibility arrays.
 *   batch      1 <= batch <= max_batch
 *   dtype      ABS_C64 (float pairs) or ABS_C128 (double pairs, rounded to FP32 on load)
 *   grids      device [batch][n][n] complex ([batch][nchan][n][n] for a multi-frequency
 *              plan: w, if batched, likewise; shared weights are one [n][n] array for every
 *              channel)
 *   w          device float [n][n] (w_batched = 0) or [batch][n][n] (w_batched = 1),
 *              interpreted by the plan's wmode; may be NULL only for ABS_W_UNIT
 *   n_given    device double [ntrip] weighted triangle counts N_t previously returned
 *              for these same weights (abs_counts), or NULL; when given, the weight
 *              fields are not recomputed (requires w_batched = 0)
 *   work       device workspace of abs_estimate_workspace bytes
 *   B          device double [batch][ntrip]  B_t = S_t / (A N_t), overwritten
 *   N          device double [batch][ntrip]  N_t, overwritten; may be NULL
 * Asynchronous on `stream`.  When the weight fields are computed (n_given NULL), they run
 * on the plan's second stream, forked from `stream` after the call's first launch and
 * joined back into it before the normalisation, so that they overlap the data fields;
 * work queued on `stream` after the call sees the whole result.  Calls on one plan from
 * several host threads at once must be serialised by the caller.  Errors: ABS_ERR_INVALID,
 * ABS_ERR_UNBOUND, ABS_ERR_NOMEM, ABS_ERR_DEVICE. */
abs_status abs_estimate(abs_plan_t plan, int32_t batch, int32_t dtype, const void* grids,
                        const float* w, int32_t w_batched, const double* n_given,
                        void* work, size_t work_bytes, double* B, double* N, void* stream);

/* The estimator for general complex gridded visibilities (Eq. 10 taken literally: the ring
 * fields D_m of W V are complex, with no Hermitian symmetrisation), giving a complex B_t
 * = S_t / (A N_t) with S_t = (1/n^2) sum_theta D_i D_j D_k, i.e. the sum of X(g1) X(g2)
 * X(g3) over closed triangles with X = W V.  For Hermitian input Im B_t = 0 and Re B_t
 * equals abs_estimate's B_t.  Computed as four real passes of the same kernels: with
 * W V = H + i G (H, G Hermitian), the triple sums of H, G, H + G and H - G combine into
 * Re S and Im S.  Arguments as abs_estimate, except:
 *   work   device workspace of abs_estimate_complex_workspace bytes (four data sets a grid)
 *   B      device double [batch][ntrip][2]  (Re B_t, Im B_t), NaN for empty triplets
 * The weights must be real, non-negative and symmetric as for abs_estimate.  Errors: as
 * abs_estimate; ABS_ERR_INVALID for a multi-frequency plan. */
abs_status abs_estimate_complex_workspace(abs_plan_t plan, int32_t batch, int32_t w_batched, int32_t have_counts,
                                          size_t* bytes);
abs_status abs_estimate_complex(abs_plan_t plan, int32_t batch, int32_t dtype, const void* grids, const float* w,
                                int32_t w_batched, const double* n_given, void* work, size_t work_bytes,
                                double* B, double* N, void* stream);

/* abs_estimate without a caller workspace and without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The arguments are those of abs_estimate minus work / work_bytes; the
 * workspace is a static device array of 256 MiB (ABS_NOALLOC_SCRATCH_BYTES), one per GPU,
 * held from the first such call on that GPU until the process ends.  A call whose
 * workspace (abs_estimate_workspace) exceeds it returns ABS_ERR_SCRATCH and launches
 * nothing; e.g. one 1024^2 grid with 20 rings and its own weights fits, 1024^2 batches of
 * more than one do not.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (on different streams, or from several threads) race and must be serialised
 * by the caller.  Nothing in the array needs to start at zero (each call writes what it
 * reads).  Errors: those of abs_estimate, ABS_ERR_SCRATCH. */
#define ABS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
abs_status abs_estimate_noalloc(abs_plan_t plan, int32_t batch, int32_t dtype, const void* grids,
                                const float* w, int32_t w_batched, const double* n_given,
                                double* B, double* N, void* stream);

/* Weighted triangle counts N_t (the denominator of Eq. 12 per triangle) for one
 * weight array, for reuse as abs_estimate's n_given.  work: abs_estimate_workspace
 * (plan, 0, 0, 0) bytes.  N: device double [ntrip]. */
abs_status abs_counts(abs_plan_t plan, const float* w, void* work, size_t work_bytes,
                      double* N, void* stream);

/* ---- after the estimator: re-binning, ensemble statistics, model prediction ---------
 * Secs. 3-4: the triplet estimates are averaged in bins of (ell1, mu, t), ell1 in bins of
 * equal logarithmic width and mu, t in equal linear bins of [0.5, 1], weighted by their
 * triangle counts; an ensemble of realisations gives the mean and sigma per bin, compared
 * with the local quadratic model averaged over the same lattice triangles, [B_Ana]_d. */

/* Bin of every triplet, from the plan's labels (host only).
 *   nl1, l1_edges  host double [nl1 + 1] increasing ell1 edges; bins are [lo, hi)
 *   nmu, nt        equal bins of 0.5 <= mu, t <= 1 (the paper uses 5 and 5); a label
 *                  below 0.5 or above 1 (mean radii of wide rings need not close a
 *                  triangle) counts in the end bin
 *   bin_of_triplet host int32 [ntrip]: (l1_bin * nmu + mu_bin) * nt + t_bin, or -1 when
 *                  ell1 lies outside the edges
 * Errors: ABS_ERR_INVALID. */
abs_status abs_rebin_table(abs_plan_t plan, int32_t nl1, const double* l1_edges, int32_t nmu, int32_t nt,
                           int32_t* bin_of_triplet);

/* Triangle-weighted bin averages for `batch` grids: Bbin[g][k] = sum N_t B_t / sum N_t over
 * the triplets of bin k whose B_t is not NaN (Eq. 12 over the union of the bin's
 * triangles), Nbin[g][k] = sum N_t; a bin without triplets gets NaN and 0.  Sums run in
 * triplet order (FP64).  All pointers are device memory:
 *   bin_of_triplet int32 [ntrip] (abs_rebin_table), B, N double [batch][ntrip] (from
 *   abs_estimate), Bbin, Nbin double [batch][nbins].
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID, ABS_ERR_DEVICE. */
abs_status abs_rebin(abs_plan_t plan, int32_t nbins, const int32_t* bin_of_triplet, int32_t batch,
                     const double* B, const double* N, double* Bbin, double* Nbin, void* stream);

/* Ensemble statistics over realisations (Sec. 3) and deviations from a model (Sec. 4):
 *   X       device double [nreal][nvals] (e.g. abs_rebin's Bbin of nreal realisations)
 *   mean    device double [nvals]: mean over the realisations
 *   sigma   device double [nvals]: sqrt(<X^2> - mean^2) (the ensemble sigma, no Bessel
 *           correction)
 *   model   device double [nvals] or NULL; with it, dB = |mean - model| / model and
 *           dsigma = |mean - model| / sigma (either may be NULL)
 * Realisations are added in order (FP64).  Asynchronous.  Errors: ABS_ERR_INVALID
 * (dB or dsigma without model), ABS_ERR_DEVICE. */
abs_status abs_ensemble(int32_t nreal, int32_t nvals, const double* X, const double* model, double* mean,
                        double* sigma, double* dB, double* dsigma, void* stream);

/* Device workspace of abs_model_discrete. */
abs_status abs_model_workspace(abs_plan_t plan, size_t* bytes);

/* [B_Ana]_d per triplet: the first-order bispectrum of the local quadratic model (Eq. 14),
 * 2 f (C1 C2 + C2 C3 + C3 C1), averaged over the triplet's closed lattice triangles with
 * the weights Y1 Y2 Y3 of Eq. (12)'s denominator (Sec. 4, the discretely sampled
 * prediction).  The weighted triangle sum is trilinear in the weights, so the pair term is
 * taken from three runs of the FP64 weight path with weights Y (1 + s C / max C),
 * s = +1, -1, 0.
 *   w      device float [n][n] weights as the plan's wmode reads them (NULL for unit)
 *   c      device float [n][n] the model C at every cell (e.g. C_ell at ell = 2 pi du |g|),
 *          taken through its even part (c(g) + c(-g)) / 2, non-negative
 *   f      f_NG / sigma_T of Eq. (13)
 *   work   device, abs_model_workspace bytes, 256-byte aligned
 *   out    device double [ntrip]; NaN for empty triplets (as B_t)
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID (also for a multi-frequency plan),
 * ABS_ERR_UNBOUND, ABS_ERR_NOMEM, ABS_ERR_DEVICE. */
abs_status abs_model_discrete(abs_plan_t plan, const float* w, const float* c, double f, void* work,
                              size_t work_bytes, double* out, void* stream);

/* ---- before gridding: visibilities of a simulated sky ---------------------------------
 * Eq. (4): V(U) = Q int d^2 theta A(theta) dT(theta) exp(+2 pi i U . theta) on a flat sky
 * grid (Sec. 3 simulates the sky on a flat grid, multiplies it by the primary beam of
 * Eq. 5 and transforms it to the baselines by a DFT).  For N x N pixels of side dtheta,
 * pixel (a, b) (a: column, theta_x; b: row, theta_y) sits at ((a - N/2), (b - N/2)) dtheta
 * and V(U) = q dtheta^2 sum_ab A(theta_ab) sky_ab exp(+2 pi i (u theta_x + v theta_y)),
 * periodic in u and v with period 1/dtheta.  Evaluated as a type-2 non-uniform FFT (a
 * zero-padded 2-D FFT on the twice-oversampled 2N grid, then an 8 x 8 "exponential of
 * semicircle" interpolation per baseline, with the kernel's transform divided out of the
 * sky first): the result matches the direct sum within about 1e-6 of the visibilities' rms
 * (FP32 transforms; the kernel's own error is about 1e-7). */
enum { ABS_BEAM_NONE = 0,   /* A = 1                                                       */
       ABS_BEAM_MWA = 1,    /* Eq. (5): sinc^2(pi d theta_x / lambda) sinc^2(pi d theta_y / lambda), */
                            /* beam_param = d / lambda (tile side in wavelengths)         */
       ABS_BEAM_GAUSS = 2 };/* Eq. (6): exp(-theta^2 / theta0^2), beam_param = theta0 (radians) */

/* Device workspace of abs_simulate for an nsky x nsky sky (16 <= nsky <= 4096, a power of
 * two): about 48 nsky^2 bytes, reused for every sky of a batch. */
abs_status abs_simulate_workspace(int32_t nsky, size_t* bytes);

/* Visibilities of `batch` skies at nvis baselines.
 *   dtheta     pixel side (radians), > 0
 *   beam, beam_param   ABS_BEAM_* and its parameter (ignored for ABS_BEAM_NONE)
 *   q          the Q of Eq. (4) (brightness-temperature to intensity factor)
 *   sky        device float [batch][nsky][nsky], row b = theta_y index, column a = theta_x
 *   uv         device double [nvis][2], baselines (u, v) in wavelengths
 *   vis        device float [batch][nvis][2], (Re V, Im V), overwritten
 *   work       device workspace of abs_simulate_workspace bytes, 256-byte aligned
 * Asynchronous on `stream`.  Errors: ABS_ERR_INVALID, ABS_ERR_NOMEM, ABS_ERR_DEVICE. */
abs_status abs_simulate(int32_t nsky, double dtheta, int32_t beam, double beam_param, double q, int32_t batch,
                        const float* sky, int64_t nvis, const double* uv, float* vis, void* work, size_t work_bytes,
                        void* stream);

/* Timing hook: record the caller's HIP events (hipEvent_t passed as void*) on the
 * call's stream immediately before and after the launches of one stage in every later
 * abs_estimate / abs_counts / abs_grid call, until replaced (NULL clears a stage).  While
 * a column- or row-pass hook is set, an estimate's weight fields run after its data fields
 * on the call's stream (not beside them), so that those hooks time the stages alone.
 * Stages: ABS_STAGE_CONTRACT (triplet contraction), ABS_STAGE_COLPASS (column FFT
 * pass), ABS_STAGE_ROWPASS (row FFT pass), ABS_STAGE_GRID (gridding scatter).
 * The events must outlive those calls.  Errors: ABS_ERR_INVALID. */
enum { ABS_STAGE_CONTRACT = 0, ABS_STAGE_COLPASS = 1, ABS_STAGE_ROWPASS = 2, ABS_STAGE_GRID = 3 };
abs_status abs_profile(abs_plan_t plan, int32_t stage, void* ev_begin, void* ev_end);

/* Wait for `stream` and report any device error seen so far. */
abs_status abs_sync(abs_plan_t plan, void* stream);

/* Free the plan's host state (never the caller's device memory). NULL is allowed. */
abs_status abs_destroy(abs_plan_t plan);

/* Static text for a status code. */
const char* abs_status_str(abs_status s);

#ifdef __cplusplus
}
#endif
#endif /* ABS_H_ */
