"""Host-side checks of libabs.so that need no GPU: exported symbols, the plan's
triplet list and labels against the oracle, error codes, and run-time compilation
of the contraction kernel (hiprtc needs no device)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import plan as oplan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "abs.h")


def _A():
    import paper_2412_02246_amd as A
    return A


def test_library_exports_every_declared_symbol():
    A = _A()
    text = open(HDR).read()
    decl = set(re.findall(r"^\s*(?:abs_status|const char\*)\s+(abs_\w+)\s*\(", text, re.M))
    assert {"abs_plan", "abs_grid", "abs_estimate", "abs_destroy", "abs_status_str"} <= decl
    L = ctypes.CDLL(A._lib.LIB_PATH)
    for name in decl:
        assert hasattr(L, name), name


CASES = {
    "c1_128_8log": (128, oplan.log_edges(2.0, 42.0, 8)),
    "c2_1024_20log": (1024, oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20)),
    "paper_22_rings": (1024, oplan.paper_ring_edges()),
    "small_odd": (32, [1.2, 2.0, 3.3, 5.1, 7.0, 10.5]),
    "thin_rings": (64, [1.0, 1.1, 2.3, 2.9, 3.0, 6.2, 9.9, 13.0, 21.0]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_plan_triplets_match_oracle(name):
    A = _A()
    n, e = CASES[name]
    p = A.Plan(n, e)
    trips, _ = oplan.plan_triplets(n, e)
    assert p.ntrip == len(trips)
    assert np.array_equal(p.triplets, trips)
    assert np.allclose(p.radius, oplan.mean_radius(n, e), equal_nan=True)
    assert np.allclose(p.labels, oplan.labels(n, e, trips, 1.0), rtol=1e-12, equal_nan=True)
    assert p.npairs == len({(int(a), int(b)) for a, b, _ in trips})


def test_wrap_plan_matches_cyclic_oracle():
    A = _A()
    n, e = 32, [1.5, 4.0, 7.0, 11.5, 15.0]
    with pytest.raises(A.AbsError) as ei:
        A.Plan(n, e)
    assert ei.value.status == 2          # ABS_ERR_ALIAS
    p = A.Plan(n, e, flags=A.ALLOW_WRAP)
    trips, _ = oplan.plan_triplets(n, e)  # the oracle's FFT counts close triangles mod n
    assert np.array_equal(p.triplets, trips)


@pytest.mark.parametrize("kw,status", [
    (dict(n=100, edges=[1, 2, 3]), 1),          # not a power of two
    (dict(n=32, edges=[2, 2, 3]), 1),           # edges not increasing
    (dict(n=32, edges=[0, 2, 3]), 1),           # DC ring without ALLOW_DC
    (dict(n=32, edges=[1, 2, 11]), 2),          # beyond n/3
    (dict(n=32, edges=[1, 2, 17], flags=1), 2),  # beyond n/2 even with ALLOW_WRAP
    (dict(n=32, edges=[1.1, 1.2]), 7),          # a ring without lattice cells
    (dict(n=32, edges=[1, 2, 3], max_batch=0), 1),
    (dict(n=32, edges=[1, 2, 3], wmode=7), 1),
])
def test_plan_errors(kw, status):
    A = _A()
    with pytest.raises(A.AbsError) as ei:
        A.Plan(**kw)
    assert ei.value.status == status


def test_dc_ring_allowed_with_flag():
    A = _A()
    p = A.Plan(16, [0.0, 0.5, 2.0, 3.5, 5.0], flags=A.ALLOW_DC)
    trips, _ = oplan.plan_triplets(16, [0.0, 0.5, 2.0, 3.5, 5.0])
    assert np.array_equal(p.triplets, trips)


def test_runtime_compilation_without_device():
    A = _A()
    p = A.Plan(128, oplan.log_edges(2.0, 42.0, 8))
    p.compile()   # hiprtc for gfx950 on the host


def test_workspace_sizes():
    A = _A()
    n, e = CASES["c2_1024_20log"]
    p = A.Plan(n, e, max_batch=4, wmode=A.W_INV_COUNT, levels=1)   # one level: the layout below
    shared = p.estimate_workspace(4, False)
    per = p.estimate_workspace(4, True)
    cached = p.estimate_workspace(4, False, True)
    assert cached < shared < per
    # fields dominate: nbins n^2 values per set, FP32 for the 4 data sets; the weight
    # sets (one shared, or one per grid) are FP64 over the half plane, rows 0 .. n/2
    # (n^2/2 + one pixel block of 4096 per ring)
    f = 20 * n * n * 4
    w = 20 * (n * n // 2 + 4096) * 8
    assert 4 * f + w < shared < (4 * f + w) * 1.3
    assert 4 * f + 4 * w < per < (4 * f + 4 * w) * 1.3
    assert 4 * f < cached < 4 * f * 1.2
    g = p.grid_workspace(1 << 20, 2)
    # gridding: cell ids, ranks, lists, counts/offsets and a realisation-minor copy of
    # the values
    assert (1 << 20) * (4 + 4 + 4 + 16) + 2 * n * n * 4 <= g < (1 << 20) * 28 + 2 * n * n * 4 + 8192
    with pytest.raises(A.AbsError):
        p.estimate_workspace(5)
    # a sorted baseline set: the run table, (n/2 + 1) n pairs x 2 sides + 1 int32 entries;
    # the sort's scratch: per baseline its key and rank, per key a count, plus the scan tiles
    import ctypes
    from paper_2412_02246_amd import _lib as L
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lib().abs_grid_sort_workspace(p.handle, 1 << 20, ctypes.byref(sb), ctypes.byref(wb)) == 0
    keys = 2 * (n // 2 + 1) * n
    assert sb.value == (keys + 1) * 4
    assert (1 << 20) * 8 + keys * 4 <= wb.value < (1 << 20) * 8 + keys * 4 + 65536
    assert L.lib().abs_grid_sort_workspace(p.handle, -1, ctypes.byref(sb), None) != 0


def test_jit_parts_code_roundtrip_and_parallel_compile():
    """The contraction code comes in separately compiled parts (at least the FP32 data
    kernel and the FP64 weight kernel); a part's code object moves between identical
    plans by key, and compiling the parts in worker processes gives the same objects."""
    A = _A()
    from paper_2412_02246_amd.jit import compile_parts
    n, e = CASES["c1_128_8log"]
    p = A.Plan(n, e)
    assert p.jit_parts >= 2
    q = A.Plan(n, e)
    codes = [p.code(k) for k in range(p.jit_parts)]
    for k, (key, blob) in enumerate(codes):
        q.set_code(k, key, blob)
    with pytest.raises(A.AbsError):
        q.set_code(0, codes[0][0] ^ 1, codes[0][1])     # key of another source
    with pytest.raises(A.AbsError):
        p.code(p.jit_parts)                              # no such part
    r = A.Plan(n, list(e[:-1]))
    assert r.code(0)[0] != codes[0][0]
    w = A.Plan(n, e)
    compile_parts([w], [w._spec], workers=2)
    assert [w.code(k) for k in range(w.jit_parts)] == codes


def test_code_variants_selected_by_each_plan():
    """Pins which contraction variant every test plan selects (the GPU variant tests compare
    each of them with the oracle on every triplet)."""
    from variant_plans import LEVELS, PLANS, VARIANTS
    A = _A()
    seen = {"contract": set(), "weight": set(), "mfma": set()}
    for name, (n, e) in PLANS.items():
        p = A.Plan(n, e, levels=LEVELS)
        q = A.Plan(n, e, precision=A.BF16X3, levels=LEVELS, flags=A.ALL_MFMA)
        got = dict(contract=p.variants["contract"], weight=p.variants["weight"], mfma=q.variants["mfma"])
        assert got == VARIANTS[name], (name, got)
        assert q.variants["contract"][0] == 0           # the precision form has no FP32 kernel
        assert q.variants["weight"] == p.variants["weight"]
        for k in seen:
            seen[k].add(got[k][1:] if k != "mfma" else got[k])
    # every order (jk plain, ij plain, ij in blocks of 4 / 8 / 16), both workgroup widths,
    # multi-part code and the three precision-form variants occur (ij in blocks of 8 at
    # 8 waves only for the FP64 kernel, jk in blocks never: no plan selects them)
    assert {(1, 0, 4), (1, 0, 8), (0, 0, 8), (0, 4, 4), (0, 8, 4), (0, 4, 8), (0, 16, 8)} <= seen["contract"]
    assert {(1, 0, 4), (1, 0, 8), (0, 0, 4), (0, 0, 8), (0, 4, 8), (0, 8, 8), (0, 16, 8)} <= seen["weight"]
    assert seen["mfma"] == {(2, 1), (12, 4), (12, 1)}
    assert any(VARIANTS[k]["contract"][0] > 1 for k in VARIANTS)
    assert any(VARIANTS[k]["weight"][0] > 2 for k in VARIANTS)


def test_4096_plan_triplets_match_oracle():
    """The 4096^2 / 32-ring plan's triplet list (2309 of 5984 combinations) equals the
    oracle's exact FFT lattice counts."""
    A = _A()
    e = oplan.log_edges(4 * 46 / (2 * np.pi), 4 * 1320 / (2 * np.pi), 32)
    p = A.Plan(4096, e)
    trips, counts = oplan.plan_triplets(4096, e)
    assert np.array_equal(p.triplets, trips)
    assert p.ntrip == 2309 and np.all(counts >= 1)


def _msgpack_uint_after(blob, key):
    """The unsigned integer a msgpack map holds under `key` in a code object's metadata."""
    i = blob.find(key)
    assert i >= 0, key
    b = blob[i + len(key):]
    if b[0] < 0x80:
        return b[0]
    width = {0xcc: 1, 0xcd: 2, 0xce: 4}[b[0]]
    return int.from_bytes(b[1:1 + width], "big")


@pytest.mark.parametrize("which", ["1024x20", "4096x32", "8192x64"])
def test_generated_contraction_kernels_do_not_spill(which):
    """The run-time generated contraction code of the three workloads' plans (FP32 data and
    FP64 weight kernels, every part) compiles without register spills: the triplet groups'
    register estimate keeps spill code (scratch memory in the inner loop) out."""
    A = _A()
    n, nb, mb = {"1024x20": (1024, 20, 16), "4096x32": (4096, 32, 16), "8192x64": (8192, 64, 8)}[which]
    s = n / 1024.0
    e = oplan.log_edges(s * 46 / (2 * np.pi), s * 1320 / (2 * np.pi), nb)
    # the benchmark's batch sizes, which set the resolution levels
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, max_batch=mb)
    p.compile(workers=8)
    for part in range(p.jit_parts):
        _, blob = p.code(part)
        assert _msgpack_uint_after(blob, b".vgpr_spill_count") == 0, (which, part)
        assert _msgpack_uint_after(blob, b".private_segment_fixed_size") == 0, (which, part)


def _ring_h(n, edges):
    """Largest |g_x| of each ring's lattice cells (brute force over the grid)."""
    g = np.arange(-(n // 2), n // 2)
    r2 = g[:, None] ** 2 + g[None, :] ** 2
    gx = np.abs(np.broadcast_to(g[None, :], r2.shape))
    e2 = np.asarray(edges, np.float64) ** 2
    return np.array([gx[(r2 >= e2[m]) & (r2 < e2[m + 1])].max(initial=-1) for m in range(len(edges) - 1)])


LEVEL_CASES = {
    # (n, edges, max_batch, levels, flags, the levels the plan picks: (m, ring0, rings,
    # triplets))
    "mwa1024_b16": (1024, oplan.log_edges(46 / (2 * np.pi), 1320 / (2 * np.pi), 20), 16, 0, 0,
                    [(1024, 15, 5, 9), (512, 0, 20, 681)]),
    "mwa4096_b16": (4096, oplan.log_edges(4 * 46 / (2 * np.pi), 4 * 1320 / (2 * np.pi), 32), 16, 0, 0,
                    [(4096, 24, 8, 23), (2048, 0, 32, 679), (1024, 0, 27, 1607)]),
    "mwa8192_b8": (8192, oplan.log_edges(8 * 46 / (2 * np.pi), 8 * 1320 / (2 * np.pi), 64), 8, 0, 0,
                   [(8192, 48, 16, 109), (4096, 0, 64, 4285), (2048, 0, 54, 10835)]),
    "every_256": (256, oplan.log_edges(3.0, 85.0, 16), 2, 8, 4, None),
    "wrap_128": (128, oplan.log_edges(2.0, 60.0, 12), 2, 8, 5, None),
}


@pytest.mark.parametrize("name", sorted(LEVEL_CASES))
def test_resolution_levels(name):
    """Levels partition the triplets; every level's triplets close their triangles exactly
    on its m x m grid (h_i + h_j + h_k < m and 2 h_k < m, h a ring's largest |g_x|) and sit
    in the smallest of the plan's levels that allows this; a level transforms the rings
    from its smallest i to its largest k; sizes are n / 2^j within the ratio.  The three
    workloads' choices are pinned."""
    A = _A()
    n, e, mb, ratio, flags, want = LEVEL_CASES[name]
    p = A.Plan(n, e, max_batch=mb, levels=ratio, flags=flags)
    got = [(lv["m"], lv["ring0"], lv["nbins"], lv["ntrip"]) for lv in p.levels]
    if want is not None:
        assert got == want, got
    h = _ring_h(n, e)
    T = p.triplets

    def need(t):
        m = 16
        while h[t].sum() >= m or 2 * h[t].max() >= m:
            m *= 2
        return m

    need = np.array([need(t) for t in T])
    sizes = sorted(lv["m"] for lv in p.levels)
    seen = np.zeros(p.ntrip, int)
    for lv in p.levels:
        m, tm = lv["m"], lv["tmap"]
        assert n % m == 0 and (n // m) & (n // m - 1) == 0 and n // m <= (ratio or 4)
        assert np.all(np.diff(tm) > 0)
        seen[tm] += 1
        assert lv["ring0"] == T[tm, 0].min() and lv["ring0"] + lv["nbins"] == T[tm, 2].max() + 1
        if m < n:
            assert np.all(need[tm] <= m), name
        # the smallest level of the plan that fits each triplet
        smallest = np.array([min([s for s in sizes if s >= need[t]] or [n]) for t in tm])
        assert np.array_equal(smallest, np.full(len(tm), m)), name
    assert np.all(seen == 1)
    one = A.Plan(n, e, max_batch=mb, levels=1, flags=flags & ~A.EVERY_LEVEL)
    assert [lv["m"] for lv in one.levels] == [n]
    assert np.array_equal(one.triplets, p.triplets)


def test_levels_argument_checks():
    A = _A()
    e = oplan.log_edges(3.0, 40.0, 8)
    for bad in (-1, 3, 12, 512):
        with pytest.raises(A.AbsError):
            A.Plan(256, e, levels=bad)
