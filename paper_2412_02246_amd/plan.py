"""Python face of the C ABI: a Plan owns an abs plan handle, its device tables (a
torch uint8 tensor) and a reusable workspace.  Methods only check and marshal
arguments; the work is done by libabs.so on the caller's current torch stream."""
import ctypes

import numpy as np

from . import _lib as L


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Plan:
    """A bispectrum plan for one grid size and ring set.

    n, edges    grid side and ring edges in grid cells (Sec. 2 rings)
    du          uv grid spacing in wavelengths (labels, gridding)
    norm        the A of Eq. (12); 0 selects pi theta0^2 / 3
    wmode       W_UNIT, W_INV_COUNT or W_GIVEN
    max_batch   largest batch of grids per call
    flags       ALLOW_WRAP | ALLOW_DC
    levels      largest n / m of a resolution level (1: evaluate every triplet at n;
                0: the library's default)
    nchan       channels of a multi-frequency plan (1: one channel); its triplets run over
                channel rings s = c * nbins + r and each grid of a call is nchan channel
                grids
    """

    def __init__(self, n, edges, du=1.0, norm=0.0, theta0=0.0, precision=L.FP32,
                 wmode=L.W_UNIT, max_batch=1, flags=0, levels=0, nchan=1):
        lib = L.lib()
        e = np.ascontiguousarray(edges, dtype=np.float64)
        self._edges = e
        self._spec = (int(n), tuple(float(x) for x in e),
                      dict(du=float(du), norm=float(norm), theta0=float(theta0),
                           precision=int(precision), wmode=int(wmode), max_batch=int(max_batch),
                           flags=int(flags), levels=int(levels), nchan=int(nchan)))
        d = L.PlanDesc(n=int(n), nbins=len(e) - 1,
                       edges=e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       du=float(du), norm=float(norm), theta0=float(theta0),
                       precision=int(precision), wmode=int(wmode), max_batch=int(max_batch),
                       flags=int(flags), levels=int(levels), nchan=int(nchan))
        h = ctypes.c_void_p()
        L.check(lib.abs_plan(ctypes.byref(d), ctypes.byref(h)), "abs_plan")
        self.handle = h
        info = L.PlanInfo()
        L.check(lib.abs_plan_info_get(h, ctypes.byref(info)), "abs_plan_info_get")
        self.n, self.nbins, self.nchan = info.n, info.nbins, info.nchan
        self.ntrip, self.npairs, self.ncols = info.ntrip, info.npairs, info.ncols
        self.plan_bytes, self.norm = info.plan_bytes, info.norm
        self.mfma_tiles = info.mfma_tiles
        self.jit_parts = info.jit_parts
        # code variants the plan selected: {"contract": (parts, jk, block, waves),
        # "weight": (parts, jk, block, waves), "mfma": (tiles per wave, depth)}
        self.variants = {
            "contract": (info.contract_parts, info.contract_jk, info.contract_block, info.contract_waves),
            "weight": (info.weight_parts, info.weight_jk, info.weight_block, info.weight_waves),
            "mfma": (info.mfma_tiles_per_wave, info.mfma_depth)}
        # resolution levels, largest first: dicts with the level's grid side m, its rings
        # ring0 .. ring0 + nbins - 1, triplets (their indices in self.triplets: "tmap"),
        # pairs and code variants
        self.levels = []
        for lv in range(info.nlevels):
            li = L.PlanInfo()
            tm = np.zeros(max(1, self.ntrip), np.int32)
            L.check(lib.abs_plan_level_info(h, lv, ctypes.byref(li), tm.ctypes.data_as(ctypes.c_void_p)),
                    "abs_plan_level_info")
            self.levels.append(dict(m=li.n, ring0=li.ring0, nbins=li.nbins, ntrip=li.ntrip, npairs=li.npairs,
                                    ncols=li.ncols,
                                    tmap=tm[:li.ntrip].copy(), mfma_tiles=li.mfma_tiles,
                                    contract=(li.contract_parts, li.contract_jk, li.contract_block,
                                              li.contract_waves),
                                    weight=(li.weight_parts, li.weight_jk, li.weight_block, li.weight_waves),
                                    mfma=(li.mfma_tiles_per_wave, li.mfma_depth)))
        self.precision = int(precision)
        self.wmode, self.max_batch = int(wmode), int(max_batch)
        ijk = np.zeros((self.ntrip, 3), np.int32)
        lab = np.zeros((self.ntrip, 5), np.float64)
        rad = np.zeros(self.nbins, np.float64)
        L.check(lib.abs_plan_triplets(h, ijk.ctypes.data_as(ctypes.c_void_p),
                                      lab.ctypes.data_as(ctypes.c_void_p),
                                      rad.ctypes.data_as(ctypes.c_void_p)), "abs_plan_triplets")
        self.triplets, self.labels, self.radius = ijk, lab, rad
        self._mem = None
        self._work = None

    # -- lifetime -------------------------------------------------------------
    def compile(self, workers=1):
        """Compile the contraction code: its parts in turn, or in `workers` worker
        processes (start those before this process first uses the GPU)."""
        if workers > 1 and self.jit_parts > 1:
            from .jit import compile_parts
            compile_parts([self], [self._spec], workers=workers)
        else:
            L.check(L.lib().abs_plan_compile(self.handle), "abs_plan_compile")
        return self

    def code(self, part):
        """(key, bytes) of one compiled part's code object (compiles it if needed)."""
        key, n = ctypes.c_uint64(), ctypes.c_size_t()
        L.check(L.lib().abs_plan_code(self.handle, int(part), ctypes.byref(key), None,
                                      ctypes.byref(n)), "abs_plan_code")
        buf = ctypes.create_string_buffer(n.value)
        L.check(L.lib().abs_plan_code(self.handle, int(part), None, buf, ctypes.byref(n)),
                "abs_plan_code")
        return key.value, buf.raw[:n.value]

    def set_code(self, part, key, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        L.check(L.lib().abs_plan_set_code(self.handle, int(part), ctypes.c_uint64(key), buf,
                                          len(blob)), "abs_plan_set_code")
        return self

    def bind(self, device=None, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(dev):
            self._mem = torch.empty(self.plan_bytes + 256, dtype=torch.uint8, device=dev)
            off = (-self._mem.data_ptr()) % 256
            ptr = ctypes.c_void_p(self._mem.data_ptr() + off)
            L.check(L.lib().abs_plan_bind(self.handle, ptr, self.plan_bytes, _stream(stream)),
                    "abs_plan_bind")
        self.device = dev
        return self

    def close(self):
        if getattr(self, "handle", None) is not None:
            L.lib().abs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspaces -------------------------------------------------------------
    def estimate_workspace(self, batch, w_batched=False, have_counts=False):
        b = ctypes.c_size_t()
        L.check(L.lib().abs_estimate_workspace(self.handle, int(batch), int(bool(w_batched)),
                                               int(bool(have_counts)), ctypes.byref(b)),
                "abs_estimate_workspace")
        return b.value

    def grid_workspace(self, nvis, batch):
        b = ctypes.c_size_t()
        L.check(L.lib().abs_grid_workspace(self.handle, int(nvis), int(batch), ctypes.byref(b)),
                "abs_grid_workspace")
        return b.value

    def _workspace(self, nbytes):
        import torch
        if self._work is None or self._work.numel() < nbytes:
            self._work = None
            self._work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._work

    # -- calls ----------------------------------------------------------------
    def estimate(self, grids, w=None, w_batched=False, n_given=None, out=None, stream=None, work=None):
        """B (and N) for a batch of gridded visibilities.

        grids: torch complex64 / complex128 [batch][n][n] (or [n][n]) on the plan's device;
               [batch * nchan][n][n] for a multi-frequency plan (channels consecutive)
        w:     torch float32 [n][n] or [batch * nchan][n][n] (w_batched), per the plan's wmode
        n_given: torch float64 [ntrip] counts from counts() for the same shared weights
        Returns (B, N), torch float64 [batch][ntrip].
        """
        import torch
        if grids.dim() == 2:
            grids = grids.unsqueeze(0)
        if grids.dtype == torch.complex64:
            dtype = L.C64
        elif grids.dtype == torch.complex128:
            dtype = L.C128
        else:
            raise TypeError("grids must be complex64 or complex128")
        if not grids.is_contiguous():
            raise ValueError("grids must be contiguous")
        if tuple(grids.shape[1:]) != (self.n, self.n) or grids.shape[0] % self.nchan:
            raise ValueError("grids must be [batch * %d][%d][%d]" % (self.nchan, self.n, self.n))
        batch = grids.shape[0] // self.nchan   # multi-frequency: nchan channel grids a grid
        if w is not None:
            if w.dtype != torch.float32 or not w.is_contiguous():
                raise TypeError("w must be a contiguous float32 tensor")
            want = (batch * self.nchan, self.n, self.n) if w_batched else (self.n, self.n)
            if tuple(w.shape) != want:
                raise ValueError("w must have shape %s" % (want,))
        if n_given is not None and (n_given.dtype != torch.float64 or n_given.numel() != self.ntrip):
            raise ValueError("n_given must be float64 [ntrip]")
        nbytes = self.estimate_workspace(batch, w_batched, n_given is not None)
        if work is None:
            work = self._workspace(nbytes)
        elif work.numel() < nbytes:
            raise ValueError("workspace too small: %d < %d bytes" % (work.numel(), nbytes))
        if out is None:
            B = torch.empty((batch, self.ntrip), dtype=torch.float64, device=grids.device)
            N = torch.empty((batch, self.ntrip), dtype=torch.float64, device=grids.device)
        else:
            B, N = out
        L.check(L.lib().abs_estimate(self.handle, batch, dtype, _ptr(grids), _ptr(w),
                                     int(bool(w_batched)), _ptr(n_given), _ptr(work),
                                     work.numel(), _ptr(B), _ptr(N), _stream(stream)),
                "abs_estimate")
        return B, N

    def estimate_complex(self, grids, w=None, w_batched=False, n_given=None, stream=None):
        """Complex B (and N) for general complex grids, without Hermitian symmetrisation:
        (B complex128 [batch][ntrip], N float64 [batch][ntrip])."""
        import torch
        if grids.dim() == 2:
            grids = grids.unsqueeze(0)
        dtype = {torch.complex64: L.C64, torch.complex128: L.C128}.get(grids.dtype)
        if dtype is None or not grids.is_contiguous() or tuple(grids.shape[1:]) != (self.n, self.n):
            raise ValueError("grids must be contiguous complex64 / complex128 [batch][%d][%d]" % (self.n, self.n))
        batch = grids.shape[0]
        if w is not None and (w.dtype != torch.float32 or not w.is_contiguous()):
            raise TypeError("w must be a contiguous float32 tensor")
        b = ctypes.c_size_t()
        L.check(L.lib().abs_estimate_complex_workspace(self.handle, batch, int(bool(w_batched)),
                                                       int(n_given is not None), ctypes.byref(b)),
                "abs_estimate_complex_workspace")
        work = self._workspace(b.value)
        B = torch.empty((batch, self.ntrip, 2), dtype=torch.float64, device=grids.device)
        N = torch.empty((batch, self.ntrip), dtype=torch.float64, device=grids.device)
        L.check(L.lib().abs_estimate_complex(self.handle, batch, dtype, _ptr(grids), _ptr(w), int(bool(w_batched)),
                                             _ptr(n_given), _ptr(work), work.numel(), _ptr(B), _ptr(N),
                                             _stream(stream)), "abs_estimate_complex")
        return torch.view_as_complex(B), N

    def counts(self, w=None, stream=None, work=None):
        import torch
        if work is None:
            work = self._workspace(self.estimate_workspace(0))
        N = torch.empty(self.ntrip, dtype=torch.float64, device=self.device)
        L.check(L.lib().abs_counts(self.handle, _ptr(w), _ptr(work), work.numel(), _ptr(N),
                                   _stream(stream)), "abs_counts")
        return N

    def grid(self, uv, vis, vis_w=None, kernel=L.NEAREST, stream=None):
        """Grid visibilities (Eq. 9).  uv: float64 [nvis][2] (wavelengths);
        vis: complex64 [batch][nvis] or [nvis].  Returns (grid complex64 [batch][n][n],
        wsum float32 [n][n], dropped int64 [1])."""
        import torch
        if vis.dim() == 1:
            vis = vis.unsqueeze(0)
        if uv.dtype != torch.float64 or vis.dtype != torch.complex64:
            raise TypeError("uv must be float64 and vis complex64")
        nvis = uv.shape[0]
        if vis.shape[1] != nvis or not (uv.is_contiguous() and vis.is_contiguous()):
            raise ValueError("vis must be contiguous [batch][nvis] matching uv [nvis][2]")
        batch = vis.shape[0]
        work = self._workspace(self.grid_workspace(nvis, batch))
        grid = torch.empty((batch, self.n, self.n), dtype=torch.complex64, device=uv.device)
        wsum = torch.empty((self.n, self.n), dtype=torch.float32, device=uv.device)
        dropped = torch.empty(1, dtype=torch.int64, device=uv.device)
        L.check(L.lib().abs_grid(self.handle, nvis, batch, _ptr(uv), _ptr(vis), _ptr(vis_w),
                                 int(kernel), _ptr(work), work.numel(), _ptr(grid), _ptr(wsum),
                                 _ptr(dropped), _stream(stream)), "abs_grid")
        return grid, wsum, dropped

    def grid_sort(self, uv, stream=None):
        """Sort a baseline set once (Eq. 9, nearest cell) for gridding many batches of
        visibilities on it with grid_sorted.  uv: float64 [nvis][2] (wavelengths).  Returns
        a BaselineSet (its perm, counts wsum and kept count; the run table stays on the
        device)."""
        import torch
        if uv.dtype != torch.float64 or not uv.is_contiguous() or uv.dim() != 2 or uv.shape[1] != 2:
            raise TypeError("uv must be contiguous float64 [nvis][2]")
        nvis = uv.shape[0]
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        L.check(L.lib().abs_grid_sort_workspace(self.handle, nvis, ctypes.byref(sb), ctypes.byref(wb)),
                "abs_grid_sort_workspace")
        dev = uv.device
        table = torch.empty(sb.value, dtype=torch.uint8, device=dev)
        work = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=dev)
        perm = torch.empty(max(nvis, 1), dtype=torch.int32, device=dev)
        wsum = torch.empty((self.n, self.n), dtype=torch.float32, device=dev)
        kept = torch.empty(1, dtype=torch.int64, device=dev)
        L.check(L.lib().abs_grid_sort(self.handle, nvis, _ptr(uv), _ptr(table), table.numel(), _ptr(work),
                                      work.numel(), _ptr(perm), _ptr(wsum), _ptr(kept), _stream(stream)),
                "abs_grid_sort")
        if stream is None:
            torch.cuda.current_stream(dev).synchronize()
        else:
            stream.synchronize()
        del work
        return BaselineSet(self, table, perm[:nvis], wsum, int(kept.item()))

    def grid_sorted(self, bset, vis, wsum=False, stream=None):
        """Grid visibilities held in bset's slot order (Eq. 9, nearest cell, unit weights).
        vis: complex64 [ld][batch] (each slot's values for the batch) with ld >= bset.kept.
        Returns grid complex64 [batch][n][n], or (grid, wsum float32 [n][n]) with wsum=True."""
        import torch
        if vis.dim() == 1:
            vis = vis.unsqueeze(1)
        if vis.dtype != torch.complex64 or not vis.is_contiguous():
            raise TypeError("vis must be contiguous complex64 [ld][batch]")
        if bset.n != self.n:
            raise ValueError("baseline set of a grid of side %d, plan has %d" % (bset.n, self.n))
        ld, batch = vis.shape
        grid = torch.empty((batch, self.n, self.n), dtype=torch.complex64, device=vis.device)
        ws = torch.empty((self.n, self.n), dtype=torch.float32, device=vis.device) if wsum else None
        L.check(L.lib().abs_grid_sorted(self.handle, _ptr(bset.table), bset.table.numel(), batch, ld,
                                        _ptr(vis), _ptr(grid), _ptr(ws), _stream(stream)), "abs_grid_sorted")
        return (grid, ws) if wsum else grid

    # -- after the estimator (Secs. 3-4) ------------------------------------------
    def rebin_table(self, l1_edges, nmu=5, nt=5):
        """Bin of every triplet (host int32 [ntrip], -1 outside the ell1 edges) and the
        number of bins."""
        e = np.ascontiguousarray(l1_edges, dtype=np.float64)
        out = np.zeros(self.ntrip, np.int32)
        L.check(L.lib().abs_rebin_table(self.handle, len(e) - 1, e.ctypes.data_as(ctypes.c_void_p), int(nmu),
                                        int(nt), out.ctypes.data_as(ctypes.c_void_p)), "abs_rebin_table")
        return out, (len(e) - 1) * int(nmu) * int(nt)

    def rebin(self, B, N, bins, nbins, stream=None):
        """Triangle-weighted bin averages of B [batch][ntrip] (device): (Bbin, Nbin) torch
        float64 [batch][nbins].  bins: device int32 [ntrip] from rebin_table."""
        import torch
        if B.dim() == 1:
            B, N = B.unsqueeze(0), N.unsqueeze(0)
        for t in (B, N):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape[1:]) != (self.ntrip,):
                raise ValueError("B and N must be contiguous float64 [batch][ntrip]")
        if bins.dtype != torch.int32 or bins.numel() != self.ntrip:
            raise ValueError("bins must be int32 [ntrip]")
        Bbin = torch.empty((B.shape[0], nbins), dtype=torch.float64, device=B.device)
        Nbin = torch.empty_like(Bbin)
        L.check(L.lib().abs_rebin(self.handle, int(nbins), _ptr(bins), B.shape[0], _ptr(B), _ptr(N), _ptr(Bbin),
                                  _ptr(Nbin), _stream(stream)), "abs_rebin")
        return Bbin, Nbin

    def model_discrete(self, c, f, w=None, stream=None):
        """[B_Ana]_d per triplet (torch float64 [ntrip]) for the model C at every cell
        (float32 [n][n], device) and f = f_NG / sigma_T, with the plan's weights w."""
        import torch
        for t in (c, w):
            if t is not None and (t.dtype != torch.float32 or tuple(t.shape) != (self.n, self.n)
                                  or not t.is_contiguous()):
                raise ValueError("c and w must be contiguous float32 [n][n]")
        b = ctypes.c_size_t()
        L.check(L.lib().abs_model_workspace(self.handle, ctypes.byref(b)), "abs_model_workspace")
        work = self._workspace(b.value)
        out = torch.empty(self.ntrip, dtype=torch.float64, device=c.device)
        L.check(L.lib().abs_model_discrete(self.handle, _ptr(w), _ptr(c), float(f), _ptr(work), work.numel(),
                                           _ptr(out), _stream(stream)), "abs_model_discrete")
        return out

    def sync(self, stream=None):
        L.check(L.lib().abs_sync(self.handle, _stream(stream)), "abs_sync")


def ensemble(X, model=None, stream=None):
    """Ensemble mean and sigma over axis 0 of X (device float64 [nreal][nvals]), and with a
    model (device float64 [nvals]) Delta_B and Delta_sigma: four torch tensors (the last two
    None without a model)."""
    import torch
    if X.dtype != torch.float64 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous float64 [nreal][nvals] tensor")
    nreal, nv = X.shape
    mean = torch.empty(nv, dtype=torch.float64, device=X.device)
    sigma = torch.empty_like(mean)
    dB = dS = None
    if model is not None:
        if model.dtype != torch.float64 or model.numel() != nv:
            raise ValueError("model must be float64 [nvals]")
        dB, dS = torch.empty_like(mean), torch.empty_like(mean)
    L.check(L.lib().abs_ensemble(nreal, nv, _ptr(X), _ptr(model), _ptr(mean), _ptr(sigma), _ptr(dB), _ptr(dS),
                                 _stream(stream)), "abs_ensemble")
    return mean, sigma, dB, dS


def simulate(sky, dtheta, uv, beam=L.BEAM_NONE, beam_param=0.0, q=1.0, stream=None, work=None):
    """Visibilities of flat-sky brightness fields at baselines (Eq. 4), on the device.

    sky   torch float32 [batch][N][N] or [N][N] (row = theta_y index, column = theta_x),
          pixel (a, b) at ((a - N/2), (b - N/2)) dtheta, N a power of two in [16, 4096]
    uv    torch float64 [nvis][2] baselines in wavelengths
    beam  BEAM_NONE, BEAM_MWA (Eq. 5, beam_param = tile side / wavelength) or BEAM_GAUSS
          (Eq. 6, beam_param = theta0 in radians)
    Returns torch complex64 [batch][nvis]."""
    import torch
    if sky.dim() == 2:
        sky = sky.unsqueeze(0)
    if sky.dtype != torch.float32 or not sky.is_contiguous() or sky.shape[1] != sky.shape[2]:
        raise ValueError("sky must be a contiguous float32 [batch][N][N] tensor")
    if uv.dtype != torch.float64 or not uv.is_contiguous() or uv.dim() != 2 or uv.shape[1] != 2:
        raise ValueError("uv must be a contiguous float64 [nvis][2] tensor")
    batch, nsky, nvis = sky.shape[0], sky.shape[1], uv.shape[0]
    b = ctypes.c_size_t()
    L.check(L.lib().abs_simulate_workspace(nsky, ctypes.byref(b)), "abs_simulate_workspace")
    if work is None or work.numel() < b.value:
        work = torch.empty(b.value + 256, dtype=torch.uint8, device=sky.device)
    off = (-work.data_ptr()) % 256
    vis = torch.empty((batch, nvis), dtype=torch.complex64, device=sky.device)
    L.check(L.lib().abs_simulate(nsky, float(dtheta), int(beam), float(beam_param), float(q), batch, _ptr(sky),
                                 nvis, _ptr(uv), _ptr(vis), ctypes.c_void_p(work.data_ptr() + off),
                                 work.numel() - off, _stream(stream)), "abs_simulate")
    return vis


class BaselineSet:
    """A baseline set sorted by Plan.grid_sort: ``perm`` (int32 [nvis], the baseline index of
    each slot, -1 from ``kept`` on), ``wsum`` (N_g, float32 [n][n]), ``kept`` and the device
    run table.  ``permute`` puts visibilities into slot order once."""

    def __init__(self, plan, table, perm, wsum, kept):
        self._plan = plan
        self.n = plan.n
        self.table, self.perm, self.wsum, self.kept = table, perm, wsum, kept
        self.nvis = perm.numel()

    def permute(self, vis, ld=None, stream=None):
        """vis complex64 [batch][nvis] in baseline order -> records [ld][batch] in slot
        order (ld = kept by default)."""
        import torch
        if vis.dim() == 1:
            vis = vis.unsqueeze(0)
        if vis.dtype != torch.complex64 or not vis.is_contiguous() or vis.shape[1] != self.nvis:
            raise TypeError("vis must be contiguous complex64 [batch][%d]" % self.nvis)
        ld = self.kept if ld is None else int(ld)
        out = torch.empty((ld, vis.shape[0]), dtype=torch.complex64, device=vis.device)
        L.check(L.lib().abs_grid_permute(self._plan.handle, self.nvis, vis.shape[0], _ptr(self.perm), ld,
                                         _ptr(vis), _ptr(out), _stream(stream)), "abs_grid_permute")
        return out
