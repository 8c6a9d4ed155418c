"""Oracle: the binned bispectrum estimator, Eqs. (10)-(12), in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Definition followed (Gill et al. 2024, Sec. 2):
    D(l_m, theta) = sum_{g in a_m} W_g V_g exp(-i l_g . theta)       Eq. (10)
    I(l_m, theta) = sum_{g in a_m} W_g     exp(-i l_g . theta)       Eq. (11)
    B-hat(l1,l2,l3) = (1/A) sum_theta D1 D2 D3 / sum_theta I1 I2 I3  Eq. (12)
with l_g . theta = 2 pi g . x / n on the n x n periodic grid, so each field is a
plain forward 2-D DFT of its masked ring (scipy.fft.fft2, FP64).

Readings of the paper where it is silent or ambiguous:
* the input is defined through its Hermitian part, X(g) = (W V(g) + conj(W V(-g)))/2
  and Y(g) = (W(g) + W(-g))/2, so both fields are real; for Hermitian input this
  is exactly the paper's sum (the imaginary part of the triple sum is zero);
* weights: UNIT (W = 1), INV_COUNT (W = 1/N_g for N_g >= 0.5, else 0, the paper's
  choice with N_g the gridded count) or GIVEN (W supplied);
* reported sums are normalised per triangle: S_t = sum_theta D_i D_j D_k / n^2 and
  N_t = sum_theta I_i I_j I_k / n^2, which equal the sums over closed triangles
  (mod n) of X X X and Y Y Y; B_t = S_t / (A N_t);
* empty triplets: with non-negative weights every closed triangle whose three cells
  are weighted adds at least w_min^3 to N_t, w_min being the smallest non-zero |Y|
  over the cells of all rings (1 for unit weights).  A triplet with
  N_t < w_min^3 / 2 therefore holds no weighted triangle (its N_t is rounding noise
  of an exact zero) and its B_t is NaN; N_t is still reported.

``estimate_multifreq`` takes the three fields of a triplet at three channels (the
multi-frequency form the paper names as its next step, Sec. 1).

Pins: tests/test_oracle_estimator.py (brute force over closed triangles on
n = 8, 16, 32 in cyclic and planar form, integer counts, invariants, the
two-field Parseval special case, zero-mean Gaussian and the closed-form
local-quadratic bispectrum of Eq. 14).
"""
import numpy as np

UNIT, INV_COUNT, GIVEN = 0, 1, 2


def mirror(A):
    """A(-g) on the periodic grid: element [i, j] -> A[-i mod n, -j mod n]."""
    n0, n1 = A.shape[-2:]
    iy = (-np.arange(n0)) % n0
    ix = (-np.arange(n1)) % n1
    return A[..., iy[:, None], ix[None, :]]


def hermitian_part(A):
    return 0.5 * (A + np.conj(mirror(A)))


def effective_weights(n, w, wmode):
    """W_g of Sec. 2 (the paragraph after Eq. 10) for the three weight modes."""
    if wmode == UNIT:
        return np.ones((n, n), np.float64)
    w = np.asarray(w, dtype=np.float64)
    if wmode == INV_COUNT:
        out = np.zeros_like(w)
        ok = w >= 0.5
        out[ok] = 1.0 / w[ok]
        return out
    if wmode == GIVEN:
        return w.copy()
    raise ValueError("unknown weight mode")


def min_weight(Y, masks):
    """w_min of the empty-triplet rule: the smallest non-zero |Y| over the cells that
    lie in any ring (inf when every ring cell has zero weight)."""
    inring = np.any(masks, axis=0)
    a = np.abs(Y[inring])
    a = a[a > 0]
    return float(a.min()) if a.size else np.inf


def ratio(S, N, norm, wmin):
    """B_t = S_t / (A N_t), NaN where N_t < w_min^3 / 2 (no weighted triangle)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        B = S / (norm * N)
    return np.where(N < 0.5 * wmin ** 3, np.nan, B)


def ring_fields(Xfull, masks):
    """Real fields sum_{g in a_m} X(g) exp(-2 pi i g.x / n) for every ring m
    (scipy.fft.fft2, FP64, on all host cores)."""
    import scipy.fft
    return np.stack([scipy.fft.fft2(np.where(m, Xfull, 0), workers=-1).real for m in masks])


def _pairs_of(trips):
    pairs = sorted(set((int(i), int(j)) for i, j, _ in trips))
    return pairs, {p: q for q, p in enumerate(pairs)}


def triple_sums(F, trips, chunk=1 << 16, power=1):
    """sum_theta (F_i F_j F_k)^power / n^2 per triplet, by chunked FP64 GEMM.

    Pair products P_(ij)(theta) = F_i F_j are formed for a chunk of pixels and
    multiplied against F_k; nothing is blocked beyond that.
    """
    trips = [tuple(int(x) for x in t) for t in trips]
    nb = F.shape[0]
    npix = F.shape[1] * F.shape[2]
    Ff = F.reshape(nb, npix)
    pairs, pidx = _pairs_of(trips)
    acc = np.zeros((len(pairs), nb), np.float64)
    pi = np.array([p[0] for p in pairs], dtype=np.int64)
    pj = np.array([p[1] for p in pairs], dtype=np.int64)
    for s in range(0, npix, chunk):
        Fc = Ff[:, s:s + chunk]
        if power != 1:
            Fc = Fc ** power
        P = Fc[pi] * Fc[pj]
        acc += P @ Fc.T
    out = np.array([acc[pidx[(i, j)], k] for i, j, k in trips], dtype=np.float64)
    return out / float(npix)


def estimate(grid, w, edges, norm, wmode=UNIT, trips=None, with_scales=False, chunk=1 << 16):
    """Eq. (12) for one n x n gridded-visibility array.

    grid  : complex [n][n], row index = v cell, column = u cell, DC at [0][0]
    w     : counts / weights [n][n] (ignored for UNIT)
    edges : ring edges (nb + 1, grid units)
    norm  : the normalisation A of Eq. (12)
    trips : (T, 3) i <= j <= k; default = plan.plan_triplets(n, edges)
    Returns a dict with B, S, N (each length T), trips, and with_scales adds the
    FP64 random-error scales rhoS = sqrt(sum (D D D)^2)/n^2, rhoN likewise.
    """
    from . import plan as _plan
    grid = np.asarray(grid).astype(np.complex128)
    n = grid.shape[0]
    if trips is None:
        trips, _ = _plan.plan_triplets(n, edges)
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    W = effective_weights(n, w, wmode)
    masks = _plan.ring_masks(n, edges)
    X = hermitian_part(W * grid)
    Y = hermitian_part(W.astype(np.complex128))
    D = ring_fields(X, masks)
    I = ring_fields(Y, masks)
    S = triple_sums(D, trips, chunk)
    N = triple_sums(I, trips, chunk)
    wmin = min_weight(Y.real, masks)
    B = ratio(S, N, norm, wmin)
    out = dict(B=B, S=S, N=N, trips=trips, wmin=wmin)
    if with_scales:
        out["rhoS"] = np.sqrt(np.maximum(triple_sums(D, trips, chunk, power=2), 0.0) / n ** 2)
        out["rhoN"] = np.sqrt(np.maximum(triple_sums(I, trips, chunk, power=2), 0.0) / n ** 2)
    return out


def estimate_complex(grid, w, edges, norm, wmode=UNIT, trips=None, chunk=1 << 16):
    """Eq. (12) for general complex gridded visibilities, taking Eq. (10) literally: the
    fields D_m of X = W V (no Hermitian symmetrisation) are complex, S_t = sum_theta
    D_i D_j D_k / n^2 is complex and B_t = S_t / (A N_t) (NaN for empty triplets).  Same
    keys as estimate(..., with_scales=True); rhoS = sqrt(sum_theta |D_i D_j D_k|^2) / n^2."""
    from . import plan as _plan
    import scipy.fft
    grid = np.asarray(grid).astype(np.complex128)
    n = grid.shape[0]
    if trips is None:
        trips, _ = _plan.plan_triplets(n, edges)
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    W = effective_weights(n, w, wmode)
    masks = _plan.ring_masks(n, edges)
    X = W * grid
    Y = hermitian_part(W.astype(np.complex128))
    D = np.stack([scipy.fft.fft2(np.where(m, X, 0), workers=-1) for m in masks])
    I = ring_fields(Y, masks)
    npix = float(n * n)
    pairs, pidx = _pairs_of(trips)
    pi = np.array([p[0] for p in pairs], dtype=np.int64)
    pj = np.array([p[1] for p in pairs], dtype=np.int64)
    Df = D.reshape(len(masks), -1)
    acc = np.zeros((len(pairs), len(masks)), np.complex128)
    acc2 = np.zeros((len(pairs), len(masks)), np.float64)
    for s0 in range(0, Df.shape[1], chunk):
        Fc = Df[:, s0:s0 + chunk]
        P = Fc[pi] * Fc[pj]
        acc += P @ Fc.T
        acc2 += (np.abs(P) ** 2) @ (np.abs(Fc) ** 2).T
    S = np.array([acc[pidx[(i, j)], k] for i, j, k in trips]) / npix
    rhoS = np.sqrt(np.array([acc2[pidx[(i, j)], k] for i, j, k in trips])) / npix
    N = triple_sums(I, trips, chunk)
    rhoN = np.sqrt(np.maximum(triple_sums(I, trips, chunk, power=2), 0.0) / n ** 2)
    wmin = min_weight(Y.real, masks)
    with np.errstate(divide="ignore", invalid="ignore"):
        B = S / (norm * N)
    B = np.where(N < 0.5 * wmin ** 3, np.nan + 1j * np.nan, B)
    return dict(B=B, S=S, N=N, trips=trips, wmin=wmin, rhoS=rhoS, rhoN=rhoN)


def estimate_subset(grid, w, edges, norm, trips, wmode=UNIT):
    """Eq. (12) and the error scales for a subset of triplets, computing only the ring
    fields those triplets use (for full-size grids where every field would not fit the
    time budget).  Same definitions and return keys as estimate(..., with_scales=True)."""
    from . import plan as _plan
    grid = np.asarray(grid).astype(np.complex128)
    n = grid.shape[0]
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    W = effective_weights(n, w, wmode)
    rc = _plan.ring_of_cell(n, edges)
    X = hermitian_part(W * grid)
    Y = hermitian_part(W.astype(np.complex128))
    import scipy.fft
    need = sorted(set(int(b) for b in trips.ravel()))
    D = {m: scipy.fft.fft2(np.where(rc == m, X, 0), workers=-1).real for m in need}
    I = {m: scipy.fft.fft2(np.where(rc == m, Y, 0), workers=-1).real for m in need}
    out = {k: np.zeros(len(trips)) for k in ("S", "N", "rhoS", "rhoN")}
    npix = float(n * n)
    for q, (i, j, k) in enumerate(trips):
        d = D[i] * D[j] * D[k]
        e = I[i] * I[j] * I[k]
        out["S"][q] = d.sum() / npix
        out["N"][q] = e.sum() / npix
        out["rhoS"][q] = np.sqrt((d * d).sum()) / npix
        out["rhoN"][q] = np.sqrt((e * e).sum()) / npix
    out["wmin"] = wmin = min_weight(Y.real, np.asarray([rc >= 0]))
    out["B"] = ratio(out["S"], out["N"], norm, wmin)
    out["trips"] = trips
    return out


def estimate_multifreq(grids, w, edges, norm, wmode=UNIT, trips=None, chunk=1 << 16):
    """Multi-frequency form of Eq. (12): the three fields of a triplet taken at channels
    a, b, c (Sec. 1 names multi-frequency observations as the estimator's next step):
    B = (1/A) sum_theta D_i(a) D_j(b) D_k(c) / sum_theta I_i(a) I_j(b) I_k(c).

    grids : complex [C][n][n], one gridded-visibility array per channel
    w     : [n][n] weights shared by every channel, or [C][n][n] (ignored for UNIT)
    trips : (T, 3) channel rings s = c nb + r, s1 <= s2 <= s3 (default: every such triple
            whose rings, sorted, form a plan triplet)
    Returns the keys of estimate(..., with_scales=True); w_min is the smallest over the
    channels (the empty-triplet rule of ``ratio``)."""
    from . import plan as _plan
    grids = np.asarray(grids).astype(np.complex128)
    C, n = grids.shape[0], grids.shape[1]
    nb = len(edges) - 1
    if trips is None:
        ring_trips, _ = _plan.plan_triplets(n, edges)
        ok = {tuple(int(x) for x in t) for t in ring_trips}
        trips = [(s1, s2, s3) for s1 in range(C * nb) for s2 in range(s1, C * nb) for s3 in range(s2, C * nb)
                 if tuple(sorted((s1 % nb, s2 % nb, s3 % nb))) in ok]
    trips = np.asarray(trips, dtype=np.int64).reshape(-1, 3)
    masks = _plan.ring_masks(n, edges)
    D, I, wmins = [], [], []
    for c in range(C):
        wc = None if wmode == UNIT else (w[c] if np.ndim(w) == 3 else w)
        W = effective_weights(n, wc, wmode)
        X = hermitian_part(W * grids[c])
        Y = hermitian_part(W.astype(np.complex128))
        D.append(ring_fields(X, masks))
        I.append(ring_fields(Y, masks))
        wmins.append(min_weight(Y.real, masks))
    D = np.concatenate(D)           # channel ring s = c nb + r
    I = np.concatenate(I)
    S = triple_sums(D, trips, chunk)
    N = triple_sums(I, trips, chunk)
    wmin = min(wmins)
    return dict(B=ratio(S, N, norm, wmin), S=S, N=N, trips=trips, wmin=wmin,
                rhoS=np.sqrt(np.maximum(triple_sums(D, trips, chunk, power=2), 0.0) / n ** 2),
                rhoN=np.sqrt(np.maximum(triple_sums(I, trips, chunk, power=2), 0.0) / n ** 2))


def relative_error(B, ref, norm):
    """Noise-scale-normalised error e_t = |B - B*| / max(|B*|, rho_t).

    rho_t = rhoS / (A |N*|) is the FP64 random-error scale of B*_t: per-triplet
    relative error is unbounded where the signed triangle sum cancels, so the
    gate compares against the larger of the value and the scale of its terms.
    ``ref`` is an ``estimate(..., with_scales=True)`` result, ``B`` the value
    under test and ``norm`` the A of Eq. (12).
    """
    Bs, N = ref["B"], ref["N"]
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = ref["rhoS"] / (norm * np.abs(N))
        return np.abs(np.asarray(B) - Bs) / np.maximum(np.abs(Bs), rho)


def count_error(N, ref):
    """|N - N*| / max(|N*|, rhoN): the same normalisation for the denominator."""
    Ns = ref["N"]
    return np.abs(np.asarray(N) - Ns) / np.maximum(np.abs(Ns), ref["rhoN"])
