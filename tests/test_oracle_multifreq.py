"""Pins of the multi-frequency estimator oracle (oracle.estimator.estimate_multifreq):
brute-force enumeration of closed triangles with the three vertices' values taken from
three channels; identical channels reduce to the single-frequency estimator; relabelling
the channels permutes the estimates."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from oracle import plan as oplan


def _channels(n, C, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((C, n, n)) + 1j * rng.standard_normal((C, n, n))


def _brute_cross(Xs, n, edges, trips):
    """sum over g1 in ring r1, g2 in ring r2, g3 = -(g1 + g2) in ring r3 (modulo n) of
    X_c1(g1) X_c2(g2) X_c3(g3), for channel rings (c r) given as s = c nb + r."""
    nb = len(edges) - 1
    rc = oplan.ring_of_cell(n, edges)
    cells = oplan.ring_cells(n, edges)
    out = np.zeros(len(trips), np.complex128)
    for t, s in enumerate(trips):
        (c1, r1), (c2, r2), (c3, r3) = [(int(x) // nb, int(x) % nb) for x in s]
        tot = 0j
        for g1 in cells[r1]:
            for g2 in cells[r2]:
                g3 = -(g1 + g2)
                g3w = ((g3 + n // 2) % n) - n // 2
                if rc[g3w[1] % n, g3w[0] % n] != r3:
                    continue
                tot += Xs[c1][g1[1] % n, g1[0] % n] * Xs[c2][g2[1] % n, g2[0] % n] * Xs[c3][g3w[1] % n, g3w[0] % n]
        out[t] = tot
    return out


@pytest.mark.parametrize("wmode", [oest.UNIT, oest.GIVEN])
def test_multifreq_equals_brute_force(wmode):
    n, C = 16, 2
    e = [1.0, 2.0, 3.1, 4.2, 5.3]
    V = _channels(n, C, 5)
    rng = np.random.default_rng(6)
    w = np.stack([synth.symmetrize(rng.uniform(0.2, 2.0, (n, n))) for _ in range(C)]) if wmode else None
    ref = oest.estimate_multifreq(V, w, e, 1.0, wmode=wmode)
    Xs, Ys = [], []
    for c in range(C):
        W = oest.effective_weights(n, None if w is None else w[c], wmode)
        Xs.append(oest.hermitian_part(W * V[c]))
        Ys.append(oest.hermitian_part(W.astype(np.complex128)))
    S = _brute_cross(Xs, n, e, ref["trips"])
    N = _brute_cross(Ys, n, e, ref["trips"])
    assert np.allclose(ref["S"], S.real, rtol=1e-10, atol=1e-10 * np.abs(S).max())
    assert np.allclose(ref["N"], N.real, rtol=1e-10, atol=1e-10 * np.abs(N).max())
    # every channel combination of every ring triplet is there, once
    rings, _ = oplan.plan_triplets(n, e)
    assert len(ref["trips"]) > C * len(rings)
    assert len({tuple(t) for t in ref["trips"]}) == len(ref["trips"])


def test_identical_channels_reduce_to_the_single_frequency_estimate():
    n, C = 64, 3
    e = oplan.log_edges(2.0, 20.0, 6)
    V = _channels(n, 1, 8)[0]
    rng = np.random.default_rng(9)
    w = synth.symmetrize(rng.integers(0, 4, (n, n)).astype(np.float64))
    one = oest.estimate(V, w, e, 1.0, wmode=oest.INV_COUNT, with_scales=True)
    mf = oest.estimate_multifreq(np.stack([V] * C), w, e, 1.0, wmode=oest.INV_COUNT)
    nb = len(e) - 1
    idx = {tuple(int(x) for x in t): q for q, t in enumerate(one["trips"])}
    for q, s in enumerate(mf["trips"]):
        t = idx[tuple(sorted(int(x) % nb for x in s))]
        assert np.isclose(mf["S"][q], one["S"][t], rtol=1e-11, atol=1e-11 * one["rhoS"][t])
        assert np.isclose(mf["N"][q], one["N"][t], rtol=1e-11, atol=1e-11 * one["rhoN"][t])
        assert (np.isnan(mf["B"][q]) and np.isnan(one["B"][t])) or np.isclose(mf["B"][q], one["B"][t],
                                                                                   rtol=1e-9, atol=1e-12)


def test_relabelling_channels_permutes_the_estimates():
    n, C = 32, 3
    e = oplan.log_edges(2.0, 10.0, 4)
    V = _channels(n, C, 12)
    ref = oest.estimate_multifreq(V, None, e, 1.0)
    perm = [2, 0, 1]                    # new channel c holds old channel perm[c]
    sw = oest.estimate_multifreq(V[perm], None, e, 1.0)
    nb = len(e) - 1
    inv = {old: new for new, old in enumerate(perm)}
    pos = {tuple(int(x) for x in t): q for q, t in enumerate(sw["trips"])}
    for q, s in enumerate(ref["trips"]):
        mapped = tuple(sorted(inv[int(x) // nb] * nb + int(x) % nb for x in s))
        assert np.isclose(sw["S"][pos[mapped]], ref["S"][q], rtol=1e-11, atol=1e-12 * np.abs(ref["rhoS"]).max())
