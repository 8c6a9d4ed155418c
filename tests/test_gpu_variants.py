"""GPU parity of every contraction code variant on every triplet: each plan of
variant_plans (between them every triplet order, workgroup width and code-part split of the
FP32 and FP64 kernels, and the three precision-form variants) estimates MWA-shaped grids
with INV_COUNT weights, and B_t, N_t of all plan triplets are compared with the FP64 oracle
(e_t <= 1e-5 in FP32, <= 1e-4 in the precision forms; the same NaN positions)."""
import numpy as np
import pytest

import synth
from oracle import estimator as oest
from variant_plans import LEVELS, PLANS, PRECISION_CASES, VARIANTS

pytestmark = pytest.mark.gpu
TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-4}
_REF = {}


def _inputs(name):
    n, _ = PLANS[name]
    V, counts = synth.mwa_like(n, synth.seed_for(5, sorted(PLANS).index(name)), U0=n / 8)
    return V.astype(np.complex64), counts


def _reference(name, trips, norm):
    if name not in _REF:
        n, e = PLANS[name]
        V, counts = _inputs(name)
        _REF.clear()           # one plan's reference at a time
        _REF[name] = oest.estimate(V, counts, e, norm, wmode=oest.INV_COUNT, trips=trips, with_scales=True)
    return _REF[name]


def _run(name, prec):
    import torch
    import paper_2412_02246_amd as A
    n, e = PLANS[name]
    P = {"fp32": A.FP32, "bf16x3": A.BF16X3, "fp16x3": A.FP16X3}[prec]
    p = A.Plan(n, e, wmode=A.W_INV_COUNT, precision=P, levels=LEVELS, flags=A.ALL_MFMA if prec != "fp32" else 0)
    want = VARIANTS[name]
    if prec == "fp32":
        assert p.variants["contract"] == want["contract"]
    else:
        assert p.variants["mfma"] == want["mfma"]
    assert p.variants["weight"] == want["weight"]
    print("%s %s: %d triplets, variants %s, %d code parts" % (name, prec, p.ntrip, p.variants, p.jit_parts),
          flush=True)
    p.compile(workers=8)
    p.bind()
    V, counts = _inputs(name)
    B, N = p.estimate(torch.from_numpy(V).cuda(), torch.from_numpy(counts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    B, N = B[0].cpu().numpy(), N[0].cpu().numpy()
    ref = _reference(name, p.triplets, p.norm)
    empty = np.isnan(ref["B"])
    assert np.array_equal(np.isnan(B), empty), name
    e_t = oest.relative_error(B, ref, p.norm)[~empty]
    e_n = oest.count_error(N, ref)
    print("%s %s: max e_t %.3g median %.3g, max e_N %.3g over all %d triplets (%d empty)"
          % (name, prec, e_t.max(), np.median(e_t), e_n.max(), p.ntrip, int(empty.sum())), flush=True)
    assert np.all(np.isfinite(B[~empty]))
    assert e_t.max() <= TOL[prec], (name, prec, e_t.max(), int(np.argmax(e_t)))
    assert e_n.max() <= 1e-5, (name, prec, e_n.max())
    p.close()


# every plan in FP32, and the precision forms on the plans that cover their variants,
# grouped by plan so that each plan's oracle reference is computed once
CASES = sorted([(name, "fp32") for name in PLANS] + PRECISION_CASES)


@pytest.mark.parametrize("name,prec", CASES)
def test_variant_all_triplets(name, prec):
    _run(name, prec)
