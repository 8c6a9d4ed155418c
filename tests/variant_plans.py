"""Plans that between them select every code variant of the contraction kernels: the
FP32 data kernel's triplet order ((D_j D_k) D_i or (D_i D_j) D_k, blocks of j), waves per
workgroup and code parts; the same for the FP64 weight kernel; and the precision form's
tiles per wave and loads in flight.  All are small enough for the oracle to evaluate every
triplet.  VARIANTS pins what each plan selects: (parts, jk, block, waves) for the FP32 and
FP64 kernels, (tiles per wave, depth) for the precision form.  The plans are built with
LEVELS = 1 (every triplet at the plan's own n), so that each variant runs at the size
pinned here, and the precision forms with ABS_ALL_MFMA (every contraction on the matrix
units); resolution levels and the per-level choice of kernel have tests of their own."""
import numpy as np

from oracle import plan as oplan

LEVELS = 1

_E5 = oplan.log_edges(8 * 46 / (2 * np.pi), 8 * 1320 / (2 * np.pi), 64)    # 8192^2 ring radii
_E3 = oplan.log_edges(4 * 46 / (2 * np.pi), 4 * 1320 / (2 * np.pi), 32)    # 4096^2 ring radii


def _log(n, lo, hi, nb):
    return oplan.log_edges(lo * n, hi * n, nb)


PLANS = {
    # the 8192^2 / 64-ring ring geometry scaled to 1024^2 (every radius / 8)
    "ensemble_1024": (1024, _E5 / 8),
    "dense_256x64": (256, _log(256, 0.02, 0.33, 64)),
    "ij_256x40": (256, _log(256, 0.05, 0.30, 40)),
    # the 4096^2 / 32-ring geometry scaled to 1024^2
    "c3_1024": (1024, _E3 / 4),
    "w0_256x16": (256, _log(256, 0.05, 0.30, 16)),
    "w4_512x24": (512, _log(512, 0.02, 0.33, 24)),
    "w4w_256x12": (256, _log(256, 0.02, 0.33, 12)),
    "jk8_256x16": (256, _log(256, 0.02, 0.33, 16)),
    # rings of similar size (narrow radius range): orders in blocks of 4 or 8 j
    "b4_256x12": (256, _log(256, 0.12, 0.25, 12)),
    "b8_256x11": (256, _log(256, 0.08, 0.20, 11)),
    "b4w_256x17": (256, _log(256, 0.12, 0.20, 17)),
}

VARIANTS = {
    "ensemble_1024": dict(contract=(2, 0, 16, 8), weight=(3, 0, 8, 8), mfma=(12, 1)),
    "dense_256x64": dict(contract=(2, 0, 16, 8), weight=(3, 0, 8, 8), mfma=(12, 1)),
    "ij_256x40": dict(contract=(1, 0, 0, 8), weight=(2, 0, 8, 8), mfma=(12, 1)),
    "c3_1024": dict(contract=(1, 1, 0, 8), weight=(1, 0, 16, 8), mfma=(12, 4)),
    "w0_256x16": dict(contract=(1, 1, 0, 4), weight=(1, 0, 0, 8), mfma=(2, 1)),
    "w4_512x24": dict(contract=(1, 1, 0, 8), weight=(1, 1, 0, 8), mfma=(2, 1)),
    "w4w_256x12": dict(contract=(1, 1, 0, 4), weight=(1, 1, 0, 4), mfma=(2, 1)),
    "jk8_256x16": dict(contract=(1, 1, 0, 4), weight=(1, 1, 0, 8), mfma=(2, 1)),
    "b4_256x12": dict(contract=(1, 0, 4, 4), weight=(1, 0, 4, 8), mfma=(2, 1)),
    "b8_256x11": dict(contract=(1, 0, 8, 4), weight=(1, 0, 0, 4), mfma=(2, 1)),
    "b4w_256x17": dict(contract=(1, 0, 4, 8), weight=(1, 0, 0, 8), mfma=(2, 1)),
}

# precision forms run on the plans whose tiling variant they cover
PRECISION_CASES = [("ensemble_1024", "bf16x3"), ("ensemble_1024", "fp16x3"), ("dense_256x64", "fp16x3"),
                   ("c3_1024", "bf16x3"), ("c3_1024", "fp16x3"), ("w4_512x24", "bf16x3"),
                   ("w4_512x24", "fp16x3")]
