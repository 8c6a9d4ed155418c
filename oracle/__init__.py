"""FP64 CPU oracle for the FFT binned angular bispectrum estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
GPU library never calls into it and shares no code, tables or constants with it.

Everything here is a plain, slow, obviously-correct restatement of
Gill, Bharadwaj, Ali & Elahi (2024), "A visibility-based angular bispectrum
estimator for radio-interferometric data":

* ``plan``      -- annular rings and the list of ring triplets (Sec. 2, the ring
                   partition of the uv plane; Sec. 3, all ring triplets).
* ``estimator`` -- Eqs. (10) D, (11) I and (12) B-hat, computed with numpy FFTs in
                   FP64 and a chunked FP64 matrix product.
* ``brute``     -- the same sums by direct enumeration of closed grid triangles
                   (Sec. 2, the weighted-average-over-triangles reading of Eq. 12).
* ``gridding``  -- nearest-cell gridding, Eq. (9).
* ``theory``    -- the closed-form local-quadratic bispectrum, Eq. (14) and its
                   discretely-sampled average, plus the paper's constants.
* ``analysis``  -- the (ell1, mu, t) re-binning of the triplet estimates, ensemble mean
                   and sigma, and the deviation metrics of Secs. 3-4.
* ``simulate``  -- visibilities of a flat-sky field through the primary beam, Eq. (4)
                   with Eqs. (5)/(6), by direct summation.

Parity status per function is stated in each module header.
"""
from . import plan, estimator, brute, gridding, theory, analysis, simulate  # noqa: F401
