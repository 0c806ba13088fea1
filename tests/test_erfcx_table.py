"""The erfcx Chebyshev table the FP64 real-space kernels use (kErfcxCheb in
kernels.hip) against erfcx in 40-digit arithmetic (mpmath): the double
Clenshaw sum of the table as the kernels evaluate it is within 1.2e-15
relative for x in [0, 8] (the range real space uses: erfc(8) ~ 1e-29) and
within 6e-15 up to 40.  CPU only."""
import os
import re

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2408_03273_amd", "csrc",
                   "kernels.hip")


def _table():
    text = open(SRC).read()
    body = re.search(r"kErfcxCheb\[23\]\s*=\s*\{([^}]*)\}", text).group(1)
    c = [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]
    assert len(c) == 23
    return c


def _clenshaw(c, x):
    t = (x - 3.0) / (x + 3.0)
    t2 = 2.0 * t
    b1 = b2 = 0.0
    for cn in reversed(c[1:]):
        b1, b2 = t2 * b1 + (cn - b2), b1  # (the kernels fuse this multiply-add)
    return t * b1 + (c[0] - b2)


def test_erfcx_table_accuracy():
    mp.mp.dps = 40
    c = _table()
    for lo, hi, n, tol in ((0.0, 8.0, 1601, 1.2e-15), (8.0, 40.0, 321, 6e-15)):
        worst = 0.0
        for x in np.linspace(lo, hi, n):
            ref = float(mp.erfc(mp.mpf(x)) * mp.exp(mp.mpf(x) ** 2))
            worst = max(worst, abs(_clenshaw(c, float(x)) / ref - 1.0))
        assert worst < tol, (lo, hi, worst)
