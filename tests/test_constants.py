"""The GPU library's generated constants: fresh and consistent with the oracle.

The header is produced by a solver of its own (mpmath); the oracle solves the
same quadrature conditions independently in binary128.  The two must agree
to the last bit or so, and the header must match its generator.
"""

import os
import re
import sys

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_00186_amd", "csrc")


def header_values():
    text = open(os.path.join(CSRC, "d2q37_constants.h")).read()
    ex = [int(v) for v in re.search(r"EX\[Q\] = \{([^}]*)\}", text).group(1).split(",")]
    ey = [int(v) for v in re.search(r"EY\[Q\] = \{([^}]*)\}", text).group(1).split(",")]
    w = [float.fromhex(v.strip()) for v in
         re.search(r"W\[Q\] = \{([^}]*)\}", text, re.S).group(1).split(",") if v.strip()]
    r = float.fromhex(re.search(r"R = ([^;]*);", text).group(1))
    return np.array(ex), np.array(ey), np.array(w), r


def test_header_is_up_to_date():
    sys.path.insert(0, CSRC)
    try:
        import gen_constants
        assert gen_constants.check()
    finally:
        sys.path.pop(0)


def test_header_matches_independent_oracle_solve():
    ex, ey, w, r = header_values()
    cx, cy, wo, ro = oracle.model()
    assert np.array_equal(ex, cx) and np.array_equal(ey, cy)
    assert abs(r - ro) <= 2e-16 * r
    assert np.allclose(w, wo, rtol=4e-16, atol=0)
