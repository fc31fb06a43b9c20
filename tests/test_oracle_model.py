"""Pins of the oracle's velocity set, weights and Hermite basis.

Each test checks the oracle against something other than itself: the
paper's propagate listing (Sec. 4, Fig. 4), the Gaussian moments that define
a degree-9 quadrature, and numpy's own Hermite-polynomial routine.
"""

import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite_e as H

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def model():
    return oracle.model()


def gauss_moment(p):
    return 0.0 if p % 2 else float(math.prod(range(p - 1, 0, -2)))


def test_velocity_set_structure(model):
    cx, cy, w, r = model
    vecs = list(zip(cx.tolist(), cy.tolist()))
    assert len(vecs) == 37 and len(set(vecs)) == 37
    # populations travel at most three sites (Sec. 2): all hops within 3 in x and y
    assert max(abs(np.concatenate([cx, cy]))) == 3
    # opposite pairs and the rest population
    for l in range(37):
        assert (cx[36 - l], cy[36 - l]) == (-cx[l], -cy[l])
    assert (cx[18], cy[18]) == (0, 0)
    # label order: cx descending, then cy ascending
    assert vecs == sorted(vecs, key=lambda c: (-c[0], c[1]))
    # family counts of D2Q37
    fams = {}
    for a, b in vecs:
        key = tuple(sorted((abs(a), abs(b))))
        fams[key] = fams.get(key, 0) + 1
    assert fams == {(0, 0): 1, (0, 1): 4, (1, 1): 4, (0, 2): 4, (1, 2): 8,
                    (2, 2): 4, (0, 3): 4, (1, 3): 8}


def test_listing_offsets(model):
    """Labels 0 and 1 hop as the paper's propagate listing gathers them."""
    cx, cy, _, _ = model
    rows = [l.split() for l in open(os.path.join(GOLDEN, "propagate_listing_offsets.txt"))
            if l.strip() and not l.startswith("#")]
    for lab, dx, dy in rows:
        l = int(lab)
        # a gather from (x+dx, y+dy) means the population moved by (-dx, -dy)
        assert (cx[l], cy[l]) == (-int(dx), -int(dy))


def test_weights_positive_and_normalised(model):
    _, _, w, r = model
    assert np.all(w > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    assert 1.0 < r < 1.5


def test_quadrature_exact_to_degree_9(model):
    """sum w xi_x^p xi_y^q equals the 2-D standard Gaussian moment, p+q <= 9."""
    cx, cy, w, r = model
    xx, xy = r * cx.astype(float), r * cy.astype(float)
    for p in range(10):
        for q in range(10 - p):
            got = np.sum(w * xx ** p * xy ** q)
            want = gauss_moment(p) * gauss_moment(q)
            assert abs(got - want) <= 1e-13 * max(1.0, want), (p, q, got, want)


def test_quadrature_fails_at_degree_10(model):
    """Exactly degree 9: the x^10 moment is not the Gaussian 945."""
    cx, _, w, r = model
    got = np.sum(w * (r * cx.astype(float)) ** 10)
    assert abs(got - 945.0) > 1.0


def test_hermite_orthogonality(model):
    """sum w He_p He_q He_p' He_q' = p! q! delta, for total orders <= 4."""
    cx, cy, w, r = model
    xx, xy = r * cx.astype(float), r * cy.astype(float)
    pq = [(p, q) for p in range(5) for q in range(5 - p)]

    def he(n, x):
        c = np.zeros(n + 1)
        c[n] = 1
        return H.hermeval(x, c)

    for (p, q) in pq:
        for (a, b) in pq:
            got = np.sum(w * he(p, xx) * he(q, xy) * he(a, xx) * he(b, xy))
            want = math.factorial(p) * math.factorial(q) if (p, q) == (a, b) else 0.0
            assert abs(got - want) < 1e-12 * max(1.0, want), ((p, q), (a, b), got)
