"""Pins of the single-layer oracle (Sections 2.1-2.2: first-kind equation,
sixth-order corrected trapezoid rule for the logarithmic singularity) against
facts of the mathematics:

* the correction weights: the two-point rule has a closed form; the leading
  error term of the punctured rule on which they are built equals the exact
  punctured sum of log|2 sin(t/2)| (prod_j 2 sin(pi j / N) = N); the six-point
  rule integrates log|2 sin((t - t0)/2)| cos t (exact value -pi cos t0) with
  an error that falls at least 2^6-fold per halving of h;
* the single layer of a constant density on a circle has the closed form
  (R/4)(1 - 2 log R) c, reached by the assembled matrix;
* the whole discretisation: boundary data from Stokeslets and rotlets outside
  the fluid (Section 4.2), solved with the first-kind matrix by LU and
  evaluated in the fluid by the plain trapezoid rule, converges to the exact
  velocity as the nodes double.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import slp
from stokes_inputs import (Geometry, build_geometry, place_pores, stokeslet_rotlet_field,
                           stokeslet_rotlet_rhs)


def test_two_point_weights_closed_form():
    g = slp.kr_log_weights(2)
    l2 = math.log(2.0)
    assert np.allclose(g, [0.5 + math.log(2 * math.pi) / (2 * l2), -math.log(2 * math.pi) / (2 * l2)],
                       rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [8, 33, 128])
def test_punctured_rule_leading_term(n):
    """int_0^{2pi} log|2 sin(t/2)| dt = 0, and h sum_{j=1}^{N-1} log|2 sin(pi j/N)|
    = h log N: the punctured rule's error is h log(h / 2 pi) for phi = 1."""
    h = 2 * math.pi / n
    t = h * np.arange(1, n)
    punct = h * np.log(np.abs(2 * np.sin(t / 2))).sum()
    assert abs((0.0 - punct) - h * math.log(h / (2 * math.pi))) < 1e-13


def test_weights_satisfy_their_moment_conditions():
    g = slp.kr_log_weights(6)
    k = np.arange(1, 7)
    assert abs(2 * g.sum() - 1.0) < 1e-12
    assert abs(2 * (g * k ** 2).sum()) < 1e-10
    assert abs(2 * (g * k ** 4).sum()) < 1e-8
    # zeta'(-2p) from the functional equation against mpmath's own derivative
    import mpmath
    for p in (1, 2, 3):
        assert abs(slp.zeta_prime_neg_even(p) - float(mpmath.zeta(-2 * p, derivative=1))) < 1e-16


def test_six_point_rule_order():
    g6 = slp.kr_log_weights(6)
    errs = []
    for n in (64, 128, 256):
        h = 2 * math.pi / n
        t = h * np.arange(n)
        i = 5
        with np.errstate(divide="ignore"):
            f = np.log(np.abs(2 * np.sin((t - t[i]) / 2))) * np.cos(t)
        errs.append(abs(slp.corrected_trapezoid(f, i, h, g6) + math.pi * math.cos(t[i])))
    assert errs[0] / errs[1] > 64 and errs[1] / errs[2] > 64
    assert errs[2] < 1e-10
    # the plain punctured rule is only first order
    h = 2 * math.pi / 256
    t = h * np.arange(256)
    with np.errstate(divide="ignore"):
        f = np.log(np.abs(2 * np.sin((t - t[5]) / 2))) * np.cos(t)
    plain = h * np.delete(f, 5).sum()
    assert abs(plain + math.pi * math.cos(t[5])) > 1e-3


def one_circle(n, r=0.37, cx=0.3, cy=-0.2):
    th = 2 * math.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    return Geometry(x=cx + r * c, y=cy + r * s, nx=-c, ny=-s, tx=-s, ty=c,
                    w=np.full(n, 2 * math.pi * r / n), kappa=np.full(n, 1 / r),
                    cx=np.zeros(0), cy=np.zeros(0), radius=np.zeros(0),
                    curve_off=np.array([0, n]), length=1.0, n_int=0, n_ext=n)


def test_constant_density_on_circle():
    r = 0.37
    exact = r / 4 * (1 - 2 * math.log(r))
    errs = []
    for n in (64, 128, 256):
        g = one_circle(n, r)
        a = slp.assemble(g)
        c = np.array([0.6, -1.1])
        u = np.concatenate([np.full(n, c[0]), np.full(n, c[1])])
        v = a @ u
        errs.append(max(np.abs(v[:n] - exact * c[0]).max(), np.abs(v[n:] - exact * c[1]).max()))
    assert errs[-1] < 1e-11
    assert errs[0] / errs[1] > 64 and errs[1] / errs[2] > 64     # sixth order or better


def test_exact_stokeslet_solution_converges():
    """Section 4.2 boundary data; first-kind solve by LU (the null vector of
    the single layer on the wall, the normal density, produces no velocity in
    the fluid); velocity at points farther than max(5h, sqrt(h)) from the
    boundary."""
    cx, cy, rr = place_pores(np.random.default_rng(1), 6, 4.0, 0.05, 0.1, 0.05, 0.1)
    errs = []
    for nint, next_ in [(32, 256), (64, 512), (128, 1024)]:
        g = build_geometry(4.0, next_, cx, cy, rr, nint)
        f, data = stokeslet_rotlet_rhs(g, 2)
        nn = g.n_nodes
        a = slp.assemble(g)
        sig = sla.lu_solve(sla.lu_factor(a), f[:2 * nn])
        h = max(2 * math.pi * rr.min() / nint, g.w[-1])
        rng = np.random.default_rng(0)
        pts = []
        while len(pts) < 50:
            p = rng.uniform([0, 0], [4, 1])
            dd = min((np.hypot(p[0] - g.cx, p[1] - g.cy) - g.radius).min(),
                     p[1], 1 - p[1], p[0], 4 - p[0])
            if dd > max(5 * h, math.sqrt(h)):
                pts.append(p)
        pts = np.array(pts)
        ux, uy = slp.velocity(g, sig, pts[:, 0], pts[:, 1])
        ex, ey = stokeslet_rotlet_field(data, pts[:, 0], pts[:, 1])
        errs.append(np.max(np.hypot(ux - ex, uy - ey)) / np.max(np.hypot(ex, ey)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 16
    assert errs[2] < 1e-6


def test_rows_agree_with_assembled_matrix():
    """The row-by-row evaluation used for sampled checks at large sizes
    equals the assembled matrix (pores and wall, corrections included)."""
    cx, cy, rr = place_pores(np.random.default_rng(3), 5, 4.0, 0.05, 0.1, 0.05, 0.1)
    g = build_geometry(4.0, 256, cx, cy, rr, 32)
    a = slp.assemble(g)
    rows = np.array([0, 5, 31, 32, 100, g.n_nodes - 1, g.n_nodes, g.n_nodes + 7, 2 * g.n_nodes - 1])
    assert np.array_equal(slp.rows_of_matrix(g, rows), a[rows])
