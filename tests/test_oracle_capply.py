"""Pins of the oracle's plain C operator (oracle/cdlp.c), which the stored
reference solutions of the large workloads are computed with.

It must agree with the NumPy oracle's assembled matrix (itself pinned by the
closed forms of test_oracle_pins.py) and reproduce the same closed forms on
its own: the circle identity and the constant-density jump.
"""
import math

import numpy as np
import pytest

from oracle import capply, dlp
from stokes_inputs import Geometry, make_geometry


def single_circle(n, r=0.3, cx=0.2, cy=-0.1):
    th = 2 * math.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    return Geometry(x=cx + r * c, y=cy + r * s, nx=-c, ny=-s, tx=-s, ty=c,
                    w=np.full(n, 2 * math.pi * r / n), kappa=np.full(n, 1 / r),
                    cx=np.array([cx]), cy=np.array([cy]), radius=np.array([r]),
                    curve_off=np.array([0, n, n]), length=1.0, n_int=n, n_ext=0)


@pytest.fixture(scope="module")
def tiny():
    g = make_geometry("tiny", 1)
    return g, dlp.assemble(g)


@pytest.mark.parametrize("extended", [False, True])
def test_matches_assembled_oracle_matrix(tiny, extended):
    g, a = tiny
    for seed in range(3):
        u = np.random.default_rng(seed).standard_normal(g.n_unknowns)
        ref = a @ u
        y = capply.apply(g, u, extended=extended)
        assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max() * 8


@pytest.mark.parametrize("n", [3, 16, 64])
def test_circle_constant_density(n):
    """One circle, density c: the double layer gives +c/2 (circle identity),
    the jump -c/2, so the node rows vanish; the lambda rows read c."""
    g = single_circle(n)
    c = np.array([0.8, -0.3])
    u = np.zeros(g.n_unknowns)
    u[:n], u[n:2 * n] = c
    for ext in (False, True):
        y = capply.apply(g, u, extended=ext)
        assert np.abs(y[:2 * n]).max() < 1e-14
        assert np.abs(y[2 * n:2 * n + 2] - c).max() < 1e-14
        assert abs(y[2 * n + 2]) < 1e-14


def test_constant_density_on_pipe(tiny):
    """(-1/2 I + D) c = -c at every node of the pipe with pores (the wall's
    rank-one term vanishes because the wall normals integrate to zero)."""
    g, _ = tiny
    nn = g.n_nodes
    u = np.zeros(g.n_unknowns)
    u[:nn] = 0.4
    y = capply.apply(g, u, extended=True)
    assert np.abs(y[:nn] + 0.4).max() < 1e-12
    assert np.abs(y[nn:2 * nn]).max() < 1e-12


def test_extended_residual_resolves_cancellation(tiny):
    """The 80-bit evaluation and the double one agree to double rounding on
    the product, and the 80-bit residual of an exact product is far below
    it: A (u) - A (u) evaluated twice in 80-bit arithmetic is identical."""
    g, a = tiny
    u = 1e3 * np.random.default_rng(7).standard_normal(g.n_unknowns)
    y80 = capply.apply(g, u, extended=True)
    y64 = capply.apply(g, u)
    assert np.abs(y80 - y64).max() <= 1e-14 * np.abs(y80).max() * 8
    assert np.array_equal(y80, capply.apply(g, u, extended=True))
