"""Pins of the oracle's completion (the removal of the double layer's rank-3
null space per pore, Section 2.1) against facts other than its own formulas.

The completion adds, per pore k, a Stokeslet column S(x - c_k), a rotlet
column r_k R(x - c_k) and three constraint rows (lambda_k = mean density,
mu_k = mean tangential moment over r_k).  Any non-zero scaling gives an
invertible operator and the same velocity in the fluid, so the exact-solution
pin cannot see these scalings; they are fixed here by:

* closed forms of the constraint functionals on the densities they measure
  (a constant density, a rigid rotation);
* the physics of the columns: the Stokeslet column is the velocity of a unit
  point force and the rotlet column that of a point torque -r_k (unit
  viscosity), measured by integrating the fluid stress of the oracle's own
  field around the pore centre, with the stress built from finite differences
  of that field (so a wrong 1/(4 pi), a swapped component or a sign slip in
  r^perp changes the measured force or torque);
* the independent Stokeslet/rotlet formula of the boundary-data generator
  (written from the paper's printed exact solution, Section 4.2, without the
  1/(4 pi)), which the exact-solution test shows to be a Stokes flow.
"""
import math

import numpy as np
import pytest

from oracle import dlp
from stokes_inputs import make_geometry, stokeslet_rotlet_field


@pytest.fixture(scope="module")
def tiny():
    return make_geometry("tiny", 1)


def pore_rows(g, k):
    nn = g.n_nodes
    return 2 * nn + 3 * k + np.arange(3)


def test_lambda_functional_reads_constant_density(tiny):
    """sigma = c on pore k only: the lambda rows of pore k read c exactly
    (sum of the trapezoid weights is the circumference 2 pi r_k), the mu row
    reads 0, and every other pore's rows read 0."""
    g = tiny
    nn = g.n_nodes
    c = np.array([0.7, -1.9])
    for k in (0, g.n_pores - 1):
        u = np.zeros(g.n_unknowns)
        sl = g.pore_slice(k)
        u[sl] = c[0]
        u[nn + sl.start:nn + sl.stop] = c[1]
        rows = np.arange(2 * nn, g.n_unknowns)
        v = dlp.apply_rows(g, u, rows).reshape(g.n_pores, 3)
        assert np.abs(v[k, :2] - c).max() < 1e-14
        assert abs(v[k, 2]) < 1e-14
        others = np.delete(v, k, axis=0)
        assert np.abs(others).max() == 0.0


def test_mu_functional_reads_rigid_rotation(tiny):
    """sigma = (x - c_k)^perp / r_k = (y - c_y, -(x - c_x)) / r_k on pore k:
    the mu row reads exactly 1 (a sign slip in the perp would read -1) and
    the lambda rows read 0."""
    g = tiny
    nn = g.n_nodes
    for k in (1, g.n_pores - 2):
        sl = g.pore_slice(k)
        u = np.zeros(g.n_unknowns)
        u[sl] = (g.y[sl] - g.cy[k]) / g.radius[k]
        u[nn + sl.start:nn + sl.stop] = -(g.x[sl] - g.cx[k]) / g.radius[k]
        v = dlp.apply_rows(g, u, pore_rows(g, k))
        assert abs(v[2] - 1.0) < 1e-13
        assert np.abs(v[:2]).max() < 1e-14


def test_constraint_rows_minus_identity_on_completion_unknowns(tiny):
    """The constraint rows hold -1 on their own completion unknown and
    nothing on any other completion unknown."""
    g = tiny
    nn = g.n_nodes
    a = dlp.rows_of_matrix(g, np.arange(2 * nn, g.n_unknowns))
    assert np.array_equal(a[:, 2 * nn:], -np.eye(3 * g.n_pores))


def test_columns_match_independent_stokeslet_rotlet(tiny):
    """Node rows of the completion columns against the boundary-data
    generator's Stokeslet/rotlet (the paper's exact-solution formula, no
    1/(4 pi)): Stokeslet column = field / (4 pi), rotlet column = field
    times r_k / (4 pi)."""
    g = tiny
    nn = g.n_nodes
    rows = np.arange(2 * nn)
    a = dlp.rows_of_matrix(g, rows)
    for k in range(g.n_pores):
        for comp in range(3):
            data = dict(cx=np.array([g.cx[k]]), cy=np.array([g.cy[k]]),
                        lam=np.zeros((1, 2)), mu=np.zeros(1))
            if comp < 2:
                data["lam"][0, comp] = 1.0
                scale = 1.0 / (4 * math.pi)
            else:
                data["mu"][0] = 1.0
                scale = g.radius[k] / (4 * math.pi)
            fx, fy = stokeslet_rotlet_field(data, g.x, g.y)
            col = a[:, 2 * nn + 3 * k + comp]
            ref = scale * np.concatenate([fx, fy])
            assert np.abs(col - ref).max() <= 1e-14 * np.abs(ref).max()


def _stress_integrals(field, c, radius=0.3, q=64, h=1e-4):
    """Force and torque (about c) exerted across a circle around c by the
    fluid outside it, for a unit-viscosity Stokes flow given only as a
    velocity field: strain rate and vorticity by central differences,
    pressure by integrating grad p = Laplacian u = (-d_y w, d_x w) along the
    circle (spectrally), traction (-p I + grad u + grad u^T) n."""
    th = 2 * math.pi * np.arange(q) / q
    nx, ny = np.cos(th), np.sin(th)
    px, py = c[0] + radius * nx, c[1] + radius * ny

    def grad(fun, x, y):
        fxp, fxm = fun(x + h, y), fun(x - h, y)
        fyp, fym = fun(x, y + h), fun(x, y - h)
        return ([(a - b) / (2 * h) for a, b in zip(fxp, fxm)],
                [(a - b) / (2 * h) for a, b in zip(fyp, fym)])

    def vort(x, y):
        gx, gy = grad(field, x, y)          # gx = d(ux, uy)/dx, gy = d(ux, uy)/dy
        return (gx[1] - gy[0],)

    (ux_x, uy_x), (ux_y, uy_y) = grad(field, px, py)
    (w_x,), (w_y,) = grad(vort, px, py)
    tx, ty = -ny, nx
    dp_dth = radius * (tx * (-w_y) + ty * w_x)
    spec = np.fft.fft(dp_dth)
    m = np.fft.fftfreq(q, d=1.0 / q)
    assert abs(spec[0]) / q < 1e-8                        # pressure is single valued
    phat = np.zeros_like(spec)
    nz = m != 0
    phat[nz] = spec[nz] / (1j * m[nz])
    p = np.fft.ifft(phat).real
    sxx, syy = -p + 2 * ux_x, -p + 2 * uy_y
    sxy = ux_y + uy_x
    trx = sxx * nx + sxy * ny
    try_ = sxy * nx + syy * ny
    ds = 2 * math.pi * radius / q
    force = np.array([trx.sum() * ds, try_.sum() * ds])
    torque = ((px - c[0]) * try_ - (py - c[1]) * trx).sum() * ds
    return force, torque


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_columns_are_unit_point_force_and_scaled_torque(tiny, comp):
    """The oracle's velocity from one completion unknown (sigma = 0) is the
    flow of a point force e_comp (Stokeslet column) or of a point torque
    -r_k (rotlet column; r^perp = (r_y, -r_x) turns clockwise): the stress
    across a circle balances it, force = -F and torque = -L."""
    g = tiny
    nn = g.n_nodes
    k = 3
    u = np.zeros(g.n_unknowns)
    u[2 * nn + 3 * k + comp] = 1.0

    def field(x, y):
        return dlp.velocity(g, u, np.ravel(x), np.ravel(y))

    force, torque = _stress_integrals(field, (g.cx[k], g.cy[k]))
    if comp < 2:
        expect_f = -np.eye(2)[comp]
        expect_t = 0.0
    else:
        expect_f = np.zeros(2)
        expect_t = g.radius[k]
    assert np.abs(force - expect_f).max() < 1e-6
    assert abs(torque - expect_t) < 1e-6 * max(1.0, g.radius[k])
