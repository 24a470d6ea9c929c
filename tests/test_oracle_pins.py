"""Pins of the CPU oracle against facts fixed by the mathematics and the paper.

Each test states what would fail if the oracle had a plausible mistake:
a dropped or mis-signed term, a wrong index, a transposed operand.
"""
import math

import numpy as np
import pytest

from oracle import dlp, solve
from stokes_inputs import (Geometry, build_geometry, make_geometry, place_pores,
                           poiseuille_rhs, random_vector, shear_rhs,
                           stokeslet_rotlet_field, stokeslet_rotlet_rhs)


def single_circle(n, r=0.3, cx=0.2, cy=-0.1):
    """A geometry made of one pore and no wall."""
    th = 2 * math.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    return Geometry(x=cx + r * c, y=cy + r * s, nx=-c, ny=-s, tx=-s, ty=c,
                    w=np.full(n, 2 * math.pi * r / n), kappa=np.full(n, 1 / r),
                    cx=np.array([cx]), cy=np.array([cy]), radius=np.array([r]),
                    curve_off=np.array([0, n, n]), length=1.0, n_int=n, n_ext=0)


@pytest.fixture(scope="module")
def tiny():
    g = make_geometry("tiny", 1)
    a = dlp.assemble(g)
    return g, a


# ---------------------------------------------------------------- geometry --

def test_geometry_wall_extents_and_closure():
    g = make_geometry("tiny", 2)
    ws = g.wall_slice
    assert abs(g.x[ws].min()) < 1e-12 and abs(g.x[ws].max() - 4.0) < 1e-12
    assert abs(g.y[ws].min()) < 1e-12 and abs(g.y[ws].max() - 1.0) < 1e-12
    # equispaced arclength: every chord equals the weight to O(h^3)
    xw, yw = g.x[ws], g.y[ws]
    ch = np.hypot(np.diff(np.r_[xw, xw[0]]), np.diff(np.r_[yw, yw[0]]))
    assert np.allclose(ch, g.w[ws], rtol=2e-3)
    # total turning of a simple closed curve, and closed normals
    assert abs((g.w[ws] * g.kappa[ws]).sum() + 2 * math.pi) < 1e-10
    for k in range(g.n_pores + 1):
        sl = slice(g.curve_off[k], g.curve_off[k + 1])
        assert abs((g.w[sl] * g.nx[sl]).sum()) < 1e-12
        assert abs((g.w[sl] * g.ny[sl]).sum()) < 1e-12
    # unit normals orthogonal to unit tangents; wall normal points out of
    # Omega_0 (so n_y < 0 on the bottom side)
    assert np.allclose(g.nx ** 2 + g.ny ** 2, 1.0)
    assert np.allclose(g.nx * g.tx + g.ny * g.ty, 0.0)
    assert g.ny[ws][0] < -0.999


def test_pores_disjoint_and_inside():
    g = make_geometry("pipe200", 101)
    d = np.hypot(g.cx[:, None] - g.cx[None, :], g.cy[:, None] - g.cy[None, :])
    gap = d - g.radius[:, None] - g.radius[None, :]
    np.fill_diagonal(gap, np.inf)
    assert gap.min() >= 0.005
    assert ((g.cy - g.radius) >= 0.05 - 1e-12).all()
    assert ((g.cy + g.radius) <= 0.95 + 1e-12).all()


# ------------------------------------------------------------- operator ----

@pytest.mark.parametrize("n", [2, 3, 7, 64, 129])
def test_P1_circle_identity(n):
    """On one circle with n toward the centre, w_j D_ij = (1/N) rhat rhat^T and
    the diagonal limit equals (1/N) t t^T; the N chord directions from a node
    are equispaced over a half turn, so the row sums are exactly I/2."""
    g = single_circle(n)
    for comp in range(2):
        u = np.zeros(2 * n + 3)
        u[comp * n:(comp + 1) * n] = 1.0
        v = dlp.dlp_only_rows(g, u, np.arange(2 * n))
        expect = np.zeros(2 * n)
        expect[comp * n:(comp + 1) * n] = 0.5
        assert np.abs(v - expect).max() < 1e-14


def test_P2_constant_density_jump(tiny):
    """Constant density c on every curve: the principal-value double layer is
    -c/2 at every node (own curve +-c/2, the wall's field inside Omega_0 is -c,
    pores contribute nothing outside themselves)."""
    g, _ = tiny
    nn = g.n_nodes
    u = np.zeros(g.n_unknowns)
    u[:nn], u[nn:2 * nn] = 0.7, -1.3
    v = dlp.dlp_only_rows(g, u, np.arange(2 * nn))
    assert np.abs(v[:nn] + 0.35).max() < 1e-12
    assert np.abs(v[nn:] - 0.65).max() < 1e-12


def test_P2_full_operator_on_constant(tiny):
    """Same identity through the assembled matrix: (-1/2 I + D) c = -c, with
    the wall's rank-one term vanishing because sum_j w_j n_j = 0."""
    g, a = tiny
    nn = g.n_nodes
    u = np.zeros(g.n_unknowns)
    u[:nn] = 0.4
    y = a @ u
    assert np.abs(y[:nn] + 0.4).max() < 1e-12
    assert np.abs(y[nn:2 * nn]).max() < 1e-12


def test_P4_completion_invertible_and_second_kind():
    """The completed operator is invertible and its smallest singular value
    stays put as the mesh is refined (second-kind equation, Section 2.1)."""
    cx, cy, rr = place_pores(np.random.default_rng(1), 10, 4.0, 0.05, 0.1, 0.05, 0.1)
    smin = []
    for nint, next_ in [(16, 128), (32, 256), (64, 512)]:
        g = build_geometry(4.0, next_, cx, cy, rr, nint)
        s = np.linalg.svd(dlp.assemble(g), compute_uv=False)
        smin.append(s[-1])
        assert s[0] / s[-1] < 5e3
    assert max(smin) / min(smin) < 2.0
    assert min(smin) > 1e-3


def test_P4_dropping_completion_makes_singular(tiny):
    """Without the pore completion columns the double layer has a null space
    (rank three per pore, Section 2.1) - so the completion is what makes the
    operator invertible."""
    g, a = tiny
    nn = g.n_nodes
    core = a[:2 * nn, :2 * nn]
    s = np.linalg.svd(core, compute_uv=False)
    assert s[-3 * g.n_pores] / s[0] < 1e-10
    assert s[-3 * g.n_pores - 1] / s[0] > 1e-5


def test_P5_exact_stokeslet_rotlet_solution_converges():
    """Boundary data from Stokeslets/rotlets (Section 4.2): the reconstructed
    velocity at interior points at distance >= max(5h, sqrt(h)) from the
    boundary converges geometrically to the exact field."""
    cx, cy, rr = place_pores(np.random.default_rng(1), 10, 4.0, 0.05, 0.1, 0.05, 0.1)
    errs = []
    for nint, next_ in [(16, 128), (32, 256), (64, 512)]:
        g = build_geometry(4.0, next_, cx, cy, rr, nint)
        a = dlp.assemble(g)
        f, data = stokeslet_rotlet_rhs(g, 1)
        sig = solve.lu_solve(a, f)
        h = max(2 * math.pi * rr.min() / nint, g.w[-1])
        dmin = max(5 * h, math.sqrt(h))
        rng = np.random.default_rng(0)
        pts = []
        while len(pts) < 60:
            p = rng.uniform([0, 0], [4, 1])
            dd = min((np.hypot(p[0] - g.cx, p[1] - g.cy) - g.radius).min(),
                     p[1], 1 - p[1], p[0], 4 - p[0])
            if dd > dmin:
                pts.append(p)
        pts = np.array(pts)
        ux, uy = dlp.velocity(g, sig, pts[:, 0], pts[:, 1])
        ex, ey = stokeslet_rotlet_field(data, pts[:, 0], pts[:, 1])
        errs.append(np.max(np.hypot(ux - ex, uy - ey)) / np.max(np.hypot(ex, ey)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[0] < 1e-2
    assert errs[2] < 1e-12


def test_P6_shear_flow_zero_pore_density(tiny):
    """Shear boundary data: the wall's density alone reproduces the linear
    field inside Omega_0, so the density on every pore and the completion
    unknowns vanish (Section 4.1)."""
    g, a = tiny
    nn = g.n_nodes
    sig = solve.lu_solve(a, shear_rhs(g))
    ws = g.wall_slice
    pore = np.r_[sig[:ws.start], sig[nn:nn + ws.start], sig[2 * nn:]]
    assert np.abs(pore).max() < 1e-10 * np.abs(sig).max()
    # and the wall density is not trivially zero
    assert np.abs(sig[ws]).max() > 1e-2


def test_P3_flux_functional_vanishes(tiny):
    """The wall's rank-one term is paired with the flux functional: projecting
    the wall rows on n gives beta = sum_wall w n.sigma = sum_wall w n.f, which
    is zero for divergence-free boundary data."""
    g, a = tiny
    nn = g.n_nodes
    ws = g.wall_slice
    for f in (poiseuille_rhs(g), stokeslet_rotlet_rhs(g, 3)[0]):
        sig = solve.lu_solve(a, f)
        beta = (g.w[ws] * (g.nx[ws] * sig[ws] + g.ny[ws] * sig[nn + ws.start:nn + ws.stop])).sum()
        assert abs(beta) < 1e-10


def test_P7_lu_residual(tiny):
    g, a = tiny
    f, _ = stokeslet_rotlet_rhs(g, 1)
    sig = solve.lu_solve(a, f)
    assert np.linalg.norm(f - a @ sig) / np.linalg.norm(f) < 1e-13


def test_rows_and_apply_agree(tiny):
    g, a = tiny
    u = random_vector(g.n_unknowns, 9)
    rows = np.array([0, 5, g.n_nodes + 3, 2 * g.n_nodes, 2 * g.n_nodes + 2, g.n_unknowns - 1])
    assert np.allclose(dlp.apply_rows(g, u, rows), (a @ u)[rows], rtol=0, atol=1e-12)
    assert np.allclose(dlp.apply(g, u, chunk=333), a @ u, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- solvers --

def test_P9_fgmres_diagonal_converges_in_k():
    d = np.arange(1.0, 13.0)
    f = random_vector(12, 4)
    r = solve.fgmres(lambda v: d * v, f, tol=1e-13)
    assert r.iters == 12 and r.converged
    assert np.allclose(r.x, f / d, rtol=1e-12)


def test_P9_fgmres_exact_start_no_iterations(tiny):
    g, a = tiny
    f, _ = stokeslet_rotlet_rhs(g, 1)
    sig = solve.lu_solve(a, f)
    r = solve.fgmres(lambda v: a @ v, f, x0=sig, tol=1e-10)
    assert r.iters == 0 and r.converged


def test_P9_fgmres_matches_lu(tiny):
    g, a = tiny
    f, _ = stokeslet_rotlet_rhs(g, 1)
    sig = solve.lu_solve(a, f)
    for pc in (None, solve.BlockDiagonal(g, a)):
        r = solve.fgmres(lambda v: a @ v, f, precond=pc, tol=1e-12)
        assert r.converged and r.rel_res_true < 1e-12
        assert np.linalg.norm(r.x - sig) / np.linalg.norm(sig) < 1e-9


def test_P9_fgmres_restart_and_cap(tiny):
    g, a = tiny
    f, _ = stokeslet_rotlet_rhs(g, 1)
    r = solve.fgmres(lambda v: a @ v, f, tol=1e-12, max_iter=5)
    assert not r.converged and r.iters == 5
    r2 = solve.fgmres(lambda v: a @ v, f, tol=1e-10, restart=20, max_iter=2000)
    assert r2.converged


def test_P10_block_diagonal_exact_on_single_pore():
    """One pore and no wall: the block-diagonal preconditioner is the exact
    inverse, so FGMRES converges in one iteration."""
    g = single_circle(32)
    a = dlp.assemble(g)
    f = random_vector(g.n_unknowns, 2)
    r = solve.fgmres(lambda v: a @ v, f, precond=solve.BlockDiagonal(g, a), tol=1e-12)
    assert r.iters == 1


def test_block_diagonal_reduces_iterations(tiny):
    """Qualitative pin from the paper's tables (Section 4): the block-diagonal
    preconditioner needs fewer iterations than none."""
    g, a = tiny
    f = poiseuille_rhs(g)
    r0 = solve.fgmres(lambda v: a @ v, f, tol=1e-10)
    r1 = solve.fgmres(lambda v: a @ v, f, precond=solve.BlockDiagonal(g, a), tol=1e-10)
    assert r1.iters < r0.iters
