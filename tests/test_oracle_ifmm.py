"""Pins of the oracle IFMM (Section 3) against properties the paper states:
a tunable accuracy that makes it a direct solver as eps -> 0, exactness when
no pair of boxes is well separated, and its use as a GMRES preconditioner
that cuts the iteration count below the block-diagonal one."""
import numpy as np
import pytest

from oracle import dlp, ifmm, solve
from stokes_inputs import make_geometry, poiseuille_rhs, stokeslet_rotlet_rhs


@pytest.fixture(scope="module")
def tiny():
    g = make_geometry("tiny", 1)
    a = dlp.assemble(g)
    f, _ = stokeslet_rotlet_rhs(g, 1)
    return g, a, f, solve.lu_solve(a, f)


def test_chebyshev_interpolation_is_exact_on_polynomials():
    """S_n reproduces polynomials of degree < n exactly (Lagrange property)."""
    n = 7
    t = np.linspace(-1, 1, 31)
    s = ifmm.cheb_interp_1d(n, t)
    nodes = ifmm.cheb_points(n)
    for deg in range(n):
        assert np.allclose(s @ nodes ** deg, t ** deg, atol=1e-12)
    # the interpolant of a node is the node's indicator
    assert np.allclose(ifmm.cheb_interp_1d(n, nodes), np.eye(n), atol=1e-13)


def test_far_kernel_matches_operator_entries():
    """The 7-component far-field kernel times the anterpolation weights gives
    the operator's entries (double layer, Stokeslet, scaled rotlet)."""
    g = make_geometry("tiny", 1)
    nn = g.n_nodes
    i, j, k = 3, nn - 7, 2           # target node, source wall node, pore
    k7 = ifmm.far_kernel(np.array([g.x[i]]), np.array([g.y[i]]),
                         np.array([g.x[j], g.cx[k]]), np.array([g.y[j], g.cy[k]]))
    k7 = k7.reshape(2, 7, 2)
    rows = dlp.rows_of_matrix(g, [i, nn + i])
    for a in range(2):
        for l in range(2):
            dl = sum(k7[a, 2 * kk + l, 0] * g.w[j] * (g.nx[j], g.ny[j])[kk] for kk in range(2))
            assert np.isclose(dl, rows[a, l * nn + j], rtol=1e-12)
        for b in range(2):
            assert np.isclose(k7[a, 4 + b, 1], rows[a, 2 * nn + 3 * k + b], rtol=1e-12)
        assert np.isclose(k7[a, 6, 1] * g.radius[k], rows[a, 2 * nn + 3 * k + 2], rtol=1e-12)


def test_no_far_field_is_exact(tiny):
    """A tree too shallow to have a well-separated pair: the IFMM is plain
    block elimination, i.e. exact."""
    g, a, f, sig = tiny
    p = ifmm.IFMM(g, eps=1e-3, cheb_n=4, max_depth=1, dense=a)
    assert p.root_level == p.tree.depth
    x = p(f)
    assert np.linalg.norm(x - sig) / np.linalg.norm(sig) < 1e-10


@pytest.mark.parametrize("n,eps,bound", [(6, 1e-3, 5e-2), (10, 1e-6, 1e-4), (14, 1e-9, 1e-6)])
def test_error_follows_eps(tiny, n, eps, bound):
    """The approximate inverse's error is controlled by eps (with the
    Chebyshev order matched to eps, as the paper advises)."""
    g, a, f, sig = tiny
    p = ifmm.IFMM(g, eps=eps, cheb_n=n, dense=a)
    err = np.linalg.norm(p(f) - sig) / np.linalg.norm(sig)
    assert err < bound
    assert err > 1e-16


def test_order_independence_within_eps(tiny):
    """Morton and colour elimination orders give different factors but the
    same solution to O(eps)."""
    g, a, f, sig = tiny
    x1 = ifmm.IFMM(g, eps=1e-8, cheb_n=12, dense=a)(f)
    x2 = ifmm.IFMM(g, eps=1e-8, cheb_n=12, dense=a, order="color")(f)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(sig) < 1e-5


def test_preconditioner_beats_block_diagonal(tiny):
    """Qualitative pin from the paper's tables: fewer GMRES iterations with
    the IFMM than with the block-diagonal preconditioner."""
    g, a, _, _ = tiny
    f = poiseuille_rhs(g)
    r_bd = solve.fgmres(lambda v: a @ v, f, precond=solve.BlockDiagonal(g, a), tol=1e-10)
    r_if = solve.fgmres(lambda v: a @ v, f, precond=ifmm.IFMM(g, eps=1e-3, cheb_n=6, dense=a),
                        tol=1e-10)
    assert r_if.converged and r_bd.converged
    assert r_if.iters < r_bd.iters / 4
