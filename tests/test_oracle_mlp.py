"""Pins of the warm-start oracle against what mathematics fixes independently
of its code: library routines for the normal CDF, nearest neighbours and the
FFT, central finite differences of the loss, the least-squares solution that
a linear network must reach, Adam's first step, exact recovery of
trigonometric polynomials, and the constraint rows of the completed system.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.stats import norm

from oracle import dlp
from oracle import mlp
from stokes_inputs import make_geometry

SMALL = dict(length=4.0, n_ext=512, n_pores=30, r_lo=0.03, r_hi=0.06, n_int=64,
             gap_pore=0.02, gap_wall=0.08)


@pytest.fixture(scope="module")
def geom30():
    return make_geometry(SMALL, 5)


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-13, atol=1e-15)
    assert mlp.gelu(0.0) == 0.0
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-8, atol=1e-9)


def _tiny_net(rng, widths):
    layers = [(rng.standard_normal((widths[l + 1], widths[l])) * 0.7,
               rng.standard_normal(widths[l + 1]) * 0.3) for l in range(len(widths) - 1)]
    return layers


def test_pack_unpack_column_major():
    rng = np.random.default_rng(0)
    widths = [3, 4, 2]
    layers = _tiny_net(rng, widths)
    flat = mlp.pack(layers)
    assert flat.shape[0] == 3 * 4 + 4 + 4 * 2 + 2
    # W_1 column-major: entry (i, j) at j * rows + i
    assert flat[1 * 4 + 2] == layers[0][0][2, 1]
    back = mlp.unpack(flat, widths)
    for (w, b), (w2, b2) in zip(layers, back):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)


def test_backward_matches_central_differences():
    """Every parameter's derivative by central differences (h = 1e-6) agrees
    with the hand-derived backward pass to 1e-6 relative."""
    rng = np.random.default_rng(1)
    widths = [5, 7, 6, 3]
    layers = _tiny_net(rng, widths)
    x = rng.standard_normal((9, 5))
    t = rng.standard_normal((9, 3))
    scaling = (rng.standard_normal(5) * 0.1, 1.0 + rng.random(5),
               rng.standard_normal(3), 0.5 + rng.random(3))
    loss, grads = mlp.mlp_loss_grad(layers, x, t, scaling)
    flat = mlp.pack(layers)
    gflat = mlp.pack(grads)
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(flat.shape[0]):
        p = flat.copy()
        p[i] += h
        lp, _ = mlp.mlp_loss_grad(mlp.unpack(p, widths), x, t, scaling)
        p[i] -= 2 * h
        lm, _ = mlp.mlp_loss_grad(mlp.unpack(p, widths), x, t, scaling)
        fd[i] = (lp - lm) / (2 * h)
    assert np.linalg.norm(fd - gflat) / np.linalg.norm(fd) < 1e-6
    # the loss is the mean squared standardised error of the forward pass
    y = mlp.mlp_forward(layers, x, scaling)
    ref = np.mean(((y - scaling[2]) / scaling[3] - (t - scaling[2]) / scaling[3]) ** 2)
    assert abs(loss - ref) < 1e-12 * max(1.0, ref)


def test_linear_network_trained_by_adam_reaches_least_squares():
    """A network with no hidden layer is linear regression: Adam must reach
    the least-squares solution that LAPACK computes."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((60, 4))
    wt = rng.standard_normal((2, 4))
    t = x @ wt.T + 0.3 + 0.05 * rng.standard_normal((60, 2))
    layers = [(np.zeros((2, 4)), np.zeros(2))]
    p = mlp.pack(layers)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4001):
        _, g = mlp.mlp_loss_grad(mlp.unpack(p, [4, 2]), x, t)
        p, m, v = mlp.adam(p, mlp.pack(g), m, v, step, lr=1e-2)
    w, b = mlp.unpack(p, [4, 2])[0]
    a = np.hstack([x, np.ones((60, 1))])
    sol, *_ = np.linalg.lstsq(a, t, rcond=None)
    np.testing.assert_allclose(w, sol[:4].T, atol=1e-5)
    np.testing.assert_allclose(b, sol[4], atol=1e-5)


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_fit_scaling_standardises():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((200, 6)) * [1, 2, 3, 0, 5, 6] + [0, 1, -1, 7, 2, 3]
    t = rng.standard_normal((200, 3)) * [0.1, 10, 1] + 4
    a, b, c, d = mlp.fit_scaling(x, t)
    xs = (x - a) * b
    np.testing.assert_allclose(xs[:, [0, 1, 2, 4, 5]].mean(axis=0), 0, atol=1e-12)
    np.testing.assert_allclose(xs[:, [0, 1, 2, 4, 5]].std(axis=0), 1, rtol=1e-12)
    assert b[3] == 1.0                      # constant column keeps scale 1
    ts = (t - c) / d
    np.testing.assert_allclose(ts.std(axis=0), 1, rtol=1e-12)


def test_features_nearest_neighbours_match_kdtree(geom30):
    g = geom30
    f = mlp.features(g)
    pts = np.stack([g.cx, g.cy], axis=1)
    _, idx = cKDTree(pts).query(pts, k=17)
    for k in range(g.n_pores):
        nb = idx[k, 1:]
        np.testing.assert_allclose(f[k, 1:49:3], g.cx[nb] - g.cx[k], rtol=0, atol=0)
        np.testing.assert_allclose(f[k, 2:49:3], g.cy[nb] - g.cy[k], rtol=0, atol=0)
        np.testing.assert_allclose(f[k, 3:49:3], g.radius[nb], rtol=0, atol=0)
    assert np.array_equal(f[:, 0], g.radius)
    # channel [0, 1]: the walls' distances add up to the height, the inflow
    # profile is 1 - 4 (y - 1/2)^2 with slope -8 (y - 1/2)
    np.testing.assert_allclose(f[:, 51] + f[:, 52], 1.0, rtol=1e-15)
    np.testing.assert_allclose(f[:, 49], 1 - 4 * (g.cy - 0.5) ** 2, rtol=1e-14)
    np.testing.assert_allclose(f[:, 50], -8 * (g.cy - 0.5), rtol=1e-14, atol=1e-15)
    assert np.all(f[:, 53:] == 0)


def test_features_pad_when_fewer_than_16_pores():
    g = make_geometry("tiny", 1)              # 10 pores: 9 neighbours each
    f = mlp.features(g)
    assert np.all(f[:, 1 + 3 * 9:49] == 0)
    assert np.all(f[:, 3:28:3] > 0)


def test_labels_recover_trigonometric_polynomial(geom30):
    """A density that is exactly a series of the kept modes is recovered
    exactly; the DFT agrees with numpy's FFT (nodes start at angle 0)."""
    g = geom30
    rng = np.random.default_rng(6)
    coef = rng.standard_normal((g.n_pores, 64))
    x0 = mlp.assemble_x0(g, coef, None)
    lab = mlp.labels(g, x0)
    np.testing.assert_allclose(lab, coef, atol=1e-12)
    nn = g.n_nodes
    for k in (0, 7):
        sl = slice(int(g.curve_off[k]), int(g.curve_off[k + 1]))
        s = x0[nn:2 * nn][sl]
        c = np.fft.rfft(s) / s.shape[0]
        assert abs(lab[k, 32] - c[0].real) < 1e-12
        np.testing.assert_allclose(lab[k, 33:48], 2 * c[1:16].real, atol=1e-12)
        np.testing.assert_allclose(lab[k, 48:63], -2 * c[1:16].imag, atol=1e-12)
        assert abs(lab[k, 63] - 2 * c[16].real) < 1e-12


def test_assemble_x0_satisfies_constraint_rows(geom30):
    """lambda and mu of the initial guess make the completion's constraint
    rows of the assembled system vanish; the wall density is copied."""
    g = geom30
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((g.n_pores, 64))
    ne = g.n_ext
    wall = rng.standard_normal(2 * ne)
    x0 = mlp.assemble_x0(g, coef, wall)
    nn = g.n_nodes
    rows = np.arange(2 * nn, g.n_unknowns)
    r = dlp.rows_of_matrix(g, rows) @ x0
    assert np.abs(r).max() < 1e-12 * np.abs(x0).max()
    ws = g.wall_slice
    assert np.array_equal(x0[:nn][ws], wall[:ne]) and np.array_equal(x0[nn:2 * nn][ws], wall[ne:])


def test_assemble_x0_series_values():
    """Closed form on one pore: a_1 = 1 (x) and b_2 = 1 (y) give
    sigma = (cos theta, sin 2 theta) at the nodes."""
    g = make_geometry("tiny", 1)
    coef = np.zeros((g.n_pores, 64))
    coef[:, 1] = 1.0
    coef[:, 32 + 15 + 2] = 1.0
    x0 = mlp.assemble_x0(g, coef, None)
    nn = g.n_nodes
    sl = g.pore_slice(3)
    th = np.arctan2(g.y[sl] - g.cy[3], g.x[sl] - g.cx[3])
    np.testing.assert_allclose(x0[:nn][sl], np.cos(th), atol=1e-14)
    np.testing.assert_allclose(x0[nn:2 * nn][sl], np.sin(2 * th), atol=1e-14)
    # mean of cos over the circle is 0 -> lambda_x = 0; mu = 0 by symmetry
    assert abs(x0[2 * nn + 9]) < 1e-14
    assert math.isfinite(x0[-1])


def test_refine_solves_wall_rows_and_minimises_along_x0(geom30):
    """Without scaling the wall rows of the residual vanish; the scaled
    guess satisfies the normal equation of min ||f - alpha A x|| and is never
    worse than the zero start."""
    from stokes_inputs import poiseuille_rhs
    g = geom30
    f = poiseuille_rhs(g)
    rng = np.random.default_rng(9)
    x0 = mlp.assemble_x0(g, rng.standard_normal((g.n_pores, 64)), None)
    a = dlp.assemble(g)
    x1, one = mlp.refine(g, f, x0, apply=lambda v: a @ v, scale=False)
    assert one == 1.0
    r = f - a @ x1
    ws = g.wall_slice
    nn = g.n_nodes
    assert np.abs(r[:nn][ws]).max() < 1e-10 * np.abs(f).max()
    assert np.abs(r[nn:2 * nn][ws]).max() < 1e-10 * np.abs(f).max()
    x2, alpha = mlp.refine(g, f, x0, apply=lambda v: a @ v)
    np.testing.assert_allclose(x2, alpha * x1, rtol=1e-12, atol=0)
    y = a @ x1
    assert abs((f - alpha * y) @ y) < 1e-10 * np.linalg.norm(f) * np.linalg.norm(y)
    assert np.linalg.norm(f - a @ x2) <= np.linalg.norm(f)
