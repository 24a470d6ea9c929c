"""Velocity evaluation in the fluid through the C ABI (Section 2.2: the
trapezoid rule for the layer potential at points of the fluid; Section
4.1.1: the relative velocity-magnitude error).

Parity: the GPU velocity against the oracle's (oracle/dlp.py velocity) on the
same density and points, FP64 bar 1e-13 relative; the error metric against
its definition evaluated on the oracle's velocity.  Then the whole path on
the GPU (FGMRES solve, velocity) reproduces the exact Stokeslet/rotlet
solution with geometric convergence under refinement, as the oracle does."""
import math

import numpy as np
import pytest

from oracle import dlp
from stokes_inputs import (build_geometry, make_geometry, place_pores, random_vector,
                           stokeslet_rotlet_field, stokeslet_rotlet_rhs)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1609_04484_amd as p
    p.load()
    return p


def interior_points(g, count, dmin, seed=0):
    """Uniform points of the pipe at distance > dmin from every curve."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < count:
        p = rng.uniform([0, 0], [g.length, 1])
        dd = min((np.hypot(p[0] - g.cx, p[1] - g.cy) - g.radius).min() if g.n_pores else 1e9,
                 p[1], 1 - p[1], p[0], g.length - p[0])
        if dd > dmin:
            pts.append(p)
    return np.array(pts)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("count", [1, 63, 257, 1000])
def test_velocity_matches_oracle_tiny(lib, count):
    g = make_geometry("tiny", 1)
    dg = lib.DeviceGeometry(g)
    sig = random_vector(g.n_unknowns, 5)
    pts = interior_points(g, count, 0.02, seed=count)
    print(f"[case] velocity tiny, {count} points", flush=True)
    ux, uy = lib.velocity(dg, dg.vector(sig), dev(pts[:, 0]), dev(pts[:, 1]))
    rx, ry = dlp.velocity(g, sig, pts[:, 0], pts[:, 1])
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    assert np.abs(ux.cpu().numpy() - rx).max() <= 1e-13 * scale
    assert np.abs(uy.cpu().numpy() - ry).max() <= 1e-13 * scale


def test_velocity_matches_oracle_pipe200_sampled(lib):
    """Full-size pipe, 20,000 points on the GPU; the oracle recomputes a
    sample of 200 of them."""
    g = make_geometry("pipe200", 100)
    dg = lib.DeviceGeometry(g)
    sig = random_vector(g.n_unknowns, 6)
    pts = interior_points(g, 20000, 0.01, seed=3)
    print("[case] velocity pipe200, 20000 points", flush=True)
    ux, uy = lib.velocity(dg, dg.vector(sig), dev(pts[:, 0]), dev(pts[:, 1]))
    pick = np.random.default_rng(4).choice(len(pts), 200, replace=False)
    rx, ry = dlp.velocity(g, sig, pts[pick, 0], pts[pick, 1])
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    assert np.abs(ux.cpu().numpy()[pick] - rx).max() <= 1e-13 * scale
    assert np.abs(uy.cpu().numpy()[pick] - ry).max() <= 1e-13 * scale


def test_error_metric(lib):
    g = make_geometry("tiny", 1)
    dg = lib.DeviceGeometry(g)
    sig = random_vector(g.n_unknowns, 8)
    pts = interior_points(g, 300, 0.05, seed=9)
    refx, refy = np.cos(pts[:, 0]) + 2.0, np.sin(pts[:, 1])
    ux, uy, err = lib.velocity(dg, dg.vector(sig), dev(pts[:, 0]), dev(pts[:, 1]),
                               uref=(dev(refx), dev(refy)))
    vx, vy = dlp.velocity(g, sig, pts[:, 0], pts[:, 1])
    expect = np.abs(np.hypot(vx, vy) - np.hypot(refx, refy)) / np.hypot(refx, refy)
    assert np.abs(err.cpu().numpy() - expect).max() <= 1e-12 * max(1.0, expect.max())


def test_no_points_and_argument_errors(lib):
    g = make_geometry("tiny", 1)
    dg = lib.DeviceGeometry(g)
    s = dg.vector(np.zeros(g.n_unknowns))
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ux, uy = lib.velocity(dg, s, e, e)
    assert ux.numel() == 0
    import ctypes
    L = lib.load()
    assert L.stokes_velocity(ctypes.byref(dg.c), None, None, None, 5, None, None, None, None, None,
                             None) == -1


def test_whole_path_converges_to_exact_solution(lib):
    """Stokeslet/rotlet boundary data (Section 4.2): GPU FGMRES solve, GPU
    velocity at points farther than max(5h, sqrt(h)) from the boundary; the
    error against the exact field falls geometrically as the nodes double."""
    cx, cy, rr = place_pores(np.random.default_rng(1), 10, 4.0, 0.05, 0.1, 0.05, 0.1)
    errs = []
    for nint, next_ in [(16, 128), (32, 256), (64, 512)]:
        g = build_geometry(4.0, next_, cx, cy, rr, nint)
        f, data = stokeslet_rotlet_rhs(g, 1)
        dg = lib.DeviceGeometry(g)
        r = lib.gmres(dg, dg.vector(f), pc=lib.BlockDiagonal(dg), tol=1e-13, max_iter=500)
        assert r.status == 0
        h = max(2 * math.pi * rr.min() / nint, g.w[-1])
        pts = interior_points(g, 60, max(5 * h, math.sqrt(h)))
        ux, uy = lib.velocity(dg, r.sigma, dev(pts[:, 0]), dev(pts[:, 1]))
        ex, ey = stokeslet_rotlet_field(data, pts[:, 0], pts[:, 1])
        e = np.max(np.hypot(ux.cpu().numpy() - ex, uy.cpu().numpy() - ey)) / np.max(np.hypot(ex, ey))
        print(f"  N_int {nint} N_ext {next_}: {r.iters} iterations, velocity error {e:.2e}")
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[0] < 1e-2
    assert errs[2] < 1e-11
