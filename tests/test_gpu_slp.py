"""The single-layer (first-kind) path through the C ABI against the
single-layer oracle (Section 2.1, equation "stokesBIE"; Section 2.2, the
corrected trapezoid rule; equation "stokesSLP_discretized").

Parity: the correction weights (two independent derivations) to 1e-14; the
matvec and block assembly to the FP64 bar (1e-13 of the row scale); the
solution's velocity in the fluid against the velocity of the oracle's LU
solution (the density itself is not unique: the single layer of the normal
density of every closed curve vanishes on the boundary, so only the
velocity, which those directions do not change, is compared)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import slp
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


@pytest.fixture(scope="module")
def small():
    cx, cy, rr = place_pores(np.random.default_rng(1), 6, 4.0, 0.05, 0.1, 0.05, 0.1)
    g = build_geometry(4.0, 512, cx, cy, rr, 64)
    return g, slp.assemble(g)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_weights_match_oracle(lib):
    g_dev = lib.slp_weights()
    g_ref = slp.kr_log_weights(6)
    assert np.abs(g_dev - g_ref).max() <= 1e-14 * np.abs(g_ref).max()


@pytest.mark.parametrize("accurate", [False, True])
def test_matvec_matches_oracle(lib, small, accurate):
    g, a = small
    dg = lib.DeviceGeometry(g)
    for seed in (1, 2):
        x = random_vector(2 * g.n_nodes, seed)
        ref = a @ x
        y = lib.slp_matvec(dg, dev(x), accurate=accurate).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_matvec_matches_oracle_rows_pipe200(lib):
    g = make_geometry("pipe200", 100)
    dg = lib.DeviceGeometry(g)
    x = random_vector(2 * g.n_nodes, 3)
    y = lib.slp_matvec(dg, dev(x)).cpu().numpy()
    rows = np.sort(np.random.default_rng(4).choice(2 * g.n_nodes, 48, replace=False))
    ref = slp.rows_of_matrix(g, rows) @ x
    assert np.abs(y[rows] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_assemble_matches_oracle(lib, small):
    g, a = small
    dg = lib.DeviceGeometry(g)
    rng = np.random.default_rng(5)
    rows = rng.choice(2 * g.n_nodes, 300, replace=False)
    cols = rng.choice(2 * g.n_nodes, 200, replace=False)
    blk = lib.slp_assemble(dg, rows, cols).cpu().numpy()
    ref = a[np.ix_(rows, cols)]
    assert np.abs(blk - ref).max() <= 1e-14 * np.abs(a).max()
    # a whole pore block, with its corrected neighbours and zero diagonal
    k = g.pore_slice(2)
    idx = np.r_[np.arange(k.start, k.stop), g.n_nodes + np.arange(k.start, k.stop)]
    blk = lib.slp_assemble(dg, idx, idx).cpu().numpy()
    assert np.abs(blk - a[np.ix_(idx, idx)]).max() <= 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("pc,tol,bound", [(None, 1e-9, 1e-6), ("bd", 1e-12, 1e-8)])
def test_solve_velocity_matches_oracle_lu(lib, small, pc, tol, bound):
    """Stokeslet/rotlet data (Section 4.2): GPU FGMRES on the first-kind
    system, GPU velocity at interior points, against the oracle's LU
    solution's velocity and the exact field.  Unpreconditioned, the
    first-kind system needs well over a thousand iterations here (the oracle's
    own FGMRES: 1500 iterations reach 1.5e-9), so it runs to 1e-9; with the
    block-diagonal preconditioner it runs to 1e-12 (oracle: 42 iterations)."""
    g, a = small
    nn = g.n_nodes
    f, data = stokeslet_rotlet_rhs(g, 2)
    f = f[:2 * nn]
    sig_ref = sla.lu_solve(sla.lu_factor(a), f)
    dg = lib.DeviceGeometry(g)
    pcobj = lib.BlockDiagonal(dg, single_layer=True) if pc else None
    print(f"[case] single layer pc={pc}", flush=True)
    r = lib.gmres_slp(dg, dev(f), pc=pcobj, tol=tol, max_iter=1800)
    print(f"  iterations {r.iters} true rel res {r.rel_res_true:.2e}")
    assert r.status == 0 and r.rel_res_true <= tol
    rng = np.random.default_rng(0)
    pts = []
    h = g.w[-1]
    while len(pts) < 80:
        p = rng.uniform([0, 0], [4, 1])
        dd = min((np.hypot(p[0] - g.cx, p[1] - g.cy) - g.radius).min(), p[1], 1 - p[1], p[0], 4 - p[0])
        if dd > max(5 * h, math.sqrt(h)):
            pts.append(p)
    pts = np.array(pts)
    ux, uy = lib.slp_velocity(dg, r.sigma, dev(pts[:, 0]), dev(pts[:, 1]))
    ux, uy = ux.cpu().numpy(), uy.cpu().numpy()
    vx, vy = slp.velocity(g, sig_ref, pts[:, 0], pts[:, 1])
    ex, ey = stokeslet_rotlet_field(data, pts[:, 0], pts[:, 1])
    scale = np.max(np.hypot(ex, ey))
    d_oracle = np.max(np.hypot(ux - vx, uy - vy)) / scale
    d_exact = np.max(np.hypot(ux - ex, uy - ey)) / scale
    print(f"  velocity vs oracle LU {d_oracle:.2e}, vs exact {d_exact:.2e}")
    assert d_oracle <= bound
    assert d_exact <= 1e-4


def test_velocity_matches_oracle(lib, small):
    g, _ = small
    dg = lib.DeviceGeometry(g)
    sig = random_vector(2 * g.n_nodes, 9)
    pts = np.random.default_rng(3).uniform([0.2, 0.2], [3.8, 0.8], size=(257, 2))
    ux, uy = lib.slp_velocity(dg, dev(sig), dev(pts[:, 0]), dev(pts[:, 1]))
    vx, vy = slp.velocity(g, sig, pts[:, 0], pts[:, 1])
    scale = max(np.abs(vx).max(), np.abs(vy).max())
    assert np.abs(ux.cpu().numpy() - vx).max() <= 1e-13 * scale
    assert np.abs(uy.cpu().numpy() - vy).max() <= 1e-13 * scale


def test_unsupported_cases(lib, small):
    """The IFMM handle (built for the double layer) and a double-layer
    block-diagonal handle are refused by the single-layer solve."""
    import ctypes
    from paper_1609_04484_amd import _lib as L
    g, _ = small
    dg = lib.DeviceGeometry(g)
    f = dev(np.ones(2 * g.n_nodes))
    ifmm = lib.IFMM(dg, eps=1e-3, cheb_n=6)
    p = L.GmresParams(tol=1e-10, max_iter=5, restart=0, pc=2, use_x0=0, bd=None,
                      ifmm=ifmm.h.value, res_hist=None)
    r = L.GmresResult()
    sig = torch.zeros_like(f)
    code = L.load().gmres_solve_slp(ctypes.byref(dg.c), L._ptr(f), L._ptr(sig), ctypes.byref(p),
                                    ctypes.byref(r), L._stream())
    assert code == -6
    with pytest.raises(lib.SbieError) as e:
        lib.gmres_slp(dg, f, pc=lib.BlockDiagonal(dg), tol=1e-10, max_iter=5)
    assert e.value.code == -1
