"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Run on an MI355X with ``pytest -m gpu``.  Every comparison is element by
element on the same seeded inputs; tolerances are stated per test.
"""
import math

import numpy as np
import pytest

from oracle import dlp, solve
from stokes_inputs import (Geometry, build_geometry, make_geometry, place_pores,
                           poiseuille_rhs, random_vector, shear_rhs,
                           stokeslet_rotlet_rhs)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1609_04484_amd as p
    p.load()
    return p


def single_circle(n, r=0.3):
    th = 2 * math.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    return Geometry(x=r * c, y=r * s, nx=-c, ny=-s, tx=-s, ty=c,
                    w=np.full(n, 2 * math.pi * r / n), kappa=np.full(n, 1 / r),
                    cx=np.array([0.0]), cy=np.array([0.0]), radius=np.array([r]),
                    curve_off=np.array([0, n, n]), length=1.0, n_int=n, n_ext=0)


def wall_only(n_ext=256, length=3.0):
    return build_geometry(length, n_ext, [], [], [], 0)


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def tiny():
    g = make_geometry("tiny", 1)
    return g, dlp.assemble(g)


# ------------------------------------------------------------------ matvec --

def test_matvec_full_matches_dense_oracle(lib, tiny):
    g, a = tiny
    dg = lib.DeviceGeometry(g)
    for seed in (1, 2):
        x = random_vector(g.n_unknowns, seed)
        y = lib.matvec(dg, dg.vector(x)).cpu().numpy()
        ref = a @ x
        assert rel_inf(y, ref) < 1e-13, rel_inf(y, ref)


def test_matvec_dlp_only_matches_oracle(lib, tiny):
    g, _ = tiny
    dg = lib.DeviceGeometry(g)
    x = random_vector(g.n_unknowns, 3)
    y = lib.matvec(dg, dg.vector(x), mode=1).cpu().numpy()
    nn = g.n_nodes
    ref = dlp.dlp_only_rows(g, x, np.arange(2 * nn))
    assert rel_inf(y[:2 * nn], ref) < 1e-13
    assert np.all(y[2 * nn:] == 0.0)


@pytest.mark.parametrize("tpt,chunks", [(1, 0), (2, 3), (4, 0), (8, 1), (4, 17), (4, 8), (2, 16), (1, 24)])
def test_matvec_launch_shapes_agree(lib, tiny, tpt, chunks):
    g, a = tiny
    dg = lib.DeviceGeometry(g)
    x = random_vector(g.n_unknowns, 4)
    try:
        lib.set_matvec_shape(tpt, chunks)
        y = lib.matvec(dg, dg.vector(x)).cpu().numpy()
    finally:
        lib.set_matvec_shape(4, 0)
    assert rel_inf(y, a @ x) < 1e-13


def test_matvec_edge_geometries(lib):
    """One pore and no wall (no rank-one term), and a wall with no pores."""
    for g in (single_circle(37), wall_only(130)):
        a = dlp.assemble(g)
        dg = lib.DeviceGeometry(g)
        x = random_vector(g.n_unknowns, 5)
        y = lib.matvec(dg, dg.vector(x)).cpu().numpy()
        assert rel_inf(y, a @ x) < 1e-13


@pytest.fixture
def symmetric_always(lib):
    lib.set_matvec_symmetric(2)
    yield
    lib.set_matvec_symmetric(1)


@pytest.mark.parametrize("mode", [0, 1])
def test_symmetric_pairs_match_oracle(lib, tiny, symmetric_always, mode):
    """The symmetric pair evaluation (each unordered pair once for both
    directions) forced on small geometries: the tiny pipe (5 tiles, one
    superblock pair, ragged last tile), one pore (one partial tile, only the
    diagonal tile), a wall without pores, and 3000 nodes (3 superblocks per
    side: off-diagonal superblock pairs and both slot families)."""
    g, a = tiny
    cases = [(g, a), (single_circle(37), None), (wall_only(130), None),
             (make_geometry(dict(length=6.0, n_ext=1024, n_pores=30, r_lo=0.03, r_hi=0.06, n_int=64,
                                 gap_pore=0.02, gap_wall=0.08), 9), None)]
    for g_, a_ in cases:
        a_ = dlp.assemble(g_) if a_ is None else a_
        dg = lib.DeviceGeometry(g_)
        x = random_vector(g_.n_unknowns, 6)
        y = lib.matvec(dg, dg.vector(x), mode).cpu().numpy()
        ref = a_ @ x if mode == 0 else dlp.dlp_only_rows(g_, x, np.arange(2 * g_.n_nodes))
        assert rel_inf(y[:ref.shape[0]], ref) < 1e-13, g_.n_nodes


def test_symmetric_and_chunked_pairs_agree(lib):
    """At the 200-pore pipe (59,992 unknowns, 15 superblocks per side) the
    default plan is symmetric; it agrees with the chunked kernel to rounding
    and is deterministic (two products bit for bit equal)."""
    g = make_geometry("pipe200", 100)
    dg = lib.DeviceGeometry(g)
    assert lib.matvec_plan(dg)["symmetric"] and lib.matvec_plan(dg, 1)["symmetric"]
    assert not lib.matvec_plan(dg, 2)["symmetric"]          # compensated: chunked kernel
    assert not lib.matvec_plan(lib.DeviceGeometry(make_geometry("tiny", 1)))["symmetric"]
    x = dg.vector(random_vector(g.n_unknowns, 12))
    y_sym = lib.matvec(dg, x)
    y_sym2 = lib.matvec(dg, x)
    assert torch.equal(y_sym, y_sym2)
    try:
        lib.set_matvec_symmetric(0)
        y_chk = lib.matvec(dg, x)
    finally:
        lib.set_matvec_symmetric(1)
    d = float((y_sym - y_chk).abs().max() / y_chk.abs().max())
    print(f"symmetric vs chunked: {d:.2e}")
    assert d < 1e-14


def test_matvec_constant_density_identity(lib, tiny):
    """Principal-value sum of a constant density is -c/2 at every node."""
    g, _ = tiny
    dg = lib.DeviceGeometry(g)
    nn = g.n_nodes
    x = np.zeros(g.n_unknowns)
    x[:nn], x[nn:2 * nn] = 0.7, -1.3
    y = lib.matvec(dg, dg.vector(x), mode=1).cpu().numpy()
    assert np.abs(y[:nn] + 0.35).max() < 1e-12
    assert np.abs(y[nn:2 * nn] - 0.65).max() < 1e-12


@pytest.mark.parametrize("name,seed", [("pipe200", 100), ("pipe1000", 300)])
def test_matvec_full_size_sampled_rows(lib, name, seed):
    """Full-size workloads: sampled rows (node rows of both components,
    pore rows and wall rows) computed one by one by the oracle."""
    g = make_geometry(name, seed)
    dg = lib.DeviceGeometry(g)
    x = random_vector(g.n_unknowns, seed)
    y = lib.matvec(dg, dg.vector(x)).cpu().numpy()
    rng = np.random.default_rng(seed)
    nn = g.n_nodes
    rows = np.unique(np.concatenate([
        rng.integers(0, 2 * nn, 120),
        2 * nn + rng.integers(0, 3 * g.n_pores, 30),
        np.arange(g.wall_slice.start, g.wall_slice.start + 5),
        nn + np.arange(nn - 5, nn),
        [0, g.n_unknowns - 1],
    ]))
    ref = dlp.apply_rows(g, x, rows)
    scale = np.abs(ref).max()
    assert np.abs(y[rows] - ref).max() / scale < 1e-13


# ---------------------------------------------------------------- assemble --

def test_assemble_matches_oracle(lib, tiny):
    g, a = tiny
    dg = lib.DeviceGeometry(g)
    rng = np.random.default_rng(7)
    n = g.n_unknowns
    rows = np.concatenate([rng.integers(0, n, 97), [0, n - 1, 2 * g.n_nodes]])
    cols = np.concatenate([rng.integers(0, n, 61), rows[:5], [n - 1]])
    blk = lib.assemble(dg, rows, cols).cpu().numpy()
    ref = a[np.ix_(rows, cols)]
    assert np.abs(blk - ref).max() <= 1e-14 * np.abs(a).max()


def test_assemble_empty(lib, tiny):
    g, _ = tiny
    dg = lib.DeviceGeometry(g)
    out = lib.assemble(dg, np.zeros(0, dtype=np.int64), np.arange(3))
    assert out.shape == (0, 3)


# -------------------------------------------------------------- block diag --

def test_block_diagonal_apply_matches_oracle(lib, tiny):
    g, a = tiny
    dg = lib.DeviceGeometry(g)
    bd = lib.BlockDiagonal(dg)
    ref = solve.BlockDiagonal(g, a)
    for seed in (11, 12):
        v = random_vector(g.n_unknowns, seed)
        z = bd.solve(dg.vector(v)).cpu().numpy()
        assert rel_inf(z, ref(v)) < 1e-11


def test_block_diagonal_medium_wall(lib):
    """A wall block spanning several 128-wide inversion tiles plus a ragged
    tail (2 * 600 = 1200 unknowns)."""
    cx, cy, rr = place_pores(np.random.default_rng(5), 6, 3.0, 0.03, 0.08, 0.02, 0.1)
    g = build_geometry(3.0, 600, cx, cy, rr, 48)
    a = dlp.assemble(g)
    dg = lib.DeviceGeometry(g)
    bd = lib.BlockDiagonal(dg)
    v = random_vector(g.n_unknowns, 13)
    z = bd.solve(dg.vector(v)).cpu().numpy()
    assert rel_inf(z, solve.BlockDiagonal(g, a)(v)) < 1e-11


# ------------------------------------------------------------------- gmres --

@pytest.mark.parametrize("pc", ["none", "bd"])
def test_gmres_matches_lu(lib, tiny, pc):
    g, a = tiny
    f, _ = stokeslet_rotlet_rhs(g, 1)
    sig = solve.lu_solve(a, f)
    dg = lib.DeviceGeometry(g)
    p = None if pc == "none" else lib.BlockDiagonal(dg)
    r = lib.gmres(dg, dg.vector(f), pc=p, tol=1e-12)
    assert r.status == 0
    x = r.sigma.cpu().numpy()
    assert np.linalg.norm(f - a @ x) / np.linalg.norm(f) < 1e-12
    assert np.linalg.norm(x - sig) / np.linalg.norm(sig) < 1e-8


def test_gmres_iteration_counts_close_to_oracle(lib, tiny):
    g, a = tiny
    f = poiseuille_rhs(g)
    dg = lib.DeviceGeometry(g)
    r_gpu = lib.gmres(dg, dg.vector(f), pc=lib.BlockDiagonal(dg), tol=1e-10)
    r_cpu = solve.fgmres(lambda v: a @ v, f, precond=solve.BlockDiagonal(g, a), tol=1e-10)
    assert abs(r_gpu.iters - r_cpu.iters) <= 2


def test_gmres_exact_start_and_cap(lib, tiny):
    g, a = tiny
    f = shear_rhs(g)
    sig = solve.lu_solve(a, f)
    dg = lib.DeviceGeometry(g)
    r = lib.gmres(dg, dg.vector(f), tol=1e-10, x0=dg.vector(sig))
    assert r.iters == 0 and r.status == 0
    r = lib.gmres(dg, dg.vector(f), tol=1e-10, max_iter=1)
    assert r.status == 1 and r.iters == 1
    # restarted GMRES(60) converges, like the oracle's restarted FGMRES
    r = lib.gmres(dg, dg.vector(f), tol=1e-10, restart=60, max_iter=600)
    ref = solve.fgmres(lambda v: a @ v, f, tol=1e-10, restart=60, max_iter=600)
    assert ref.converged
    assert r.status == 0 and r.rel_res_true < 1e-10
    # the device cycles aim at tol/2 before the compensated true-residual
    # check, so they may run a few iterations longer than the oracle's
    assert abs(r.iters - ref.iters) <= max(5, 0.1 * ref.iters)
    # short restarts stagnate on this system on both sides
    r = lib.gmres(dg, dg.vector(f), tol=1e-10, restart=15, max_iter=300)
    ref = solve.fgmres(lambda v: a @ v, f, tol=1e-10, restart=15, max_iter=300)
    assert r.status == 1 and not ref.converged


def test_gmres_nonfinite_rhs_is_an_error(lib, tiny):
    g, _ = tiny
    dg = lib.DeviceGeometry(g)
    f = poiseuille_rhs(g)
    f[3] = np.nan
    with pytest.raises(lib.SbieError) as e:
        lib.gmres(dg, dg.vector(f), tol=1e-10)
    assert e.value.code == -5


def test_gmres_zero_rhs(lib, tiny):
    g, _ = tiny
    dg = lib.DeviceGeometry(g)
    r = lib.gmres(dg, dg.vector(np.zeros(g.n_unknowns)), tol=1e-10)
    assert r.iters == 0 and float(r.sigma.abs().max()) == 0.0


def test_matvec_compensated_mode(lib, tiny):
    """The compensated mode computes the same product; on the full-size
    workload it agrees with the plain mode to the plain mode's rounding and
    with the oracle's rows."""
    g, a = tiny
    dg = lib.DeviceGeometry(g)
    x = random_vector(g.n_unknowns, 21)
    y = lib.matvec(dg, dg.vector(x), mode=2).cpu().numpy()
    assert rel_inf(y, a @ x) < 1e-14


def test_matvec_compensated_full_size(lib):
    g = make_geometry("pipe1000", 300)
    dg = lib.DeviceGeometry(g)
    f = poiseuille_rhs(g)
    # a density of the size the solver produces: large pore densities
    x = 100.0 * random_vector(g.n_unknowns, 5)
    y2 = lib.matvec(dg, dg.vector(x), mode=2).cpu().numpy()
    y0 = lib.matvec(dg, dg.vector(x), mode=0).cpu().numpy()
    rows = np.sort(np.random.default_rng(3).choice(g.n_unknowns, 200, replace=False))
    ref = dlp.apply_rows(g, x, rows)
    scale = np.abs(ref).max()
    assert np.abs(y2[rows] - ref).max() / scale < 1e-13
    assert np.abs(y2 - y0).max() / np.abs(y2).max() < 1e-12
