"""End-to-end parity at the two large workloads: FGMRES solutions from the
C ABI against the stored oracle solutions sigma* = A^{-1} F.

The stored solutions (tests/golden/sigma_*.npy) were written by
tests/golden/make_sigma.py, which calls only the CPU oracle: a dense LU with
iterative refinement for the 200-pore pipe (n = 59,992) and the oracle's
block-diagonal FGMRES with 80-bit residuals for the 1000-pore pipe
(n = 139,192).  Their JSON records hold the final residuals.

Tolerance: every solution must match sigma* to a relative error of 1e-8
(the accuracy target of the whole solve).  The solves run to a true
relative residual of 1e-11, a decade below the bench's 1e-10, because the
density is ~1e3 times larger than the data on these pipes, so the error
bound ||A^-1|| ||r|| / ||sigma|| is up to that factor above the residual
(Section 3.3 makes the IFMM accuracy eps a preconditioner parameter only: it
must not change the converged solution).
"""
import json
import os

import numpy as np
import pytest

from stokes_inputs import make_geometry, poiseuille_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1609_04484_amd as p
    p.load()
    return p


def golden(work, seed):
    base = os.path.join(GOLDEN, f"sigma_{work}_s{seed}")
    sig = np.load(base + ".npy", allow_pickle=False)
    with open(base + ".json") as fh:
        meta = json.load(fh)
    # a residual of 1e-12, or the floor that rounding sigma* to FP64 leaves,
    # u ||A|| ||sigma*|| / ||f|| with ||A|| ~ 1 (||sigma*|| / ||f|| = 1.8e5 on
    # the 1000-pore pipe: its stored residual, 5.3e-12, sits at that floor)
    floor = 2.2e-16 * meta["sigma_norm_over_f_norm"]
    assert meta["final_rel_residual_80bit"] < max(1e-12, 0.5 * floor), meta
    return sig, meta


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


@pytest.fixture(scope="module")
def pipe200(lib):
    g = make_geometry("pipe200", 100)
    f = poiseuille_rhs(g)
    sig, _ = golden("pipe200", 100)
    dg = lib.DeviceGeometry(g)
    return g, dg, dg.vector(f), sig


@pytest.fixture(scope="module")
def pipe1000(lib):
    g = make_geometry("pipe1000", 300)
    f = poiseuille_rhs(g)
    sig, _ = golden("pipe1000", 300)
    dg = lib.DeviceGeometry(g)
    return g, dg, dg.vector(f), sig


def _solve(lib, dg, fd, kind, eps=None, cheb_n=None, precision=0, tol=1e-11):
    if kind == "bd":
        pc = lib.BlockDiagonal(dg)
    else:
        pc = lib.IFMM(dg, eps=eps, cheb_n=cheb_n, precision=precision)
    try:
        r = lib.gmres(dg, fd, pc=pc, tol=tol, max_iter=2000)
    finally:
        pc.close()
    return r


def test_stored_solutions_satisfy_the_oracle_operator():
    """The stored records: residuals far below the solve tolerance."""
    for work, seed in (("pipe200", 100), ("pipe1000", 300)):
        _, meta = golden(work, seed)
        assert meta["n"] == make_geometry(work, seed).n_unknowns


@pytest.mark.parametrize("kind,eps,cheb_n,precision", [
    ("bd", None, None, 0),
    ("ifmm", 1e-3, 6, 0),
    ("ifmm", 1e-3, 6, 1),
    ("ifmm", 1e-3, 6, 2),
    ("ifmm", 1e-6, 10, 0),
    ("ifmm", 1e-6, 10, 1),
    ("ifmm", 1e-6, 10, 2),
])
def test_pipe200_solution_matches_dense_lu(lib, pipe200, kind, eps, cheb_n, precision):
    g, dg, fd, sig = pipe200
    print(f"[case] pipe200 seed 100 {kind} eps={eps} n={cheb_n} precision={precision}", flush=True)
    r = _solve(lib, dg, fd, kind, eps, cheb_n, precision)
    err = rel(r.sigma.cpu().numpy(), sig)
    print(f"  iters {r.iters} true rel res {r.rel_res_true:.2e} error vs sigma* {err:.2e}")
    assert r.status == 0 and r.rel_res_true <= 1e-11
    assert err <= 1e-8


@pytest.mark.parametrize("kind,eps,cheb_n,precision", [
    ("ifmm", 1e-5, 6, 0),
    ("ifmm", 1e-5, 6, 2),
    ("bd", None, None, 0),
])
def test_pipe1000_solution_matches_oracle_fgmres(lib, pipe1000, kind, eps, cheb_n, precision):
    """The bench workload (9-level tree, ranks above 200): the headline
    solver settings, to the bench's tolerance 1e-10, against the oracle's
    solution.  (A true residual of 1e-11 is at the floor that FP64 leaves on
    this pipe, where ||sigma|| / ||f|| = 1.8e5: the oracle's own solve stopped
    at 5.3e-12.)"""
    g, dg, fd, sig = pipe1000
    print(f"[case] pipe1000 seed 300 {kind} eps={eps} n={cheb_n} precision={precision}", flush=True)
    r = _solve(lib, dg, fd, kind, eps, cheb_n, precision, tol=1e-10)
    err = rel(r.sigma.cpu().numpy(), sig)
    print(f"  iters {r.iters} true rel res {r.rel_res_true:.2e} error vs sigma* {err:.2e}")
    assert r.status == 0 and r.rel_res_true <= 1e-10
    assert err <= 1e-8
