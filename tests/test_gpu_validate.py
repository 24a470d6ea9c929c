"""Geometry validation through the C ABI: the solver entry points reject a
geometry that breaks what the operator assumes (Section 2: disjoint circular
pores strictly inside a closed wall, distinct quadrature nodes) with
SBIE_INVALID_GEOMETRY before any factorisation or iteration runs.  Every
case is built on the host from a valid pipe; the kernels only read it."""
import copy
import math

import numpy as np
import pytest

from stokes_inputs import make_geometry, poiseuille_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1609_04484_amd as p
    p.load()
    return p


def move_pore(g, k, cx, cy):
    sl = g.pore_slice(k)
    g.x[sl] += cx - g.cx[k]
    g.y[sl] += cy - g.cy[k]
    g.cx[k], g.cy[k] = cx, cy


def broken(case):
    g = copy.deepcopy(make_geometry("tiny", 1))
    if case == "overlap":
        move_pore(g, 1, g.cx[0] + 0.5 * g.radius[0], g.cy[0])
    elif case == "outside":
        move_pore(g, 2, 1.0, 1.6)
    elif case == "crosses_wall":
        move_pore(g, 3, 2.0, 0.5 * g.radius[3])
    elif case == "nan":
        g.x[5] = math.nan
    elif case == "duplicate":
        ws = g.wall_slice
        g.x[ws.start + 7] = g.x[ws.start + 8]
        g.y[ws.start + 7] = g.y[ws.start + 8]
    elif case == "off_circle":
        g.x[g.pore_slice(4).start] += 1e-3
    elif case == "bad_radius":
        g.radius[0] = -g.radius[0]
    return g


def test_valid_geometries_pass(lib):
    for name, seed in (("tiny", 1), ("pipe200", 100), ("pipe1000", 300)):
        lib.validate(lib.DeviceGeometry(make_geometry(name, seed)))


@pytest.mark.parametrize("case", ["overlap", "outside", "crosses_wall", "nan", "duplicate",
                                  "off_circle", "bad_radius"])
def test_invalid_geometry_rejected(lib, case):
    g = broken(case)
    dg = lib.DeviceGeometry(g)
    print(f"[case] {case}", flush=True)
    with pytest.raises(lib.SbieError) as e:
        lib.validate(dg)
    assert e.value.code == -2
    with pytest.raises(lib.SbieError) as e:
        lib.BlockDiagonal(dg)
    assert e.value.code == -2
    with pytest.raises(lib.SbieError) as e:
        lib.IFMM(dg, eps=1e-3, cheb_n=6)
    assert e.value.code == -2
    f = dg.vector(np.nan_to_num(poiseuille_rhs(g)))
    with pytest.raises(lib.SbieError) as e:
        lib.gmres(dg, f, tol=1e-10, max_iter=5)
    assert e.value.code == -2
