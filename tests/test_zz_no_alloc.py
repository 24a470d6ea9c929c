"""The matvec entry point that allocates nothing, through the C ABI, against
the allocating entry point on the same inputs (the product of Section 2.2's
Nystrom operator; FP64 parity bar 1e-13 relative, and bit-identical when
both use the same source-chunk count).

Two calls in a row share the library's fixed scratch array; the second one
is smaller, so stale contents of the first must not leak into it."""
import math

import numpy as np
import pytest

from stokes_inputs import Geometry, make_geometry, random_vector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1609_04484_amd as p
    p.load()
    return p


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_noalloc_matches_matvec_two_calls(lib, mode):
    big = lib.DeviceGeometry(make_geometry("pipe1000", 300))
    small = lib.DeviceGeometry(make_geometry("tiny", 1))
    print(f"[case] noalloc mode {mode}: pipe1000 then tiny", flush=True)
    for dg, seed in ((big, 11), (small, 12)):
        x = dg.vector(random_vector(dg.n, seed))
        ref = lib.matvec(dg, x, mode=mode)
        out = torch.full_like(x, math.nan)
        lib.matvec_noalloc(dg, x, out, mode=mode)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert rel(out, ref) <= 1e-13
    # the small call uses the same chunk count as the allocating one
    assert torch.equal(out, ref)


def test_noalloc_repeated_calls_are_stable(lib):
    dg = lib.DeviceGeometry(make_geometry("pipe200", 100))
    x = dg.vector(random_vector(dg.n, 3))
    out1 = torch.empty_like(x)
    out2 = torch.empty_like(x)
    lib.matvec_noalloc(dg, x, out1)
    lib.matvec_noalloc(dg, x, out2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    assert rel(out1, lib.matvec(dg, x)) <= 1e-13


def test_noalloc_rejects_problems_beyond_its_scratch(lib):
    """A valid single-curve geometry with 0.9 M nodes needs more than the
    fixed array holds: the call fails on the host before any launch."""
    n = 900_000
    th = 2 * math.pi * np.arange(n) / n
    c, s = np.cos(th), np.sin(th)
    g = Geometry(x=c, y=s, nx=c, ny=s, tx=-s, ty=c, w=np.full(n, 2 * math.pi / n),
                 kappa=np.full(n, -1.0), cx=np.zeros(0), cy=np.zeros(0), radius=np.zeros(0),
                 curve_off=np.array([0, n]), length=2.0, n_int=0, n_ext=n)
    dg = lib.DeviceGeometry(g)
    x = dg.vector(np.zeros(dg.n))
    out = torch.empty_like(x)
    with pytest.raises(lib.SbieError) as e:
        lib.matvec_noalloc(dg, x, out)
    assert e.value.code == -1
