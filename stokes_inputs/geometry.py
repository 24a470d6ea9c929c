"""Seeded synthetic geometries for the porous-pipe Stokes problem.

This module only *describes the input*: the boundary curves, their Nystrom
nodes, unit normals, quadrature weights and curvature, and the pore centres.
It contains none of the solver's arithmetic and is shared by the CPU oracle
and by the GPU path as their common input.

Geometry (Section 2 of the paper): the outer wall Gamma_0 is a smoothed
("mollified") rectangle [0, L] x [0, 1] and the pores Gamma_k are circles of
varying radii.  The paper does not say how the corners are rounded; here the
wall is a C-infinity curve parameterised by arclength whose curvature is a sum
of four periodised Gaussian bumps of width ``delta`` centred on the corners,
each carrying a quarter turn.  Nodes are equispaced in arclength, so the
trapezoid rule applies with weight ``perimeter / N_ext`` (Section 2.2).

Node order: pores 1..M first (N_int nodes each), then the wall (N_ext nodes),
following the paper's numbering of the degrees of freedom (Section 4.1.1).

Orientation conventions:
* ``n`` is the unit normal pointing OUT of the fluid: away from Omega_0 on the
  wall, towards the pore centre on a pore.
* ``kappa`` holds x_ss . n (curvature vector dotted with n): +1/r on a pore
  and minus the geometric curvature (<= 0) on the convex wall.
* ``(tx, ty)`` is the unit tangent (wall: counter-clockwise).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf


@dataclasses.dataclass
class Geometry:
    """Discretised boundary: SoA node arrays plus per-pore data."""

    x: np.ndarray
    y: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    tx: np.ndarray
    ty: np.ndarray
    w: np.ndarray
    kappa: np.ndarray
    cx: np.ndarray  # pore centres (completion points), length M
    cy: np.ndarray
    radius: np.ndarray  # pore radii, length M
    curve_off: np.ndarray  # int64, M + 2 offsets; curve M is the wall
    length: float  # pipe length L
    n_int: int  # nodes per pore (0 if no pores)
    n_ext: int  # wall nodes

    @property
    def n_pores(self) -> int:
        return int(self.cx.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_unknowns(self) -> int:
        return 2 * self.n_nodes + 3 * self.n_pores

    @property
    def wall_slice(self) -> slice:
        return slice(int(self.curve_off[-2]), int(self.curve_off[-1]))

    def pore_slice(self, k: int) -> slice:
        return slice(int(self.curve_off[k]), int(self.curve_off[k + 1]))


# ----------------------------------------------------------------------------
# Outer wall: C-infinity rounded rectangle
# ----------------------------------------------------------------------------

def _corner_layout(a: float, b: float):
    """Arclength positions of the four corners; s = 0 is mid-bottom side."""
    return np.array([0.5 * a, 0.5 * a + b, 1.5 * a + b, 1.5 * a + 2.0 * b])


def _theta(s: np.ndarray, a: float, b: float, delta: float) -> np.ndarray:
    """Tangent angle theta(s) = integral_0^s kappa, with theta(0) = 0."""
    per = 2.0 * a + 2.0 * b
    th = np.zeros_like(s)
    for sc in _corner_layout(a, b):
        for img in range(-2, 3):
            c = sc + img * per
            # Phi(u) - Phi(v) with Phi the unit Gaussian CDF
            th += 0.5 * (erf((s - c) / (math.sqrt(2.0) * delta))
                         - erf((0.0 - c) / (math.sqrt(2.0) * delta)))
    return th * (math.pi / 2.0)


def _curvature(s: np.ndarray, a: float, b: float, delta: float) -> np.ndarray:
    per = 2.0 * a + 2.0 * b
    k = np.zeros_like(s)
    g = 1.0 / (math.sqrt(2.0 * math.pi) * delta)
    for sc in _corner_layout(a, b):
        for img in range(-2, 3):
            d = s - sc - img * per
            k += g * np.exp(-0.5 * (d / delta) ** 2)
    return k * (math.pi / 2.0)


def _wall_positions(s_nodes: np.ndarray, a: float, b: float, delta: float,
                    refine: int = 8):
    """Spectrally integrate (cos theta, sin theta) and sample at the nodes.

    The tangent is sampled on a grid ``refine`` times finer than the nodes
    (which are a subset of it), integrated in Fourier space, and the periodic
    primitive is read off at the nodes.
    """
    per = 2.0 * a + 2.0 * b
    n = s_nodes.shape[0]
    kf = n * refine
    sf = np.arange(kf) * (per / kf)
    th = _theta(sf, a, b, delta)
    out = []
    for comp in (np.cos(th), np.sin(th)):
        c = np.fft.rfft(comp) / kf
        m = np.arange(c.shape[0])
        kk = 2.0 * math.pi * m / per
        # closure: the mean of the tangent over one period is zero
        prim = np.zeros_like(c)
        prim[1:] = c[1:] / (1j * kk[1:])
        # primitive P(s) = sum prim_m e^{i k s}; integral_0^s = P(s) - P(0)
        full = np.fft.irfft(prim * kf, n=kf)
        vals = full[::refine] - full[0]
        out.append(vals)
    return out[0], out[1]


def rounded_rectangle(length: float, n_ext: int, delta: float = 0.1,
                      height: float = 1.0):
    """Nodes of the smoothed rectangle [0, length] x [0, height].

    Returns arrays x, y, tx, ty, nx, ny, w, kappa (x_ss . n) and the
    perimeter.  The straight-side lengths are adjusted by a short fixed-point
    iteration so that the extents are exactly the requested rectangle.
    """
    if n_ext < 16 or n_ext % 2:
        raise ValueError("n_ext must be an even number >= 16")
    a = length - 0.6 * delta
    b = height - 0.6 * delta
    for _ in range(6):
        probe = np.array([0.0, 0.5 * a + 0.5 * b, a + b, 1.5 * a + 1.5 * b])
        # the extents are attained at the side midpoints (symmetry)
        px, py = _probe_positions(probe, a, b, delta)
        width = px[1] - px[3]
        hgt = py[2] - py[0]
        a += length - width
        b += height - hgt
    per = 2.0 * a + 2.0 * b
    sn = np.arange(n_ext) * (per / n_ext)
    x, y = _wall_positions(sn, a, b, delta)
    th = _theta(sn, a, b, delta)
    tx, ty = np.cos(th), np.sin(th)
    # counter-clockwise: the outward normal of Omega_0 is (ty, -tx)
    nx, ny = ty.copy(), -tx.copy()
    kappa = -_curvature(sn, a, b, delta)
    # place the bottom-side midpoint (s = 0) at (length/2, 0)
    x = x + 0.5 * length
    y = y - 0.0
    w = np.full(n_ext, per / n_ext)
    return dict(x=x, y=y, tx=tx, ty=ty, nx=nx, ny=ny, w=w, kappa=kappa,
                perimeter=per, a=a, b=b)


def _probe_positions(s_probe, a, b, delta, n_quad: int = 8192):
    """Positions at arbitrary arclengths (relative to s = 0) by evaluating the
    Fourier series of the primitive of the tangent."""
    per = 2.0 * a + 2.0 * b
    sf = np.arange(n_quad) * (per / n_quad)
    th = _theta(sf, a, b, delta)
    m = np.fft.fftfreq(n_quad, d=1.0 / n_quad)
    kk = 2.0 * math.pi * m / per
    nz = m != 0
    res = []
    for comp in (np.cos(th), np.sin(th)):
        c = np.fft.fft(comp) / n_quad
        vals = []
        for sp in np.atleast_1d(s_probe):
            ph = np.exp(1j * kk[nz] * sp) - 1.0
            vals.append(float((c[nz] / (1j * kk[nz]) * ph).sum().real))
        res.append(np.array(vals))
    return res[0], res[1]


# ----------------------------------------------------------------------------
# Pores
# ----------------------------------------------------------------------------

def place_pores(rng: np.random.Generator, n_pores: int, length: float,
                r_lo: float, r_hi: float, gap_pore: float, gap_wall: float,
                x_margin: float = 0.5, max_tries: int = 1_000_000,
                height: float = 1.0):
    """Random non-overlapping circles by rejection sampling.

    Radius ~ U[r_lo, r_hi]; centre x ~ U[x_margin, L - x_margin],
    y ~ U[r + gap_wall, height - r - gap_wall]; a candidate is accepted when
    its gap to every accepted pore is at least ``gap_pore``.
    """
    cell = 2.0 * r_hi + gap_pore
    grid: dict = {}
    cx = np.empty(n_pores)
    cy = np.empty(n_pores)
    rr = np.empty(n_pores)
    k = 0
    tries = 0
    while k < n_pores:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("pore placement failed: too many rejections")
        r = rng.uniform(r_lo, r_hi)
        x = rng.uniform(x_margin, length - x_margin)
        lo, hi = r + gap_wall, height - r - gap_wall
        if hi <= lo:
            raise RuntimeError("pore does not fit between the walls")
        y = rng.uniform(lo, hi)
        gx, gy = int(x // cell), int(y // cell)
        ok = True
        for ix in (gx - 1, gx, gx + 1):
            for iy in (gy - 1, gy, gy + 1):
                for j in grid.get((ix, iy), ()):
                    d = math.hypot(x - cx[j], y - cy[j])
                    if d - r - rr[j] < gap_pore:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        cx[k], cy[k], rr[k] = x, y, r
        grid.setdefault((gx, gy), []).append(k)
        k += 1
    return cx, cy, rr


def build_geometry(length: float, n_ext: int, cx, cy, radius, n_int: int,
                   delta: float = 0.1, n_int_per_pore=None) -> Geometry:
    """Assemble the SoA node arrays (pores first, then the wall)."""
    cx = np.asarray(cx, dtype=np.float64)
    cy = np.asarray(cy, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    m = cx.shape[0]
    counts = (np.full(m, n_int, dtype=np.int64) if n_int_per_pore is None
              else np.asarray(n_int_per_pore, dtype=np.int64))
    parts = {k: [] for k in ("x", "y", "nx", "ny", "tx", "ty", "w", "kappa")}
    for k in range(m):
        nk = int(counts[k])
        th = 2.0 * math.pi * np.arange(nk) / nk
        c, s = np.cos(th), np.sin(th)
        r = radius[k]
        parts["x"].append(cx[k] + r * c)
        parts["y"].append(cy[k] + r * s)
        parts["nx"].append(-c)
        parts["ny"].append(-s)
        parts["tx"].append(-s)
        parts["ty"].append(c)
        parts["w"].append(np.full(nk, 2.0 * math.pi * r / nk))
        parts["kappa"].append(np.full(nk, 1.0 / r))
    wall = rounded_rectangle(length, n_ext, delta)
    for key in parts:
        parts[key].append(wall[key])
    arrs = {k: np.ascontiguousarray(np.concatenate(v)) for k, v in parts.items()}
    off = np.zeros(m + 2, dtype=np.int64)
    off[1:m + 1] = np.cumsum(counts)
    off[m + 1] = off[m] + n_ext
    return Geometry(cx=cx, cy=cy, radius=radius, curve_off=off,
                    length=float(length), n_int=int(n_int), n_ext=int(n_ext),
                    **arrs)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

CONFIGS = {
    # plain method, tiny: 512 wall nodes + 10 pores x 64 nodes
    "tiny": dict(length=4.0, n_ext=512, n_pores=10, r_lo=0.05, r_hi=0.1,
                 n_int=64, gap_pore=0.05, gap_wall=0.1),
    # IFMM FP64 case: 4096 wall nodes + 200 pores x 128 nodes
    "pipe200": dict(length=20.0, n_ext=4096, n_pores=200, r_lo=0.02,
                    r_hi=0.05, n_int=128, gap_pore=0.005, gap_wall=0.05),
    # headline case: 4096 wall nodes + 1000 pores x 64 nodes (n = 139,192)
    "pipe1000": dict(length=50.0, n_ext=4096, n_pores=1000, r_lo=0.02,
                     r_hi=0.05, n_int=64, gap_pore=0.005, gap_wall=0.1),
}


def make_geometry(name_or_cfg, seed: int, **overrides) -> Geometry:
    """Seeded geometry for a named workload (or an explicit parameter dict)."""
    cfg = dict(CONFIGS[name_or_cfg]) if isinstance(name_or_cfg, str) else dict(name_or_cfg)
    cfg.update(overrides)
    rng = np.random.default_rng(seed)
    cx, cy, rr = place_pores(rng, cfg["n_pores"], cfg["length"], cfg["r_lo"],
                             cfg["r_hi"], cfg["gap_pore"], cfg["gap_wall"])
    return build_geometry(cfg["length"], cfg["n_ext"], cx, cy, rr, cfg["n_int"],
                          delta=cfg.get("delta", 0.1))


def batch_member(seed: int) -> Geometry:
    """One geometry of the uneven batch: M ~ U{10..400}, pipe length
    max(4, M/20), 64 or 128 nodes per pore (64 when the unknown count would
    exceed about 60k)."""
    rng = np.random.default_rng(seed)
    m = int(rng.integers(10, 401))
    length = max(4.0, m / 20.0)
    n_ext = max(512, 64 * int(math.ceil(204.8 * length / 64.0)))
    n_int = int(rng.choice([64, 128]))
    if 2 * (m * n_int + n_ext) + 3 * m > 60_000:
        n_int = 64
    cx, cy, rr = place_pores(rng, m, length, 0.02, 0.05, 0.005,
                             max(0.05, 4.0 * length * 2.0 / n_ext))
    return build_geometry(length, n_ext, cx, cy, rr, n_int)
