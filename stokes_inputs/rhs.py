"""Boundary data f for the three flows the paper studies, and seeded vectors.

Each right-hand side is returned in the unknown layout shared by every part
of the solver: ``[f_x at nodes | f_y at nodes | 0 for the 3M pore rows]``.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry


def _pack(geom: Geometry, fx: np.ndarray, fy: np.ndarray) -> np.ndarray:
    out = np.zeros(geom.n_unknowns)
    nn = geom.n_nodes
    out[:nn] = fx
    out[nn:2 * nn] = fy
    return out


def poiseuille_rhs(geom: Geometry, k: float = 4.0, half_height: float = 0.5):
    """Pipe flow (Section 2, no-slip pores): on the wall
    f = (k (H^2 - (y - H)^2), 0) for the pipe [0, L] x [0, 2H]; zero on the
    pores.  The paper's [-H, H] is shifted to [0, 2H]; k = 4 gives a peak
    inflow of 1."""
    fx = np.zeros(geom.n_nodes)
    ws = geom.wall_slice
    yw = geom.y[ws] - half_height
    fx[ws] = k * (half_height ** 2 - yw ** 2)
    return _pack(geom, fx, np.zeros(geom.n_nodes))


def shear_rhs(geom: Geometry, y0: float = 0.5):
    """Shear flow u = (y - y0, 0) on every boundary (Section 4.1); the exact
    solution in the fluid is the same linear field."""
    return _pack(geom, geom.y - y0, np.zeros(geom.n_nodes))


def stokeslet_rotlet_data(geom: Geometry, seed: int):
    """Random source points and strengths for the Stokeslet/rotlet boundary
    condition (Section 4.2): c_0 lies outside the wall region (below the
    pipe), c_k inside pore k; lambda_k ~ N(0, I_2), mu_k ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    m = geom.n_pores
    u = rng.uniform(0.0, 1.0, size=m)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=m)
    rad = 0.5 * geom.radius * np.sqrt(u)
    cx = np.concatenate([[0.5 * geom.length], geom.cx + rad * np.cos(ang)])
    cy = np.concatenate([[-0.5], geom.cy + rad * np.sin(ang)])
    lam = rng.standard_normal((m + 1, 2))
    mu = rng.standard_normal(m + 1)
    return dict(cx=cx, cy=cy, lam=lam, mu=mu)


def stokeslet_rotlet_field(data, px: np.ndarray, py: np.ndarray):
    """The Stokeslet/rotlet combination of Section 4.2 evaluated at points
    (px, py), without any 1/(4 pi) factor.  It is the boundary data on the
    curves and the exact velocity inside the fluid."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    ux = np.zeros_like(px)
    uy = np.zeros_like(py)
    for k in range(data["cx"].shape[0]):
        rx = px - data["cx"][k]
        ry = py - data["cy"][k]
        r2 = rx * rx + ry * ry
        lg = 0.5 * np.log(r2)
        lx, ly = data["lam"][k]
        dot = (rx * lx + ry * ly) / r2
        ux += -lg * lx + rx * dot
        uy += -lg * ly + ry * dot
        # (x - c)^perp = (r_y, -r_x)
        ux += data["mu"][k] * ry / r2
        uy += -data["mu"][k] * rx / r2
    return ux, uy


def stokeslet_rotlet_rhs(geom: Geometry, seed: int):
    data = stokeslet_rotlet_data(geom, seed)
    fx, fy = stokeslet_rotlet_field(data, geom.x, geom.y)
    return _pack(geom, fx, fy), data


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 vector (test densities)."""
    return np.random.default_rng(seed).standard_normal(n)
