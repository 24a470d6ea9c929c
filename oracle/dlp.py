"""Oracle: the completed double-layer Nystrom matrix, written out entry by entry.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
it is used by the tests, by the entry-point smoke check and by the CPU
baseline leg of the benchmark.  Plain FP64 NumPy, no blocking or fusion beyond
what the definitions below state.

The operator (Section 2.1 gives the double-layer kernel; Section 2.2 the
Nystrom discretisation; the removal of the double layer's null space is
mentioned in Section 2.1 and is realised here by the reading recorded in the
design notes):

Unknowns ``u = [sigma_x (Nn) | sigma_y (Nn) | (lambda_x, lambda_y, mu)_k for
k = 1..M]``.  With r = x_i - x_j, rho = |r|:

node rows (component a):
    (A u)_i = -1/2 sigma_i
            + sum_{j != i} w_j (1/pi) (r . n_j) r r^T / rho^4  sigma_j
            + w_i kappa_i / (2 pi) t_i t_i^T sigma_i          (smooth limit)
            + [i on wall] n_i / |Gamma_0| sum_{j on wall} w_j n_j . sigma_j
            + sum_k [ S(x_i - c_k) lambda_k + r_k R(x_i - c_k) mu_k ]
    S(r) = (1/4pi)(-log rho I + r r^T / rho^2)   (Stokeslet)
    R(r) = (1/4pi) r_perp / rho^2, r_perp = (r_y, -r_x)   (rotlet)

pore rows (pore k with radius r_k and centre c_k):
    lambda row: 1/(2 pi r_k) sum_{j in k} w_j sigma_j - lambda_k
    mu row:     1/(2 pi r_k^2) sum_{j in k} w_j (x_j - c_k)_perp . sigma_j - mu_k
"""
from __future__ import annotations

import math

import numpy as np


def _row_info(geom, rows):
    """Split global row (or column) indices into node/component/pore parts."""
    nn = geom.n_nodes
    rows = np.asarray(rows, dtype=np.int64)
    is_node = rows < 2 * nn
    node = np.where(rows < nn, rows, rows - nn)
    comp = np.where(rows < nn, 0, 1)
    pk = (rows - 2 * nn) // 3
    pc = (rows - 2 * nn) % 3
    return is_node, node, comp, pk, pc


def wall_mask(geom) -> np.ndarray:
    m = np.zeros(geom.n_nodes, dtype=bool)
    m[geom.wall_slice] = True
    return m


def node_curve(geom) -> np.ndarray:
    """Curve index of every node: 0..M-1 for pores, M for the wall."""
    cid = np.empty(geom.n_nodes, dtype=np.int64)
    for k in range(geom.n_pores + 1):
        cid[geom.curve_off[k]:geom.curve_off[k + 1]] = k
    return cid


def rows_of_matrix(geom, rows) -> np.ndarray:
    """Rows ``rows`` of the completed double-layer matrix, shape (len(rows), n)."""
    nn = geom.n_nodes
    m = geom.n_pores
    n = geom.n_unknowns
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], n))
    is_node, node, comp, pk, pc = _row_info(geom, rows)
    wmask = wall_mask(geom)
    wall_len = geom.w[wmask].sum()
    cid = node_curve(geom)

    # ---------------- node rows ----------------
    ridx = np.nonzero(is_node)[0]
    if ridx.size:
        i = node[ridx]
        a = comp[ridx]
        xi = geom.x[i][:, None]
        yi = geom.y[i][:, None]
        rx = xi - geom.x[None, :]
        ry = yi - geom.y[None, :]
        rho2 = rx * rx + ry * ry
        self_pair = rho2 == 0.0
        rho2s = np.where(self_pair, 1.0, rho2)
        rn = rx * geom.nx[None, :] + ry * geom.ny[None, :]
        base = (geom.w[None, :] / math.pi) * rn / (rho2s * rho2s)
        base = np.where(self_pair, 0.0, base)
        ra = np.where(a[:, None] == 0, rx, ry)
        # D_ab = base * r_a * r_b
        out[ridx, :nn] = base * ra * rx
        out[ridx, nn:2 * nn] = base * ra * ry
        # jump and smooth diagonal limit
        ti = np.where(a == 0, geom.tx[i], geom.ty[i])
        dcoef = geom.w[i] * geom.kappa[i] / (2.0 * math.pi)
        out[ridx, i] += dcoef * ti * geom.tx[i]
        out[ridx, nn + i] += dcoef * ti * geom.ty[i]
        out[ridx, a * nn + i] += -0.5
        # rank-one wall term n_i (w_j n_j)^T / |Gamma_0|
        on_wall = wmask[i]
        if on_wall.any():
            wr = ridx[on_wall]
            nia = np.where(a[on_wall] == 0, geom.nx[i[on_wall]], geom.ny[i[on_wall]])
            wj = np.where(wmask, geom.w, 0.0)
            out[wr, :nn] += (nia[:, None] / wall_len) * (wj * geom.nx)[None, :]
            out[wr, nn:2 * nn] += (nia[:, None] / wall_len) * (wj * geom.ny)[None, :]
        # Stokeslet and rotlet completion columns
        if m:
            cx = geom.cx[None, :]
            cy = geom.cy[None, :]
            sx = geom.x[i][:, None] - cx
            sy = geom.y[i][:, None] - cy
            s2 = sx * sx + sy * sy
            lg = 0.5 * np.log(s2)
            sa = np.where(a[:, None] == 0, sx, sy)
            inv4pi = 1.0 / (4.0 * math.pi)
            col = 2 * nn + 3 * np.arange(m)
            delta_ax = (a[:, None] == 0).astype(float)
            delta_ay = 1.0 - delta_ax
            out[ridx[:, None], col[None, :]] = inv4pi * (-lg * delta_ax + sa * sx / s2)
            out[ridx[:, None], col[None, :] + 1] = inv4pi * (-lg * delta_ay + sa * sy / s2)
            # r_perp = (r_y, -r_x)
            perp_a = np.where(a[:, None] == 0, sy, -sx)
            out[ridx[:, None], col[None, :] + 2] = inv4pi * geom.radius[None, :] * perp_a / s2

    # ---------------- pore constraint rows ----------------
    cidx = np.nonzero(~is_node)[0]
    for rr in cidx:
        k = int(pk[rr])
        c = int(pc[rr])
        sl = geom.pore_slice(k)
        rk = geom.radius[k]
        js = np.arange(sl.start, sl.stop)
        if c < 2:
            out[rr, c * nn + js] = geom.w[js] / (2.0 * math.pi * rk)
        else:
            px = geom.x[js] - geom.cx[k]
            py = geom.y[js] - geom.cy[k]
            # (x_j - c_k)_perp = (p_y, -p_x)
            out[rr, js] = geom.w[js] * py / (2.0 * math.pi * rk * rk)
            out[rr, nn + js] = -geom.w[js] * px / (2.0 * math.pi * rk * rk)
        out[rr, 2 * nn + 3 * k + c] = -1.0
    return out


def assemble(geom, chunk: int = 2048) -> np.ndarray:
    """The full dense matrix A (n x n), FP64."""
    n = geom.n_unknowns
    a = np.empty((n, n))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a[s:e] = rows_of_matrix(geom, np.arange(s, e))
    return a


def block(geom, rows, cols, chunk: int = 256) -> np.ndarray:
    """A[rows, cols], computed from whole rows ``chunk`` rows at a time."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty((rows.shape[0], cols.shape[0]))
    for s in range(0, rows.shape[0], chunk):
        out[s:s + chunk] = rows_of_matrix(geom, rows[s:s + chunk])[:, cols]
    return out


def apply(geom, u: np.ndarray, chunk: int = 1024) -> np.ndarray:
    """A @ u by rows (O(n^2) work, O(chunk * n) memory)."""
    n = geom.n_unknowns
    out = np.empty(n)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = rows_of_matrix(geom, np.arange(s, e)) @ u
    return out


def apply_rows(geom, u: np.ndarray, rows) -> np.ndarray:
    """(A @ u)[rows] for a sample of rows."""
    return rows_of_matrix(geom, rows) @ u


def dlp_only_rows(geom, u: np.ndarray, rows) -> np.ndarray:
    """Principal-value double-layer sum with its smooth diagonal limit,
    sum_{j != i} w_j D(x_i, x_j, n_j) sigma_j + w_i kappa_i/(2pi) t t^T sigma_i,
    for node rows only (no jump, no wall term, no completion)."""
    nn = geom.n_nodes
    rows = np.asarray(rows, dtype=np.int64)
    assert (rows < 2 * nn).all()
    i = np.where(rows < nn, rows, rows - nn)
    a = np.where(rows < nn, 0, 1)
    rx = geom.x[i][:, None] - geom.x[None, :]
    ry = geom.y[i][:, None] - geom.y[None, :]
    rho2 = rx * rx + ry * ry
    self_pair = rho2 == 0.0
    rho2s = np.where(self_pair, 1.0, rho2)
    rn = rx * geom.nx[None, :] + ry * geom.ny[None, :]
    base = np.where(self_pair, 0.0, (geom.w[None, :] / math.pi) * rn / (rho2s * rho2s))
    ra = np.where(a[:, None] == 0, rx, ry)
    sx, sy = u[:nn], u[nn:2 * nn]
    val = (base * ra * (rx * sx[None, :] + ry * sy[None, :])).sum(axis=1)
    ti = np.where(a == 0, geom.tx[i], geom.ty[i])
    val += geom.w[i] * geom.kappa[i] / (2.0 * math.pi) * ti * (geom.tx[i] * sx[i] + geom.ty[i] * sy[i])
    return val


def velocity(geom, u: np.ndarray, px, py) -> tuple:
    """Velocity in the fluid from a solved density (no jump, no wall term):
    u(p) = sum_j w_j D(p, x_j, n_j) sigma_j + sum_k [S(p - c_k) lambda_k
    + r_k R(p - c_k) mu_k]; the trapezoid rule of Section 2.2."""
    nn = geom.n_nodes
    px = np.atleast_1d(np.asarray(px, dtype=np.float64))
    py = np.atleast_1d(np.asarray(py, dtype=np.float64))
    rx = px[:, None] - geom.x[None, :]
    ry = py[:, None] - geom.y[None, :]
    rho2 = rx * rx + ry * ry
    rn = rx * geom.nx[None, :] + ry * geom.ny[None, :]
    sx, sy = u[:nn], u[nn:2 * nn]
    rs = rx * sx[None, :] + ry * sy[None, :]
    coef = (geom.w[None, :] / math.pi) * rn * rs / (rho2 * rho2)
    ux = (coef * rx).sum(axis=1)
    uy = (coef * ry).sum(axis=1)
    m = geom.n_pores
    if m:
        lam = u[2 * nn:].reshape(m, 3)
        qx = px[:, None] - geom.cx[None, :]
        qy = py[:, None] - geom.cy[None, :]
        q2 = qx * qx + qy * qy
        lg = 0.5 * np.log(q2)
        inv4pi = 1.0 / (4.0 * math.pi)
        dot = (qx * lam[None, :, 0] + qy * lam[None, :, 1]) / q2
        ux += inv4pi * (-lg * lam[None, :, 0] + qx * dot).sum(axis=1)
        uy += inv4pi * (-lg * lam[None, :, 1] + qy * dot).sum(axis=1)
        rot = inv4pi * geom.radius[None, :] * lam[None, :, 2] / q2
        ux += (rot * qy).sum(axis=1)
        uy += (-rot * qx).sum(axis=1)
    return ux, uy
