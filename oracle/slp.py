"""Oracle: the single-layer (first-kind) formulation of Section 2 with the
sixth-order corrected trapezoid rule of Section 2.2, in plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (tests and the CPU-baseline leg of the benchmark).

Section 2.1 represents the velocity by the single layer
    u(x) = S[sigma](x) = 1/(4 pi) int_Gamma ( -log rho I + r r^T / rho^2 ) sigma ds,
and its boundary limit gives the first-kind equation f = S[sigma] on Gamma
(equation "stokesBIE").  Section 2.2 collocates at the nodes and integrates
the logarithmic singularity with the corrected trapezoid rule of Kapur and
Rokhlin: the plain rule with the singular node left out and the weights of
the six nodes on either side of it (same curve) multiplied by (1 + gamma_k).
The smooth part r r^T / rho^2 is corrected by the same weights (one rule for
the whole integrand).  After the solve, the velocity in the fluid is the
plain trapezoid rule (equation "stokesSLP_discretized").

The correction weights are not printed in the paper; they are derived here
from the error expansion of the punctured trapezoid rule for
f(t) = phi(t) log|t - t_i| + psi(t) (phi, psi smooth, periodic setting,
step h):

    int f - h sum_{j != i} f(t_j) = h phi(t_i) log(h / 2 pi) + h psi(t_i)
                                   + 2 sum_{p >= 1} zeta'(-2p) h^{2p+1} phi^{(2p)}(t_i) / (2p)!

(the generalised Euler-Maclaurin expansion; the h log h term is checked
against the exact punctured sum of log|2 sin(t/2)| in the tests).  With
symmetric weights gamma_{+-k}, k = 1..m, and f(t_{i+k}) = phi (log|k| +
log h) + psi, the corrections reproduce the right-hand side up to
O(h^{2P+3} log h) when
    2 sum_k gamma_k k^{2p}       = [p == 0],          p = 0..P
    2 sum_k gamma_k k^{2p} log k = -log(2 pi) (p = 0), 2 zeta'(-2p) (p >= 1),
which for m = 6 nodes per side (P = 2) is a 6 x 6 linear system.  zeta'(-2p)
follows from the functional equation: zeta'(-2p) = (-1)^p (2p)! zeta(2p+1)
/ (2 (2 pi)^{2p}).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import zeta


def zeta_prime_neg_even(p: int) -> float:
    """zeta'(-2p) for p >= 1 from the functional equation."""
    return (-1) ** p * math.factorial(2 * p) * zeta(2 * p + 1) / (2.0 * (2 * math.pi) ** (2 * p))


def kr_log_weights(m: int = 6) -> np.ndarray:
    """Correction weights gamma_1..gamma_m (m even) of the corrected
    trapezoid rule for a logarithmic singularity at a node.  The moment
    system is solved in 40-digit arithmetic (mpmath) and rounded once: its
    condition number (2.7e5 for m = 6) would cost five digits in FP64."""
    import mpmath
    assert m % 2 == 0 and m >= 2
    nP = m // 2
    with mpmath.workdps(40):
        rows, rhs = [], []
        for p in range(nP):
            rows.append([2 * mpmath.mpf(k) ** (2 * p) for k in range(1, m + 1)])
            rhs.append(mpmath.mpf(1) if p == 0 else mpmath.mpf(0))
        for p in range(nP):
            rows.append([2 * mpmath.mpf(k) ** (2 * p) * mpmath.log(k) for k in range(1, m + 1)])
            if p == 0:
                rhs.append(-mpmath.log(2 * mpmath.pi))
            else:
                # zeta'(-2p) from the functional equation
                rhs.append(2 * (-1) ** p * mpmath.factorial(2 * p) * mpmath.zeta(2 * p + 1)
                           / (2 * (2 * mpmath.pi) ** (2 * p)))
        sol = mpmath.lu_solve(mpmath.matrix(rows), mpmath.matrix(rhs))
        return np.array([float(sol[i]) for i in range(m)])


def corrected_trapezoid(f_vals: np.ndarray, i: int, h: float, gamma: np.ndarray) -> float:
    """h sum_{j != i} f_j + h sum_{0 < |k| <= m} gamma_|k| f_{i+k} on a
    periodic grid (f_vals[i] is not used)."""
    n = f_vals.shape[0]
    w = np.ones(n)
    w[i] = 0.0
    for k, g in enumerate(gamma, start=1):
        w[(i + k) % n] += g
        w[(i - k) % n] += g
    return h * float(np.dot(w, np.where(np.arange(n) == i, 0.0, f_vals)))


def quadrature_factors(geom, gamma: np.ndarray | None = None):
    """Per ordered node pair on one curve, the factor (1 + gamma_k) of the
    corrected rule: returns (rows, cols, factor) for every pair at periodic
    index distance 1..m on the same curve (the diagonal is left out)."""
    gamma = kr_log_weights() if gamma is None else gamma
    m = gamma.shape[0]
    ri, ci, fv = [], [], []
    for k in range(geom.n_pores + 1):
        a, b = int(geom.curve_off[k]), int(geom.curve_off[k + 1])
        n = b - a
        if n == 0:
            continue
        assert n > 2 * m, "a curve needs more than 2m nodes for the corrected rule"
        idx = np.arange(n)
        for d in range(1, m + 1):
            for sgn in (1, -1):
                ri.append(a + idx)
                ci.append(a + (idx + sgn * d) % n)
                fv.append(np.full(n, 1.0 + gamma[d - 1]))
    if not ri:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0)
    return np.concatenate(ri), np.concatenate(ci), np.concatenate(fv)


def assemble(geom, gamma: np.ndarray | None = None) -> np.ndarray:
    """The 2Nn x 2Nn matrix of equation "dense_matrix" for the single layer:
    A[(a, i), (b, j)] = w_j (1 + gamma_ij) G_ab(x_i - x_j) / (4 pi), j != i,
    G = -log rho I + r r^T / rho^2, zero diagonal blocks (punctured rule),
    gamma_ij the correction of the pair (zero beyond m nodes or across
    curves).  Unknowns [sigma_x | sigma_y]."""
    nn = geom.n_nodes
    rx = geom.x[:, None] - geom.x[None, :]
    ry = geom.y[:, None] - geom.y[None, :]
    rho2 = rx * rx + ry * ry
    np.fill_diagonal(rho2, 1.0)
    lg = 0.5 * np.log(rho2)
    wt = np.broadcast_to(geom.w[None, :], (nn, nn)).copy()
    ri, ci, fv = quadrature_factors(geom, gamma)
    wt[ri, ci] *= fv
    np.fill_diagonal(wt, 0.0)
    c = wt / (4.0 * math.pi)
    a = np.empty((2 * nn, 2 * nn))
    a[:nn, :nn] = c * (-lg + rx * rx / rho2)
    a[:nn, nn:] = c * (rx * ry / rho2)
    a[nn:, :nn] = c * (rx * ry / rho2)
    a[nn:, nn:] = c * (-lg + ry * ry / rho2)
    return a


def rows_of_matrix(geom, rows, gamma: np.ndarray | None = None) -> np.ndarray:
    """Rows ``rows`` (global indices in [0, 2 Nn)) of the matrix of
    ``assemble``, computed entry by entry from the same definition."""
    gamma = kr_log_weights() if gamma is None else gamma
    m = gamma.shape[0]
    nn = geom.n_nodes
    rows = np.asarray(rows, dtype=np.int64)
    i = np.where(rows < nn, rows, rows - nn)
    a = np.where(rows < nn, 0, 1)
    rx = geom.x[i][:, None] - geom.x[None, :]
    ry = geom.y[i][:, None] - geom.y[None, :]
    rho2 = rx * rx + ry * ry
    self_pair = np.arange(nn)[None, :] == i[:, None]
    rho2 = np.where(self_pair, 1.0, rho2)
    lg = 0.5 * np.log(rho2)
    # correction factor of every (row node, column node) pair
    cid = np.empty(nn, dtype=np.int64)
    for k in range(geom.n_pores + 1):
        cid[geom.curve_off[k]:geom.curve_off[k + 1]] = k
    fac = np.ones((rows.shape[0], nn))
    for r_, ii in enumerate(i):
        k = cid[ii]
        st, en = int(geom.curve_off[k]), int(geom.curve_off[k + 1])
        n = en - st
        for d in range(1, m + 1):
            fac[r_, st + (ii - st + d) % n] += gamma[d - 1]
            fac[r_, st + (ii - st - d) % n] += gamma[d - 1]
    c = np.where(self_pair, 0.0, geom.w[None, :] * fac / (4.0 * math.pi))
    ra = np.where(a[:, None] == 0, rx, ry)
    out = np.empty((rows.shape[0], 2 * nn))
    out[:, :nn] = c * (np.where(a[:, None] == 0, -lg, 0.0) + ra * rx / rho2)
    out[:, nn:] = c * (np.where(a[:, None] == 1, -lg, 0.0) + ra * ry / rho2)
    return out


def velocity(geom, sigma: np.ndarray, px, py) -> tuple:
    """Equation "stokesSLP_discretized": u(p) = 1/(4 pi) sum_j G(p - x_j)
    sigma_j w_j (plain trapezoid rule, p in the fluid)."""
    nn = geom.n_nodes
    px = np.atleast_1d(np.asarray(px, dtype=np.float64))
    py = np.atleast_1d(np.asarray(py, dtype=np.float64))
    rx = px[:, None] - geom.x[None, :]
    ry = py[:, None] - geom.y[None, :]
    rho2 = rx * rx + ry * ry
    lg = 0.5 * np.log(rho2)
    sx, sy = sigma[:nn] * geom.w, sigma[nn:2 * nn] * geom.w
    dot = (rx * sx[None, :] + ry * sy[None, :]) / rho2
    ux = (-lg * sx[None, :] + rx * dot).sum(axis=1) / (4.0 * math.pi)
    uy = (-lg * sy[None, :] + ry * dot).sum(axis=1) / (4.0 * math.pi)
    return ux, uy
