"""Oracle solvers: dense LU, the block-diagonal preconditioner and flexible
right-preconditioned GMRES.

TEST INFRASTRUCTURE ONLY (tests, the entry-point smoke check and the CPU
baseline leg of the benchmark).  Plain FP64 NumPy/SciPy.

* ``lu_solve``: the plain definition sigma* = A^{-1} F (LAPACK getrf/getrs).
* ``BlockDiagonal``: the comparison preconditioner of Section 4.1.1: one block
  per pore (its nodes and its three completion unknowns) and one for the wall,
  each assembled, factorised and applied exactly.
* ``fgmres``: Saad's flexible GMRES with right preconditioning, classical
  Gram-Schmidt applied twice, Givens rotations, and a convergence test on the
  true residual relative to ||F|| (the paper's runs use left preconditioning
  and a preconditioned residual, Section 4; the reading taken here tests the
  true residual so that an inexact preconditioner cannot hide it).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import dlp


def lu_solve(a: np.ndarray, f: np.ndarray) -> np.ndarray:
    lu, piv = sla.lu_factor(a)
    return sla.lu_solve((lu, piv), f)


def bd_block_indices(geom):
    """Unknown indices of each diagonal block: pores 1..M, then the wall."""
    nn = geom.n_nodes
    blocks = []
    for k in range(geom.n_pores):
        sl = geom.pore_slice(k)
        js = np.arange(sl.start, sl.stop)
        blocks.append(np.concatenate([js, nn + js, 2 * nn + 3 * k + np.arange(3)]))
    ws = geom.wall_slice
    js = np.arange(ws.start, ws.stop)
    blocks.append(np.concatenate([js, nn + js]))
    return blocks


class BlockDiagonal:
    """Exact inverse of the block diagonal of A (pores and wall blocks)."""

    def __init__(self, geom, a: np.ndarray | None = None):
        self.blocks = bd_block_indices(geom)
        self.factors = []
        for idx in self.blocks:
            blk = a[np.ix_(idx, idx)] if a is not None else dlp.block(geom, idx, idx)
            self.factors.append(sla.lu_factor(blk))

    def __call__(self, v: np.ndarray) -> np.ndarray:
        z = np.zeros_like(v)
        for idx, fac in zip(self.blocks, self.factors):
            z[idx] = sla.lu_solve(fac, v[idx])
        return z


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    rel_res_true: float
    converged: bool
    history: list


def fgmres(matvec, f: np.ndarray, precond=None, x0=None, tol: float = 1e-10,
           max_iter: int = 2000, restart: int | None = None, residual=None,
           log=None) -> GmresResult:
    """Flexible GMRES (right preconditioning), CGS2 Arnoldi.

    Stops when the (recurrence) residual falls to tol * ||F||, then checks the
    true residual and restarts from the current iterate if it is still above
    the tolerance and iterations remain.  ``residual(x)``, if given, computes
    the true residual F - A x (for instance in extended precision); otherwise
    it is F - matvec(x).  ``log(iters, estimate)`` is called after each step.
    """
    n = f.shape[0]
    restart = max_iter if restart is None else restart
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fnorm = np.linalg.norm(f)
    if fnorm == 0.0:
        return GmresResult(np.zeros(n), 0, 0.0, True, [0.0])
    hist = []
    total = 0
    while True:
        r = residual(x) if residual is not None else f - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / fnorm)
        if beta <= tol * fnorm or total >= max_iter:
            return GmresResult(x, total, beta / fnorm, beta <= tol * fnorm, hist)
        m = min(restart, max_iter - total)
        v = np.zeros((m + 1, n))
        z = np.zeros((m, n))
        h = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        v[0] = r / beta
        k_used = 0
        for j in range(m):
            z[j] = v[j] if precond is None else precond(v[j])
            w = matvec(z[j])
            hj = v[:j + 1] @ w
            w = w - hj @ v[:j + 1]
            hj2 = v[:j + 1] @ w
            w = w - hj2 @ v[:j + 1]
            h[:j + 1, j] = hj + hj2
            h[j + 1, j] = np.linalg.norm(w)
            breakdown = h[j + 1, j] == 0.0
            if not breakdown:
                v[j + 1] = w / h[j + 1, j]
            for i in range(j):
                t = cs[i] * h[i, j] + sn[i] * h[i + 1, j]
                h[i + 1, j] = -sn[i] * h[i, j] + cs[i] * h[i + 1, j]
                h[i, j] = t
            den = np.hypot(h[j, j], h[j + 1, j])
            cs[j] = h[j, j] / den
            sn[j] = h[j + 1, j] / den
            h[j, j] = den
            h[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k_used = j + 1
            hist.append(abs(g[j + 1]) / fnorm)
            if log is not None:
                log(total, hist[-1])
            if abs(g[j + 1]) <= tol * fnorm or breakdown or total >= max_iter:
                break
        y = sla.solve_triangular(h[:k_used, :k_used], g[:k_used])
        x = x + y @ z[:k_used]
