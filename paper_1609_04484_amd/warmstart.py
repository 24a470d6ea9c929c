"""Learned warm start for the FGMRES solve.

A per-pore network (64 geometry features -> 64 Fourier coefficients of the
density on the pore, see ``csrc/mlp.hip``) gives an initial guess x0: the
predicted series on every pore and lambda, mu from the completion's
constraint functionals; the wall density then comes from one exact solve of
the wall rows (the wall block is factored once per pipe), and x0 is scaled to
minimise the residual along it, so it is never worse than the zero start.
FGMRES still solves to the same true-residual tolerance; its convergence
test is relative to ||F||, so a good x0 saves iterations.

Everything numerical runs in the HIP library: the solver that generates the
training labels, the feature and label kernels, the forward/backward passes
and Adam.  This module only orchestrates (geometry generation on the host,
shuffling indices, bookkeeping) and offers a command-line A/B run:

    python -m paper_1609_04484_amd.warmstart --train 200 --test 5
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib as L

WIDTHS = (64, 256, 256, 256, 64)

# geometry families (pipe [0, L] x [0, 1]); "pipe200" is the 200-pore,
# 128-nodes-per-pore pipe of length 20
FAMILIES = {
    "pipe200": dict(length=20.0, n_ext=4096, n_pores=200, r_lo=0.02, r_hi=0.05,
                    n_int=128, gap_pore=0.005, gap_wall=0.05),
    "small": dict(length=4.0, n_ext=512, n_pores=30, r_lo=0.03, r_hi=0.06,
                  n_int=64, gap_pore=0.02, gap_wall=0.08),
}


def _make_pc(dg, pc, eps):
    if pc == "bd":
        return L.BlockDiagonal(dg)
    if pc == "ifmm":
        return L.IFMM(dg, eps=eps, cheb_n=8)
    return None


def pore_free(length, n_ext, delta=0.1):
    """The same pipe without pores (device geometry)."""
    from stokes_inputs import build_geometry
    return L.DeviceGeometry(build_geometry(length, n_ext, [], [], [], 64, delta=delta))


def generate(family, seeds, pc="ifmm", eps=1e-4, tol=1e-10, log=None):
    """Solve one seeded geometry per seed; return the features X (S x 64) and
    Fourier labels T (S x 64) of all pores (device FP32) and solve records."""
    from stokes_inputs import make_geometry, poiseuille_rhs
    cfg = FAMILIES[family] if isinstance(family, str) else family
    xs, ts, recs = [], [], []
    for s in seeds:
        g = make_geometry(cfg, int(s))
        dg = L.DeviceGeometry(g)
        r = L.gmres(dg, dg.vector(poiseuille_rhs(g)), pc=_make_pc(dg, pc, eps), tol=tol)
        if r.status != 0:
            raise RuntimeError(f"training solve for seed {s} did not converge")
        xs.append(L.warmstart_features(dg))
        ts.append(L.warmstart_labels(dg, r.sigma))
        recs.append(dict(seed=int(s), iters=r.iters, t=r.t_total_s))
        if log:
            log(f"[warmstart] data seed {s}: {r.iters} iters {r.t_total_s:.2f}s")
    return torch.cat(xs), torch.cat(ts), recs


def train(net, X, T, epochs=20, batch=4096, lr=1e-3, seed=0, log=None):
    """Adam on the standardised MSE; minibatches from a seeded permutation.
    Returns the mean loss of every epoch."""
    net.fit_scaling(X, T)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    hist = []
    s = X.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(s, device=X.device, generator=gen)
        tot, cnt = 0.0, 0
        for b0 in range(0, s, batch):
            idx = perm[b0:b0 + batch]
            loss, _ = net.loss_grad(X.index_select(0, idx), T.index_select(0, idx))
            net.adam_step(lr=lr)
            tot += loss * idx.shape[0]
            cnt += idx.shape[0]
        hist.append(tot / cnt)
        if log:
            log(f"[warmstart] epoch {ep}: loss {hist[-1]:.4e}")
    return hist


class WarmStart:
    """A trained network plus, per pipe, the inverse of the wall block (the
    block-diagonal preconditioner of the pipe without pores: A_ww depends on
    the wall alone, so it is factored once per pipe)."""

    def __init__(self, net=None, seed=0):
        self.net = net if net is not None else L.MLP(WIDTHS, seed=seed)
        self._walls = {}

    def wall_block(self, geom):
        key = (geom.length, geom.n_ext)
        if key not in self._walls:
            dg0 = pore_free(geom.length, geom.n_ext)
            self._walls[key] = (dg0, L.BlockDiagonal(dg0))
        return self._walls[key][1]

    def initial_guess(self, dg, f):
        """x0 from the network on every pore, then the exact wall solve and
        the minimal-residual scaling (``warmstart_refine``)."""
        g = dg.geom
        coef = (self.net.forward(L.warmstart_features(dg)) if g.n_pores
                else torch.zeros(0, device="cuda"))
        x0 = L.warmstart_assemble(dg, coef, None)
        self.last_alpha = L.warmstart_refine(dg, self.wall_block(g), f, x0)
        return x0


def ab_test(ws, family, seeds, pc="ifmm", eps=1e-4, tol=1e-10, log=None):
    """Solve each held-out geometry from zero and from the learned x0."""
    from stokes_inputs import make_geometry, poiseuille_rhs
    cfg = FAMILIES[family] if isinstance(family, str) else family
    out = []
    for s in seeds:
        g = make_geometry(cfg, int(s))
        dg = L.DeviceGeometry(g)
        f = dg.vector(poiseuille_rhs(g))
        fn = float(torch.linalg.vector_norm(f))
        ws.wall_block(g)                     # factored once per pipe, not timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cold = L.gmres(dg, f, pc=_make_pc(dg, pc, eps), tol=tol)
        torch.cuda.synchronize()
        t_cold = time.perf_counter() - t0
        t0 = time.perf_counter()
        x0 = ws.initial_guess(dg, f)
        warm = L.gmres(dg, f, pc=_make_pc(dg, pc, eps), tol=tol, x0=x0)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        r0 = f - L.matvec(dg, x0)
        rec = dict(seed=int(s), iters_cold=cold.iters, iters_warm=warm.iters, alpha=ws.last_alpha,
                   s_cold=t_cold, s_warm=t_warm,
                   rel_res0_warm=float(torch.linalg.vector_norm(r0)) / fn,
                   rel_res_true_cold=cold.rel_res_true, rel_res_true_warm=warm.rel_res_true,
                   density_rel_diff=float(torch.linalg.vector_norm(warm.sigma - cold.sigma)
                                          / torch.linalg.vector_norm(cold.sigma)))
        out.append(rec)
        if log:
            log(f"[warmstart] A/B seed {s}: {rec}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="pipe200", choices=sorted(FAMILIES))
    ap.add_argument("--train", type=int, default=200, help="training geometries")
    ap.add_argument("--test", type=int, default=5, help="held-out geometries")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pc", default="ifmm", choices=["ifmm", "bd", "none"])
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    # training seeds 10000.., held-out evaluation seeds 20000.. (the
    # warm-start workload's split)
    X, T, recs = generate(a.family, range(10000 + a.seed, 10000 + a.seed + a.train), a.pc, a.eps,
                          a.tol, log)
    t_data = time.perf_counter() - t0
    ws = WarmStart(seed=a.seed)
    t0 = time.perf_counter()
    hist = train(ws.net, X, T, a.epochs, a.batch, a.lr, a.seed, log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ab = ab_test(ws, a.family, range(20000 + a.seed, 20000 + a.seed + a.test), a.pc, a.eps,
                 a.tol, log)
    cold = np.mean([r["iters_cold"] for r in ab])
    warm = np.mean([r["iters_warm"] for r in ab])
    print(json.dumps(dict(family=a.family, train_geometries=a.train, samples=int(X.shape[0]),
                          epochs=a.epochs, loss_first=hist[0], loss_last=hist[-1],
                          t_data_s=t_data, t_train_s=t_train, pc=a.pc,
                          iters_cold=cold, iters_warm=warm,
                          solves_per_s_cold=len(ab) / sum(r["s_cold"] for r in ab),
                          solves_per_s_warm=len(ab) / sum(r["s_warm"] for r in ab),
                          ab=ab)), flush=True)


if __name__ == "__main__":
    main()
