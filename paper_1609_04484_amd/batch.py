"""Solve a batch of independent pipes: sequentially, one geometry after the
other, and batched (concurrent IFMM factorisations plus lockstep FGMRES with
one launch per matvec stage for the whole batch).

    python -m paper_1609_04484_amd.batch --members 64 --eps 1e-4 --cheb-n 8

Members follow the uneven batch recipe of ``stokes_inputs.batch_member``
(10-400 pores, pipe length max(4, M/20), 64 or 128 nodes per pore), each with
Poiseuille inflow.  Prints one JSON line with both solves/s figures.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib as L


def make_batch(members, seed):
    from stokes_inputs import batch_member, poiseuille_rhs
    geoms = [batch_member(seed + b) for b in range(members)]
    dgs = [L.DeviceGeometry(g) for g in geoms]
    fs = [dg.vector(poiseuille_rhs(g)) for dg, g in zip(dgs, geoms)]
    return geoms, dgs, fs


def run_sequential(dgs, fs, eps, cheb_n, precision, tol, restart):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = []
    for dg, f in zip(dgs, fs):
        pc = L.IFMM(dg, eps=eps, cheb_n=cheb_n, precision=precision)
        out.append(L.gmres(dg, f, pc=pc, tol=tol, restart=restart))
        pc.close()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def run_batched(dgs, fs, eps, cheb_n, precision, tol, restart, workers):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pcs = L.ifmm_factor_batched(dgs, eps=eps, cheb_n=cheb_n, precision=precision, workers=workers)
    t1 = time.perf_counter()
    out = L.gmres_batched(dgs, fs, pcs, tol=tol, restart=restart)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for p in pcs:
        p.close()
    return out, t2 - t0, t1 - t0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--cheb-n", type=int, default=8)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--autotune", default=None, help="JSON cache path: tune the matvec shape")
    ap.add_argument("--schedule", default="queue", choices=["queue", "grid"],
                    help="pair stage of the batched products: persistent work-queue grid or "
                         "one workgroup per item")
    a = ap.parse_args(argv)
    L.set_batched_schedule(a.schedule == "queue")
    log = lambda m: print(m, file=sys.stderr, flush=True)
    geoms, dgs, fs = make_batch(a.members, a.seed)
    ns = [g.n_unknowns for g in geoms]
    log(f"[batch] {a.members} members, n from {min(ns)} to {max(ns)} (total {sum(ns)})")
    shape = None
    if a.autotune:
        from .autotune import Autotuner
        big = max(range(len(dgs)), key=lambda b: ns[b])
        shape = Autotuner(a.autotune).apply_matvec_shape(dgs[big])
        log(f"[batch] matvec shape {shape}")
    # warm-up on the first member (library load, graph capture paths)
    run_sequential(dgs[:1], fs[:1], a.eps, a.cheb_n, a.precision, a.tol, a.restart)
    seq, t_seq = run_sequential(dgs, fs, a.eps, a.cheb_n, a.precision, a.tol, a.restart)
    log(f"[batch] sequential: {t_seq:.2f}s")
    bat, t_bat, t_fac = run_batched(dgs, fs, a.eps, a.cheb_n, a.precision, a.tol, a.restart,
                                    a.workers)
    log(f"[batch] batched: {t_bat:.2f}s (factor {t_fac:.2f}s)")
    diff = max(float(torch.linalg.vector_norm(b.sigma - s.sigma) / torch.linalg.vector_norm(s.sigma))
               for s, b in zip(seq, bat))
    print(json.dumps(dict(
        members=a.members, n_min=min(ns), n_max=max(ns), n_total=sum(ns),
        eps=a.eps, cheb_n=a.cheb_n, precision=a.precision, tol=a.tol, workers=a.workers,
        schedule=a.schedule,
        matvec_shape=shape,
        sequential_s=t_seq, batched_s=t_bat, batched_factor_s=t_fac,
        solves_per_s_sequential=a.members / t_seq, solves_per_s_batched=a.members / t_bat,
        speedup=t_seq / t_bat,
        iters_sequential=[r.iters for r in seq], iters_batched=[r.iters for r in bat],
        converged_sequential=all(r.status == 0 for r in seq),
        converged_batched=all(r.status == 0 for r in bat),
        max_rel_res_true_batched=max(r.rel_res_true for r in bat),
        max_solution_rel_diff=diff)), flush=True)


if __name__ == "__main__":
    main()
