#!/usr/bin/env python3
"""Write the stored reference solutions sigma* = A^{-1} F of the large
workloads, using the CPU oracle only (``oracle/`` and the seeded inputs).

    python tests/golden/make_sigma.py pipe200    # n = 59,992: dense LU
    python tests/golden/make_sigma.py pipe1000   # n = 139,192: oracle FGMRES
    python tests/golden/make_sigma.py batch      # batch members with n <= 20,000: dense LU
    python tests/golden/make_sigma.py refine pipe1000 300   # continue from a stored solution

* pipe200 (seed 100, Poiseuille data): the completed double-layer matrix is
  assembled densely by the NumPy oracle (28.8 GB), factorised by LAPACK
  (getrf, partial pivoting, in place) and solved; then two steps of iterative
  refinement with residuals F - A sigma evaluated in 80-bit arithmetic by the
  C oracle.
* pipe1000 (seed 300, Poiseuille data): a dense LU would need 155 GB, so the
  oracle's flexible GMRES is run with the oracle's block-diagonal
  preconditioner (Section 4's comparison preconditioner) and the C oracle's
  double-precision operator in the Arnoldi steps; every true residual is
  evaluated in 80-bit arithmetic, and the run stops at a true relative
  residual of 1e-13 (a restart from the current iterate is one step of
  iterative refinement).

* batch members (seeds 1000-1063 of the batched workload, Poiseuille data):
  those with at most 20,000 unknowns, by the dense LU of pipe200.
* refine: the same FGMRES started from a stored solution (one more round of
  restarts, i.e. iterative refinement with 80-bit residuals); of every
  iterate whose true residual is evaluated the best one is kept.

Each run writes ``sigma_<workload>_s<seed>.npy`` (FP64, no pickle) and a
JSON record with the method, the final residual (80-bit evaluation), the
iteration count, the wall-clock time and the host it ran on.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import capply, dlp, solve  # noqa: E402
from stokes_inputs import batch_member, make_geometry, poiseuille_rhs  # noqa: E402

SEEDS = {"pipe200": 100, "pipe1000": 300}


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def true_residual(g, f, x):
    return f - capply.apply(g, x, extended=True)


def dense_lu(g, f):
    n = g.n_unknowns
    t0 = time.perf_counter()
    a = dlp.assemble(g)
    log(f"assembled {n}x{n} in {time.perf_counter() - t0:.0f}s")
    import scipy.linalg as sla
    t1 = time.perf_counter()
    # a is C-ordered, so a.T is the Fortran-ordered A^T: factor it in place
    # and solve with the transpose flag (A x = F)
    lu, piv = sla.lu_factor(a.T, overwrite_a=True, check_finite=False)
    log(f"LU in {time.perf_counter() - t1:.0f}s")
    x = sla.lu_solve((lu, piv), f, trans=1, check_finite=False)
    hist = []
    for step in range(2):
        r = true_residual(g, f, x)
        hist.append(float(np.linalg.norm(r) / np.linalg.norm(f)))
        log(f"refinement {step}: rel residual {hist[-1]:.3e}")
        x = x + sla.lu_solve((lu, piv), r, trans=1, check_finite=False)
    r = true_residual(g, f, x)
    hist.append(float(np.linalg.norm(r) / np.linalg.norm(f)))
    log(f"final rel residual {hist[-1]:.3e}")
    return x, dict(method="dense LU (LAPACK getrf/getrs) + 2 steps of iterative refinement "
                          "with 80-bit residuals", residual_history=hist, iters=0)


def fgmres_bd(g, f, tol=1e-13, max_iter=3000):
    t0 = time.perf_counter()
    bd = solve.BlockDiagonal(g)
    log(f"block-diagonal factor in {time.perf_counter() - t0:.0f}s")

    def mv(v):
        return capply.apply(g, v)

    last = [time.perf_counter()]

    def progress(it, est):
        if it % 25 == 0:
            now = time.perf_counter()
            log(f"iter {it}: estimate {est:.3e} ({(now - last[0]) / 25:.2f}s/iter)")
            last[0] = now

    res = solve.fgmres(mv, f, precond=bd, tol=tol, max_iter=max_iter,
                       residual=lambda x: true_residual(g, f, x), log=progress)
    log(f"FGMRES: {res.iters} iterations, true rel residual {res.rel_res_true:.3e}, "
        f"converged {res.converged}")
    return res.x, dict(method="flexible GMRES (CGS2, unrestarted) with the block-diagonal "
                              "preconditioner; double-precision Arnoldi operator, 80-bit "
                              "true residuals",
                       residual_history=[float(h) for h in res.history if h is not None][-5:],
                       iters=int(res.iters), converged=bool(res.converged),
                       rel_res_true=float(res.rel_res_true), tol=tol)


BATCH_SEEDS = range(1000, 1064)      # the 64 members of the batched workload
BATCH_MAX_N = 20000                   # members solved by dense LU here


def refine(work, seed, tol=1e-13, max_iter=600):
    g = make_geometry(work, seed)
    f = poiseuille_rhs(g)
    base = os.path.join(HERE, f"sigma_{work}_s{seed}")
    x0 = np.load(base + ".npy", allow_pickle=False)
    with open(base + ".json") as fh:
        meta = json.load(fh)
    fn = np.linalg.norm(f)
    r0 = float(np.linalg.norm(true_residual(g, f, x0)) / fn)
    log(f"{work} seed {seed}: refining from true rel residual {r0:.3e}")
    best = [r0, x0.copy()]

    def resid(x):
        r = true_residual(g, f, x)
        rr = float(np.linalg.norm(r) / fn)
        if rr < best[0]:
            best[0], best[1] = rr, x.copy()
        return r

    t0 = time.perf_counter()
    bd = solve.BlockDiagonal(g)
    log(f"block-diagonal factor in {time.perf_counter() - t0:.0f}s")
    last = [time.perf_counter()]

    def progress(it, est):
        if it % 25 == 0:
            now = time.perf_counter()
            log(f"iter {it}: estimate {est:.3e} ({(now - last[0]) / 25:.2f}s/iter)")
            last[0] = now

    res = solve.fgmres(lambda v: capply.apply(g, v), f, precond=bd, x0=x0, tol=tol, max_iter=max_iter,
                       residual=resid, log=progress)
    x = best[1]
    r = true_residual(g, f, x)
    meta.update(method=meta["method"] + "; then refined: the same FGMRES from the stored solution, "
                "keeping the iterate of smallest 80-bit true residual",
                refine_iters=int(res.iters), refine_start_residual=r0,
                final_rel_residual_80bit=float(np.linalg.norm(r) / fn),
                wall_s=meta.get("wall_s", 0.0) + time.perf_counter() - t0)
    np.save(base + ".npy", x)
    with open(base + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"wrote {base}.npy: final rel residual {meta['final_rel_residual_80bit']:.3e}")


def main():
    work = sys.argv[1] if len(sys.argv) > 1 else "pipe200"
    if work == "refine":
        refine(sys.argv[2], int(sys.argv[3]))
        return
    if work == "batch":
        # every member of the batched workload small enough for a dense LU
        for sd in BATCH_SEEDS:
            if batch_member(sd).n_unknowns <= BATCH_MAX_N:
                solve_one("member", sd)
        return
    seed = int(sys.argv[2]) if len(sys.argv) > 2 else SEEDS[work]
    solve_one(work, seed)


def solve_one(work, seed):
    g = batch_member(seed) if work == "member" else make_geometry(work, seed)
    f = poiseuille_rhs(g)
    log(f"{work} seed {seed}: Nn={g.n_nodes} n={g.n_unknowns}")
    t0 = time.perf_counter()
    x, meta = dense_lu(g, f) if work in ("pipe200", "member") else fgmres_bd(g, f)
    wall = time.perf_counter() - t0
    r = true_residual(g, f, x)
    meta.update(workload=work, seed=seed, n=int(g.n_unknowns), rhs="poiseuille k=4",
                final_rel_residual_80bit=float(np.linalg.norm(r) / np.linalg.norm(f)),
                sigma_norm_over_f_norm=float(np.linalg.norm(x) / np.linalg.norm(f)),
                wall_s=wall, host_cpu=cpu_model(), host_cores=os.cpu_count())
    base = os.path.join(HERE, f"sigma_{work}_s{seed}")
    np.save(base + ".npy", x)
    with open(base + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    log(f"wrote {base}.npy ({meta})")


if __name__ == "__main__":
    main()
