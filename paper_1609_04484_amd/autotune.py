"""Autotuning of launch shapes and IFMM accuracy, cached as JSON.

Two choices are tuned per size class (node count rounded up to a power of
two) and per precision:

* the pair kernel's launch shape, targets per thread x source chunks, timed
  with the kernel's own HIP events (``stokes_dlp_matvec_set_shape``; the
  shape is process-wide and also used by the batched matvec);
* the IFMM accuracy (eps, Chebyshev order), chosen by the measured time of a
  whole solve (factor + FGMRES to the tolerance) on a representative
  geometry: a looser eps factors faster but costs iterations.

The cache is a JSON file (``$SBIE_AUTOTUNE_CACHE``, else
``~/.cache/paper_1609_04484_amd/autotune.json``) keyed by device name, size
class and precision; a cached entry is used without re-measuring.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import _lib as L

TPT = (1, 2, 4, 8)
CHUNKS = (0, 32, 64, 128, 256)          # 0 = the library's own choice
IFMM_CANDIDATES = ((1e-3, 6), (1e-4, 8), (1e-6, 10))
DEFAULT_SHAPE = (4, 0)


def default_cache_path() -> str:
    env = os.environ.get("SBIE_AUTOTUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1609_04484_amd", "autotune.json")


def size_class(n_nodes: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(1, n_nodes))))


def _device() -> str:
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


class Autotuner:
    def __init__(self, path: str | None = None):
        self.path = path or default_cache_path()
        self.table = {}
        if os.path.exists(self.path):
            with open(self.path) as fh:
                self.table = json.load(fh)

    def _key(self, kind, n_nodes, precision=0):
        return f"{_device()}|{kind}|nn{size_class(n_nodes)}|p{precision}"

    def save(self):
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    # ---------------- pair-kernel launch shape ----------------
    def matvec_shape(self, dg, reps=5, candidates=None, force=False):
        """Best (targets_per_thread, source_chunks) for this size class."""
        key = self._key("matvec", dg.geom.n_nodes)
        if key in self.table and not force:
            e = self.table[key]
            return (e["tpt"], e["chunks"])
        cands = candidates or [(t, c) for t in TPT for c in CHUNKS]
        x = torch.randn(dg.n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        best, timings = None, {}
        try:
            for tpt, ch in cands:
                L.set_matvec_shape(tpt, ch)
                L.matvec(dg, x, out=y)             # warm
                torch.cuda.synchronize()
                L.kernel_timing(True)
                L.kernel_time()
                for _ in range(reps):
                    L.matvec(dg, x, out=y)
                torch.cuda.synchronize()
                L.kernel_timing(False)
                ms, cnt = L.kernel_time()
                t = ms / max(cnt, 1)
                timings[f"{tpt}x{ch}"] = t
                if best is None or t < best[0]:
                    best = (t, tpt, ch)
        finally:
            L.kernel_timing(False)
            L.set_matvec_shape(*DEFAULT_SHAPE)
        self.table[key] = dict(tpt=best[1], chunks=best[2], ms=best[0], timings=timings)
        self.save()
        return (best[1], best[2])

    def apply_matvec_shape(self, dg, **kw):
        shape = self.matvec_shape(dg, **kw)
        L.set_matvec_shape(*shape)
        return shape

    # ---------------- IFMM accuracy ----------------
    def ifmm_params(self, dg, f, precision=0, tol=1e-10, candidates=IFMM_CANDIDATES,
                    force=False):
        """Best (eps, cheb_n) by the time of a whole solve on this geometry."""
        key = self._key("ifmm", dg.geom.n_nodes, precision)
        if key in self.table and not force:
            e = self.table[key]
            return (e["eps"], e["cheb_n"])
        best, timings = None, {}
        for eps, cn in candidates:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = L.IFMM(dg, eps=eps, cheb_n=cn, precision=precision)
            r = L.gmres(dg, f, pc=pc, tol=tol)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            pc.close()
            ok = r.status == 0
            timings[f"{eps:g}/{cn}"] = dict(s=t, iters=r.iters, converged=ok)
            if ok and (best is None or t < best[0]):
                best = (t, eps, cn)
        if best is None:
            raise RuntimeError("no IFMM candidate converged")
        self.table[key] = dict(eps=best[1], cheb_n=best[2], s=best[0], timings=timings)
        self.save()
        return (best[1], best[2])
