"""ctypes binding of libstokes_ifmm.so (argument marshalling only).

Every computation happens in the HIP library; this module moves the seeded
geometry to device memory with PyTorch, passes raw device pointers and the
current HIP stream, and turns status codes into exceptions.  There is no CPU
fallback: if the library is missing or no GPU is present, calls fail.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstokes_ifmm.so")

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_dp = ctypes.c_void_p


class SbieGeom(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("n_pores", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("curve_off", _c_i64p),
        ("curve_off_dev", ctypes.c_void_p),
        ("x", _c_dp), ("y", _c_dp),
        ("nx", _c_dp), ("ny", _c_dp),
        ("w", _c_dp), ("kappa", _c_dp),
        ("cx", _c_dp), ("cy", _c_dp),
        ("radius", _c_dp),
    ]


class IfmmParams(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("cheb_n", ctypes.c_int32),
        ("leaf_target", ctypes.c_int32),
        ("max_depth", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("compress", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


COMPRESS = {"working": 0, "fp16": 1, "bf16": 2}


def _compress(c):
    return COMPRESS[c] if isinstance(c, str) else int(c)


class IfmmStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("leaves", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("factor_bytes", ctypes.c_int64),
        ("factor_seconds", ctypes.c_double),
        ("gemm_flops", ctypes.c_double),
        ("inverse_flops", ctypes.c_double),
        ("gemm_low_flops", ctypes.c_double),
    ]


class GmresParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("pc", ctypes.c_int32),
        ("use_x0", ctypes.c_int32),
        ("bd", ctypes.c_void_p),
        ("ifmm", ctypes.c_void_p),
        ("res_hist", ctypes.POINTER(ctypes.c_double)),
        ("fmm", ctypes.c_void_p),
    ]


class FmmParams(ctypes.Structure):
    _fields_ = [
        ("cheb_n", ctypes.c_int32),
        ("leaf_target", ctypes.c_int32),
        ("max_depth", ctypes.c_int32),
        ("adaptive", ctypes.c_int32),
    ]


class FmmStats(ctypes.Structure):
    _fields_ = [
        ("depth", ctypes.c_int32),
        ("leaves", ctypes.c_int32),
        ("boxes", ctypes.c_int32),
        ("min_leaf_level", ctypes.c_int32),
        ("m2l_box_pairs", ctypes.c_int64),
        ("near_node_pairs", ctypes.c_int64),
        ("m2p_box_pairs", ctypes.c_int64),
        ("p2l_box_pairs", ctypes.c_int64),
    ]


class GmresResult(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("rel_res_true", ctypes.c_double),
        ("rel_res_pc", ctypes.c_double),
        ("t_precond_s", ctypes.c_double),
        ("t_matvec_s", ctypes.c_double),
        ("t_arnoldi_s", ctypes.c_double),
        ("t_total_s", ctypes.c_double),
    ]


class GmresMember(ctypes.Structure):
    _fields_ = [
        ("pc", ctypes.c_int32),
        ("use_x0", ctypes.c_int32),
        ("bd", ctypes.c_void_p),
        ("ifmm", ctypes.c_void_p),
    ]


EXPORTS = {
    "sbie_last_error": (ctypes.c_char_p, []),
    "sbie_validate_geometry": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp]),
    "stokes_bie_assemble": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, ctypes.c_int64,
                                           _c_dp, ctypes.c_int64, _c_dp, ctypes.c_int64, _c_dp]),
    "stokes_dlp_matvec": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, ctypes.c_int, _c_dp]),
    "stokes_dlp_matvec_noalloc": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, ctypes.c_int,
                                                 _c_dp]),
    "stokes_velocity": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, _c_dp, ctypes.c_int64,
                                       _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]),
    "stokes_slp_weights": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double)]),
    "stokes_slp_matvec": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, ctypes.c_int, _c_dp]),
    "stokes_slp_assemble": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, ctypes.c_int64,
                                           _c_dp, ctypes.c_int64, _c_dp, ctypes.c_int64, _c_dp]),
    "bd_factor_slp": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.POINTER(ctypes.c_void_p), _c_dp]),
    "gmres_solve_slp": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp,
                                       ctypes.POINTER(GmresParams), ctypes.POINTER(GmresResult), _c_dp]),
    "stokes_slp_velocity": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, _c_dp, ctypes.c_int64,
                                           _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]),
    "fmm_plan": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.POINTER(FmmParams),
                                ctypes.POINTER(ctypes.c_void_p), _c_dp]),
    "stokes_dlp_matvec_fmm": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, ctypes.c_int, _c_dp]),
    "fmm_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(FmmStats)]),
    "fmm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "stokes_dlp_matvec_set_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "stokes_dlp_matvec_batched_set_schedule": (ctypes.c_int, [ctypes.c_int]),
    "stokes_dlp_matvec_set_symmetric": (ctypes.c_int, [ctypes.c_int]),
    "stokes_dlp_matvec_describe_plan": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_int,
                                                       ctypes.POINTER(ctypes.c_int32),
                                                       ctypes.POINTER(ctypes.c_int32),
                                                       ctypes.POINTER(ctypes.c_int32)]),
    "sbie_kernel_timing": (ctypes.c_int, [ctypes.c_int]),
    "sbie_kernel_time": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "bd_factor": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.POINTER(ctypes.c_void_p), _c_dp]),
    "bd_solve": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, _c_dp]),
    "bd_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ifmm_factor": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.POINTER(IfmmParams),
                                   ctypes.POINTER(ctypes.c_void_p), _c_dp]),
    "ifmm_solve": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, _c_dp]),
    "ifmm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ifmm_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(IfmmStats)]),
    "gmres_solve": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp,
                                   ctypes.POINTER(GmresParams), ctypes.POINTER(GmresResult), _c_dp]),
    "stokes_dlp_matvec_batched": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_void_p),
                                                 ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, _c_dp]),
    "gmres_solve_batched": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(GmresMember), ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(GmresResult), _c_dp]),
    "ifmm_factor_batched": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_int32,
                                           ctypes.POINTER(IfmmParams),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
    "mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64,
                                  ctypes.POINTER(ctypes.c_void_p), _c_dp]),
    "mlp_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "mlp_num_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp]),
    "mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp]),
    "mlp_forward": (ctypes.c_int, [ctypes.c_void_p, _c_dp, ctypes.c_int32, _c_dp, _c_dp]),
    "mlp_loss_grad": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, ctypes.c_int32, _c_dp,
                                     ctypes.POINTER(ctypes.c_double), _c_dp]),
    "warmstart_refine": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_void_p, _c_dp, _c_dp,
                                        ctypes.POINTER(ctypes.c_double), _c_dp]),
    "mlp_set_scaling": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]),
    "mlp_get_scaling": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp]),
    "mlp_fit_scaling": (ctypes.c_int, [ctypes.c_void_p, _c_dp, _c_dp, ctypes.c_int32, _c_dp]),
    "mlp_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, _c_dp]),
    "warmstart_features": (ctypes.c_int, [ctypes.POINTER(SbieGeom), ctypes.c_double, ctypes.c_double,
                                          _c_dp, _c_dp]),
    "warmstart_labels": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, _c_dp]),
    "warmstart_assemble": (ctypes.c_int, [ctypes.POINTER(SbieGeom), _c_dp, _c_dp, _c_dp, _c_dp]),
}

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARGUMENT", -2: "INVALID_GEOMETRY",
          -3: "OUT_OF_MEMORY", -4: "HIP_ERROR", -5: "BREAKDOWN", -6: "UNSUPPORTED"}

_lib = None


class SbieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1609_04484_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int) -> int:
    if code < 0:
        raise SbieError(code, load().sbie_last_error().decode())
    return code


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: torch.Tensor) -> int:
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


class DeviceGeometry:
    """A geometry resident in device memory plus its C descriptor."""

    def __init__(self, geom, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the HIP library needs an MI355X")
        self.geom = geom
        dev = torch.device(device)
        to = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
        self.t = {k: to(getattr(geom, k)) for k in ("x", "y", "nx", "ny", "w", "kappa")}
        m = geom.n_pores
        pore = lambda a: to(a) if m else torch.zeros(1, dtype=torch.float64, device=dev)
        self.t["cx"] = pore(geom.cx)
        self.t["cy"] = pore(geom.cy)
        self.t["radius"] = pore(geom.radius)
        self.off_host = np.ascontiguousarray(geom.curve_off, dtype=np.int64)
        self.off_dev = torch.as_tensor(self.off_host).to(dev)
        self.n = geom.n_unknowns
        self.c = SbieGeom(
            n_nodes=geom.n_nodes, n_pores=m, reserved=0,
            curve_off=self.off_host.ctypes.data_as(_c_i64p),
            curve_off_dev=self.off_dev.data_ptr(),
            **{k: v.data_ptr() for k, v in self.t.items()},
        )

    def vector(self, a) -> torch.Tensor:
        return torch.as_tensor(np.asarray(a, dtype=np.float64)).to(self.t["x"].device).contiguous()


def validate(dg: DeviceGeometry, stream=None):
    """Device-side geometry checks; raises SbieError(INVALID_GEOMETRY)."""
    check(load().sbie_validate_geometry(ctypes.byref(dg.c), _stream(stream)))


def matvec(dg: DeviceGeometry, x: torch.Tensor, mode: int = 0, out=None, stream=None):
    y = torch.empty_like(x) if out is None else out
    check(load().stokes_dlp_matvec(ctypes.byref(dg.c), _ptr(x), _ptr(y), mode, _stream(stream)))
    return y


def matvec_noalloc(dg: DeviceGeometry, x: torch.Tensor, out: torch.Tensor, mode: int = 0, stream=None):
    """y = A x through the entry point that allocates nothing (the output
    must be passed in)."""
    check(load().stokes_dlp_matvec_noalloc(ctypes.byref(dg.c), _ptr(x), _ptr(out), mode,
                                           _stream(stream)))
    return out


def velocity(dg: DeviceGeometry, sigma: torch.Tensor, px: torch.Tensor, py: torch.Tensor,
             uref=None, stream=None):
    """(ux, uy) at the points (px, py); with uref = (ux_ref, uy_ref) also the
    relative velocity-magnitude error per point: returns (ux, uy, err)."""
    npts = px.numel()
    ux = torch.empty_like(px)
    uy = torch.empty_like(px)
    err = torch.empty_like(px) if uref is not None else None
    rx, ry = (uref if uref is not None else (None, None))
    check(load().stokes_velocity(ctypes.byref(dg.c), _ptr(sigma), _ptr(px), _ptr(py), npts,
                                 _ptr(ux), _ptr(uy), _ptr(rx) if rx is not None else None,
                                 _ptr(ry) if ry is not None else None,
                                 _ptr(err) if err is not None else None, _stream(stream)))
    return (ux, uy, err) if uref is not None else (ux, uy)


def set_matvec_shape(targets_per_thread: int, source_chunks: int = 0):
    check(load().stokes_dlp_matvec_set_shape(targets_per_thread, source_chunks))


def set_matvec_symmetric(mode: int):
    """Symmetric pair evaluation of the plain products: 0 never, 1 where it
    pays (the default), 2 always (up to 131,072 nodes)."""
    check(load().stokes_dlp_matvec_set_symmetric(int(mode)))


def matvec_plan(dg: DeviceGeometry, mode: int = 0) -> dict:
    """The launch plan of stokes_dlp_matvec for this geometry and mode."""
    sym, ch, tpt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(load().stokes_dlp_matvec_describe_plan(ctypes.byref(dg.c), mode, ctypes.byref(sym),
                                                 ctypes.byref(ch), ctypes.byref(tpt)))
    return {"symmetric": bool(sym.value), "chunks": ch.value, "targets_per_thread": tpt.value}


def set_batched_schedule(persistent: bool):
    """Pair stage of the batched products: persistent work-queue grid (True,
    the default) or one workgroup per item (False)."""
    check(load().stokes_dlp_matvec_batched_set_schedule(int(persistent)))


def kernel_timing(enable: bool):
    """Start or stop event bracketing of the matvec's pair kernel."""
    check(load().sbie_kernel_timing(int(enable)))


def kernel_time():
    """(total milliseconds, launches) of the pair kernel since the last call."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    check(load().sbie_kernel_time(ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def assemble(dg: DeviceGeometry, rows, cols, stream=None) -> torch.Tensor:
    dev = dg.t["x"].device
    r = torch.as_tensor(np.asarray(rows, dtype=np.int64)).to(dev)
    c = torch.as_tensor(np.asarray(cols, dtype=np.int64)).to(dev)
    out = torch.empty((c.numel(), r.numel()), dtype=torch.float64, device=dev)
    check(load().stokes_bie_assemble(ctypes.byref(dg.c), _ptr(r), r.numel(), _ptr(c),
                                     c.numel(), _ptr(out), r.numel(), _stream(stream)))
    return out.t()  # column-major storage -> (nr, nc) view


class BlockDiagonal:
    """Block-diagonal preconditioner of the completed double layer, or of
    the single layer with single_layer=True."""

    def __init__(self, dg: DeviceGeometry, stream=None, single_layer=False):
        self.dg = dg
        self.single_layer = single_layer
        h = ctypes.c_void_p()
        fn = load().bd_factor_slp if single_layer else load().bd_factor
        check(fn(ctypes.byref(dg.c), ctypes.byref(h), _stream(stream)))
        self.h = h

    def solve(self, b: torch.Tensor, stream=None) -> torch.Tensor:
        x = torch.empty_like(b)
        check(load().bd_solve(self.h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def close(self):
        if self.h:
            load().bd_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IFMM:
    def __init__(self, dg: DeviceGeometry, eps=1e-6, cheb_n=10, leaf_target=64,
                 max_depth=0, precision=0, compress=0, stream=None, handle=None):
        """compress: inputs of the recompression's Gaussian sketches, 0 or
        "working" (the factor's precision), 1 or "fp16", 2 or "bf16"."""
        self.dg = dg
        if handle is not None:          # adopt a handle made by ifmm_factor_batched
            self.h = handle
            return
        p = IfmmParams(eps=eps, cheb_n=cheb_n, leaf_target=leaf_target,
                       max_depth=max_depth, precision=precision, compress=_compress(compress))
        h = ctypes.c_void_p()
        check(load().ifmm_factor(ctypes.byref(dg.c), ctypes.byref(p), ctypes.byref(h),
                                 _stream(stream)))
        self.h = h

    def solve(self, b: torch.Tensor, stream=None) -> torch.Tensor:
        x = torch.empty_like(b)
        check(load().ifmm_solve(self.h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def stats(self) -> dict:
        s = IfmmStats()
        check(load().ifmm_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in IfmmStats._fields_ if k != "reserved"}

    def close(self):
        if self.h:
            load().ifmm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class SolveResult:
    sigma: torch.Tensor
    iters: int
    status: int
    rel_res_true: float
    rel_res_pc: float
    t_precond_s: float
    t_matvec_s: float
    t_arnoldi_s: float
    t_total_s: float
    history: np.ndarray


def gmres(dg: DeviceGeometry, f: torch.Tensor, pc=None, tol=1e-10, max_iter=2000,
          restart=0, x0: torch.Tensor | None = None, stream=None, fmm=None) -> SolveResult:
    """FGMRES solve of A sigma = f; pc is None, a BlockDiagonal or an IFMM;
    fmm (an FMM plan of dg) evaluates the Arnoldi products."""
    sigma = torch.zeros_like(f) if x0 is None else x0.clone()
    hist = np.zeros(max_iter + 2)
    kind = 0 if pc is None else (1 if isinstance(pc, BlockDiagonal) else 2)
    p = GmresParams(tol=tol, max_iter=max_iter, restart=restart, pc=kind,
                    use_x0=int(x0 is not None),
                    bd=pc.h.value if kind == 1 else None,
                    ifmm=pc.h.value if kind == 2 else None,
                    res_hist=hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    fmm=fmm.h.value if fmm is not None else None)
    r = GmresResult()
    check(load().gmres_solve(ctypes.byref(dg.c), _ptr(f), _ptr(sigma), ctypes.byref(p),
                             ctypes.byref(r), _stream(stream)))
    return SolveResult(sigma, r.iters, r.status, r.rel_res_true, r.rel_res_pc, r.t_precond_s,
                       r.t_matvec_s, r.t_arnoldi_s, r.t_total_s, hist[:r.iters + 1].copy())


class FMM:
    """Fast-multipole plan of a geometry (Chebyshev interpolation on a
    uniform quadtree) for the double-layer pair sum."""

    def __init__(self, dg: DeviceGeometry, cheb_n=12, leaf_target=64, max_depth=0, adaptive=False,
                 stream=None):
        self.dg = dg
        p = FmmParams(cheb_n=cheb_n, leaf_target=leaf_target, max_depth=max_depth,
                      adaptive=int(adaptive))
        h = ctypes.c_void_p()
        check(load().fmm_plan(ctypes.byref(dg.c), ctypes.byref(p), ctypes.byref(h), _stream(stream)))
        self.h = h

    def matvec(self, x: torch.Tensor, mode: int = 0, out=None, stream=None) -> torch.Tensor:
        y = torch.empty_like(x) if out is None else out
        check(load().stokes_dlp_matvec_fmm(self.h, _ptr(x), _ptr(y), mode, _stream(stream)))
        return y

    def stats(self) -> dict:
        s = FmmStats()
        check(load().fmm_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in FmmStats._fields_}

    def close(self):
        if self.h:
            load().fmm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def slp_weights() -> np.ndarray:
    """The six correction weights of the single-layer quadrature."""
    g = (ctypes.c_double * 6)()
    check(load().stokes_slp_weights(g))
    return np.array(list(g))


def slp_matvec(dg: DeviceGeometry, x: torch.Tensor, accurate=False, out=None, stream=None):
    """y = A x for the single-layer matrix (2 Nn unknowns)."""
    y = torch.empty_like(x) if out is None else out
    check(load().stokes_slp_matvec(ctypes.byref(dg.c), _ptr(x), _ptr(y), 2 if accurate else 0,
                                   _stream(stream)))
    return y


def slp_assemble(dg: DeviceGeometry, rows, cols, stream=None) -> torch.Tensor:
    dev = dg.t["x"].device
    r = torch.as_tensor(np.asarray(rows, dtype=np.int64)).to(dev)
    c = torch.as_tensor(np.asarray(cols, dtype=np.int64)).to(dev)
    out = torch.empty((c.numel(), r.numel()), dtype=torch.float64, device=dev)
    check(load().stokes_slp_assemble(ctypes.byref(dg.c), _ptr(r), r.numel(), _ptr(c), c.numel(),
                                     _ptr(out), r.numel(), _stream(stream)))
    return out.t()


def gmres_slp(dg: DeviceGeometry, f: torch.Tensor, pc=None, tol=1e-10, max_iter=2000,
              restart=0, x0: torch.Tensor | None = None, stream=None, fmm=None) -> SolveResult:
    """FGMRES on the single-layer system; pc is None or a single-layer
    BlockDiagonal (an FMM plan is refused: it evaluates the double layer)."""
    sigma = torch.zeros_like(f) if x0 is None else x0.clone()
    hist = np.zeros(max_iter + 2)
    kind = 0 if pc is None else 1
    p = GmresParams(tol=tol, max_iter=max_iter, restart=restart, pc=kind,
                    use_x0=int(x0 is not None), bd=pc.h.value if kind == 1 else None, ifmm=None,
                    res_hist=hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    fmm=fmm.h.value if fmm is not None else None)
    r = GmresResult()
    check(load().gmres_solve_slp(ctypes.byref(dg.c), _ptr(f), _ptr(sigma), ctypes.byref(p),
                                 ctypes.byref(r), _stream(stream)))
    return SolveResult(sigma, r.iters, r.status, r.rel_res_true, r.rel_res_pc, r.t_precond_s,
                       r.t_matvec_s, r.t_arnoldi_s, r.t_total_s, hist[:r.iters + 1].copy())


def slp_velocity(dg: DeviceGeometry, sigma: torch.Tensor, px: torch.Tensor, py: torch.Tensor,
                 uref=None, stream=None):
    """Velocity from a single-layer density at (px, py); as velocity()."""
    npts = px.numel()
    ux = torch.empty_like(px)
    uy = torch.empty_like(px)
    err = torch.empty_like(px) if uref is not None else None
    rx, ry = (uref if uref is not None else (None, None))
    check(load().stokes_slp_velocity(ctypes.byref(dg.c), _ptr(sigma), _ptr(px), _ptr(py), npts,
                                     _ptr(ux), _ptr(uy), _ptr(rx) if rx is not None else None,
                                     _ptr(ry) if ry is not None else None,
                                     _ptr(err) if err is not None else None, _stream(stream)))
    return (ux, uy, err) if uref is not None else (ux, uy)


class MLP:
    """The warm-start network (device parameters, hand-written kernels)."""

    def __init__(self, widths=(64, 256, 256, 256, 64), seed=0, stream=None):
        self.widths = list(widths)
        w = (ctypes.c_int32 * len(widths))(*widths)
        h = ctypes.c_void_p()
        check(load().mlp_create(len(widths) - 1, w, seed, ctypes.byref(h), _stream(stream)))
        self.h = h
        n = ctypes.c_int64()
        check(load().mlp_num_params(self.h, ctypes.byref(n)))
        self.n_params = n.value

    def params(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(load().mlp_get_params(self.h, _ptr(out), _stream(stream)))
        return out

    def set_params(self, p: torch.Tensor, stream=None):
        p = p.to(device="cuda", dtype=torch.float32).contiguous()
        check(load().mlp_set_params(self.h, _ptr(p), _stream(stream)))

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        """X: (batch, in) float32 row-major == (in x batch) column-major."""
        X = X.contiguous()
        Y = torch.empty((X.shape[0], self.widths[-1]), dtype=torch.float32, device=X.device)
        check(load().mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(Y), _stream(stream)))
        return Y

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor, want_grad=False, stream=None):
        X, T = X.contiguous(), T.contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device) if want_grad else None
        loss = ctypes.c_double()
        check(load().mlp_loss_grad(self.h, _ptr(X), _ptr(T), X.shape[0],
                                   _ptr(g) if g is not None else None, ctypes.byref(loss),
                                   _stream(stream)))
        return loss.value, g

    def scaling(self, stream=None):
        """(in_mean, in_scale, out_mean, out_std) as device tensors."""
        a = [torch.empty(w, dtype=torch.float32, device="cuda")
             for w in (self.widths[0], self.widths[0], self.widths[-1], self.widths[-1])]
        check(load().mlp_get_scaling(self.h, *[_ptr(t) for t in a], _stream(stream)))
        return tuple(a)

    def set_scaling(self, in_mean, in_scale, out_mean, out_std, stream=None):
        a = [t.to(device="cuda", dtype=torch.float32).contiguous()
             for t in (in_mean, in_scale, out_mean, out_std)]
        check(load().mlp_set_scaling(self.h, *[_ptr(t) for t in a], _stream(stream)))

    def fit_scaling(self, X: torch.Tensor, T: torch.Tensor, stream=None):
        X, T = X.contiguous(), T.contiguous()
        check(load().mlp_fit_scaling(self.h, _ptr(X), _ptr(T), X.shape[0], _stream(stream)))

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(load().mlp_adam_step(self.h, lr, beta1, beta2, eps, _stream(stream)))

    def close(self):
        if self.h:
            load().mlp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def warmstart_features(dg: DeviceGeometry, y_lo=0.0, y_hi=1.0, stream=None) -> torch.Tensor:
    m = dg.geom.n_pores
    out = torch.zeros((max(m, 1), 64), dtype=torch.float32, device="cuda")
    check(load().warmstart_features(ctypes.byref(dg.c), y_lo, y_hi, _ptr(out), _stream(stream)))
    return out[:m]


def warmstart_labels(dg: DeviceGeometry, sigma: torch.Tensor, stream=None) -> torch.Tensor:
    m = dg.geom.n_pores
    out = torch.zeros((max(m, 1), 64), dtype=torch.float32, device="cuda")
    check(load().warmstart_labels(ctypes.byref(dg.c), _ptr(sigma), _ptr(out), _stream(stream)))
    return out[:m]


def warmstart_assemble(dg: DeviceGeometry, coeffs: torch.Tensor, wall_sigma=None,
                       stream=None) -> torch.Tensor:
    x0 = torch.empty(dg.n, dtype=torch.float64, device="cuda")
    c = coeffs.contiguous() if coeffs.numel() else torch.zeros(64, dtype=torch.float32, device="cuda")
    check(load().warmstart_assemble(ctypes.byref(dg.c), _ptr(c),
                                    _ptr(wall_sigma) if wall_sigma is not None else None,
                                    _ptr(x0), _stream(stream)))
    return x0


def warmstart_refine(dg: DeviceGeometry, wall_bd, f: torch.Tensor, x0: torch.Tensor,
                     stream=None) -> float:
    """Wall solve and minimal-residual scaling of x0 in place; returns alpha."""
    alpha = ctypes.c_double()
    check(load().warmstart_refine(ctypes.byref(dg.c), wall_bd.h, _ptr(f), _ptr(x0),
                                  ctypes.byref(alpha), _stream(stream)))
    return alpha.value


def _geom_array(dgs):
    arr = (SbieGeom * len(dgs))()
    for i, dg in enumerate(dgs):
        arr[i] = dg.c
    return arr


def matvec_batched(dgs, xs, mode: int = 0, stream=None):
    """y_b = A_b x_b for every member, one launch per stage for the batch."""
    ys = [torch.empty_like(x) for x in xs]
    xp = (ctypes.c_void_p * len(xs))(*[_ptr(x) for x in xs])
    yp = (ctypes.c_void_p * len(ys))(*[_ptr(y) for y in ys])
    check(load().stokes_dlp_matvec_batched(_geom_array(dgs), len(dgs), xp, yp, mode,
                                           _stream(stream)))
    return ys


def ifmm_factor_batched(dgs, eps=1e-6, cheb_n=10, leaf_target=64, max_depth=0, precision=0,
                        workers=4, compress=0):
    """IFMM factorisations of every member, several in flight at once."""
    p = IfmmParams(eps=eps, cheb_n=cheb_n, leaf_target=leaf_target, max_depth=max_depth,
                   precision=precision, compress=_compress(compress))
    hs = (ctypes.c_void_p * len(dgs))()
    torch.cuda.synchronize()
    check(load().ifmm_factor_batched(_geom_array(dgs), len(dgs), ctypes.byref(p), hs, workers))
    return [IFMM(dg, handle=ctypes.c_void_p(h)) for dg, h in zip(dgs, hs)]


def gmres_batched(dgs, fs, pcs=None, tol=1e-10, max_iter=2000, restart=0, x0s=None,
                  stream=None):
    """Lockstep FGMRES over the batch; pcs[b] is None, a BlockDiagonal or an IFMM."""
    nb = len(dgs)
    pcs = pcs if pcs is not None else [None] * nb
    sig = [torch.zeros_like(f) if (x0s is None or x0s[b] is None) else x0s[b].clone()
           for b, f in enumerate(fs)]
    mem = (GmresMember * nb)()
    for b, pc in enumerate(pcs):
        kind = 0 if pc is None else (1 if isinstance(pc, BlockDiagonal) else 2)
        mem[b] = GmresMember(pc=kind, use_x0=int(x0s is not None and x0s[b] is not None),
                             bd=pc.h.value if kind == 1 else None,
                             ifmm=pc.h.value if kind == 2 else None)
    res = (GmresResult * nb)()
    fp = (ctypes.c_void_p * nb)(*[_ptr(f) for f in fs])
    sp = (ctypes.c_void_p * nb)(*[_ptr(x) for x in sig])
    check(load().gmres_solve_batched(_geom_array(dgs), nb, fp, sp, mem, tol, max_iter, restart,
                                     res, _stream(stream)))
    return [SolveResult(sig[b], r.iters, r.status, r.rel_res_true, r.rel_res_pc, r.t_precond_s,
                        r.t_matvec_s, r.t_arnoldi_s, r.t_total_s, np.zeros(0))
            for b, r in enumerate(res)]
