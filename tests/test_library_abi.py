"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these run without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokes_ifmm.h")
LIB = os.path.join(ROOT, "paper_1609_04484_amd", "libstokes_ifmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"if", "sizeof"})


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("stokes_bie_assemble", "stokes_dlp_matvec", "ifmm_factor",
                     "ifmm_solve", "gmres_solve", "bd_factor", "bd_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_has_no_undefined_symbols_of_its_own():
    """Every symbol the library references is defined in it or in a library
    it links (checked with immediate binding, as the loader on a GPU host
    would find it)."""
    code = ("import ctypes, os; ctypes.CDLL(%r, mode=os.RTLD_NOW | os.RTLD_GLOBAL); print('ok')" % LIB)
    r = subprocess.run(["python3", "-c", code], capture_output=True, text=True)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr
    out = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    own = [ln.split()[-1] for ln in out.splitlines() if "sbie" in ln]
    assert not own, own


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_every_kernel_launched_from_host_code_has_device_code():
    """Each host-side launch stub names a kernel whose gfx950 code object
    entry (``<name>.kd``) is in the library.  A source edited between the
    device and the host compilation passes breaks this, and such a launch
    aborts the process on the GPU."""
    syms = subprocess.run(["nm", LIB], capture_output=True, text=True, check=True).stdout
    stubs = {ln.split()[-1].split("__device_stub__", 1)[1]
             for ln in syms.splitlines() if "__device_stub__" in ln}
    assert stubs
    strings = subprocess.run(["strings", "-n", "8", LIB], capture_output=True, text=True,
                             check=True).stdout
    kd = [w for w in strings.split() if w.endswith(".kd")]
    missing = sorted(st for st in stubs if not any(st + ".kd" in w for w in kd))
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_matches_header():
    import paper_1609_04484_amd as p
    lib = p.load()
    for name in declared_functions():
        assert hasattr(lib, name)
    from paper_1609_04484_amd import _lib
    assert set(declared_functions()) <= set(_lib.EXPORTS)
    assert lib.sbie_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_errors_without_gpu():
    """Argument validation happens before any device work."""
    import ctypes
    import paper_1609_04484_amd._lib as L
    lib = L.load()
    assert lib.stokes_dlp_matvec(None, None, None, 0, None) == -1
    assert b"null geometry" in lib.sbie_last_error()
    assert lib.stokes_dlp_matvec_set_shape(3, 0) == -1
    assert lib.gmres_solve(None, None, None, None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.bd_factor(None, ctypes.byref(h), None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_uses_no_vendor_math_library():
    """Every kernel of the hot path is the project's own: the library links
    no BLAS/LAPACK/solver library and references none of their symbols."""
    needed = subprocess.run(["readelf", "-d", LIB], capture_output=True, text=True,
                            check=True).stdout
    libs = re.findall(r"Shared library: \[([^\]]+)\]", needed)
    banned = ("rocblas", "hipblas", "rocsolver", "hipsolver", "blaslt", "miopen", "rocfft")
    assert not [n for n in libs if any(b in n.lower() for b in banned)], libs
    undef = subprocess.run(["nm", "-D", "--undefined-only", LIB], capture_output=True,
                           text=True, check=True).stdout.lower()
    assert not [b for b in banned if b in undef]
