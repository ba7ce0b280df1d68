"""Oracle projector P_theta (Sec. 2.2, eq. ptheta2 / eq. ptheta1) and transpose.

Test infrastructure only (see ``oracle/__init__``).  Thin ctypes wrapper
around the plain C loops in ``proj.c`` (compiled with gcc on first use, or by
the package build step).

Pins (tests/test_oracle_projector.py): the closed-form line integral of an
isotropic Gaussian (exact at 0 and 90 degrees, second order in the grid step
at oblique angles), the adjoint identity <P rho, g> = <rho, P^T g>, and a
brute-force dense matrix on 8^3 volumes written from the bilinear-weight
formula.
"""
import ctypes
import os
import subprocess
import numpy as np

from .geometry import detector_grid, ray_samples

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "proj.c")
_LIB = os.path.join(_HERE, "_proj.so")
_lib = None


def build(force=False):
    """Compile proj.c with gcc (-O2, IEEE arithmetic, OpenMP over slices)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        ci = ctypes.c_int
        for name in ("oracle_project", "oracle_backproject"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [dp, ci, ci, ci, ci, dp, dp, dp, ci, dp, ci, dp]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tables(g):
    c = np.ascontiguousarray(np.cos(g.theta))
    s = np.ascontiguousarray(np.sin(g.theta))
    return c, s, np.ascontiguousarray(detector_grid(g)), np.ascontiguousarray(ray_samples(g))


def project(g, vol):
    """rho_theta[m, k, p] = sum_q bilerp(vol[k]; u_p c + y_q s, -u_p s + y_q c)."""
    vol = np.ascontiguousarray(vol, dtype=np.float64).reshape(g.nz, g.ny, g.nx)
    c, s, u, y = _tables(g)
    out = np.empty((g.n_angles, g.nz, g.n_u), dtype=np.float64)
    _load().oracle_project(_ptr(vol), g.nx, g.ny, g.nz, g.n_angles, _ptr(c), _ptr(s),
                           _ptr(u), g.n_u, _ptr(y), len(y), _ptr(out))
    return out


def backproject(g, proj):
    """Exact transpose of ``project``."""
    proj = np.ascontiguousarray(proj, dtype=np.float64).reshape(g.n_angles, g.nz, g.n_u)
    c, s, u, y = _tables(g)
    out = np.empty((g.nz, g.ny, g.nx), dtype=np.float64)
    _load().oracle_backproject(_ptr(proj), g.nx, g.ny, g.nz, g.n_angles, _ptr(c), _ptr(s),
                               _ptr(u), g.n_u, _ptr(y), len(y), _ptr(out))
    return out
