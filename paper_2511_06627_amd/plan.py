"""Torch-facing wrapper of the libmpi3d C ABI.

``Plan`` owns one ``mpi3d_plan`` (device tables for one scan geometry) and
calls the library's entry points with torch device buffers.  PyTorch only
provides memory and the stream; every operator step is a HIP kernel of the
library.  Layouts match the C header: volumes float32 (nz, ny, nx), data
complex64 (n_angles, nz, n_bins), projections float32 (n_angles, nz, n_u).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import MPI3D_FP32, MPI3D_MIXED, MPI3D_PRECOMPOSED, check

PRECISION = {"fp32": MPI3D_FP32, "mixed": MPI3D_MIXED, "precomposed": MPI3D_PRECOMPOSED}
SOLVER = {"cgls": 0, "momentum": 1}
REG = {"identity": 0, "fd": 1}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    def __init__(self, nx, ny, nz, n_angles, n_t, drive_cycles, psf_width, harm_lo, harm_hi, half_band,
                 op_scale, theta=None, n_u=0, drive_amp=0.0, rx_filter=None, precisions=("fp32",), device=0,
                 raster_sweep=0.0, psf_rows=0, drive_axes=1, drive_amp_z=0.0):
        lib = _lib.load()
        self.device = torch.device("cuda", device)
        g = _lib.Geometry()
        g.nx, g.ny, g.nz, g.n_angles = nx, ny, nz, n_angles
        self._theta = None
        if theta is not None:
            self._theta = np.ascontiguousarray(theta, dtype=np.float64)
            g.theta_rad = self._theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.n_u = n_u
        g.n_t = n_t
        g.drive_cycles = drive_cycles
        g.drive_amp = drive_amp
        g.psf_width = psf_width
        g.harm_lo, g.harm_hi, g.half_band = harm_lo, harm_hi, half_band
        self._rx = None
        if rx_filter is not None:
            self._rx = np.ascontiguousarray(np.stack([np.real(rx_filter), np.imag(rx_filter)], -1),
                                            dtype=np.float32).ravel()
            g.rx_filter = self._rx.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        g.op_scale = op_scale
        mask = 0
        for p in precisions:
            mask |= 1 << PRECISION[p]
        g.precisions = mask
        g.raster_sweep = raster_sweep
        g.psf_rows = psf_rows
        g.drive_axes = drive_axes
        g.drive_amp_z = drive_amp_z
        self.precisions = tuple(precisions)
        self.raster_sweep = float(raster_sweep)
        self.psf_rows = int(psf_rows)
        handle = ctypes.c_void_p()
        check("mpi3d_plan_create", lib.mpi3d_plan_create(ctypes.byref(g), device, ctypes.byref(handle)))
        self._h = handle
        info = _lib.PlanInfo()
        check("mpi3d_plan_query", lib.mpi3d_plan_query(self._h, ctypes.byref(info)))
        self.info = info
        self.op_scale = float(info.op_scale)      # c_A in use (estimated when 0 was passed)
        self.norm_iters = int(info.norm_iters)
        self.dft_cycles = int(info.dft_cycles)   # FP32 band DFT factored over C-sample blocks (0: dense)
        self.dft_residues = int(info.dft_residues)
        self.shape = (nz, ny, nx)
        self.n_u = n_u or nx
        self.drive_axes = 2 if drive_axes == 2 else 1
        if self.drive_axes == 2:    # x-drive lines, then z-drive lines
            self.data_shape = (int(info.n_lines), int(info.n_bins))
        else:
            self.data_shape = (n_angles, nz, int(info.n_bins))
        self.proj_shape = (n_angles, nz, self.n_u)
        # the signal stage's lines: the projections, plus the z-drive lines
        self.lines_shape = (int(info.n_lines), self.n_u) if self.drive_axes == 2 else self.proj_shape
        self._ws = None

    @classmethod
    def from_config(cls, cfg, op_scale, precisions=("fp32",), device=0, **kw):
        return cls(cfg.nx, cfg.ny, cfg.nz, cfg.n_angles, cfg.n_t, cfg.drive_cycles, cfg.psf_width,
                   cfg.harm_lo, cfg.harm_hi, cfg.half_band, op_scale, precisions=precisions, device=device, **kw)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mpi3d_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers -----------------------------------------------------------
    def workspace(self, kind="op"):
        n = self.info.op_ws_bytes if kind == "op" else self.info.solve_ws_bytes
        return torch.empty(int(n), dtype=torch.uint8, device=self.device)

    def _op_ws(self, ws):
        if ws is None:
            if self._ws is None:
                self._ws = self.workspace("op")
            ws = self._ws
        self._check_ws(ws, "op")
        return ws

    def _check_vol(self, x):
        if x.dtype != torch.float32 or x.device != self.device or not x.is_contiguous() or x.numel() != self.info.n_vox:
            raise ValueError("volume must be a contiguous float32 tensor of %s on %s" % (self.shape, self.device))

    def _check_data(self, b):
        if b.dtype != torch.complex64 or b.device != self.device or not b.is_contiguous() or \
                b.numel() * 2 != self.info.n_data_floats:
            raise ValueError("data must be a contiguous complex64 tensor of %s on %s" % (self.data_shape, self.device))

    def _check_f32(self, t, shape, what):
        n = int(np.prod(shape))
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s must be a contiguous float32 tensor of %s on %s" % (what, shape, self.device))

    def _check_ws(self, ws, kind):
        need = self.info.op_ws_bytes if kind == "op" else self.info.solve_ws_bytes
        if ws.device != self.device or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous tensor on %s" % self.device)
        if ws.numel() * ws.element_size() < need:
            raise ValueError("workspace holds %d bytes, %d needed" % (ws.numel() * ws.element_size(), need))
        return ws.numel() * ws.element_size()

    # ---- operator ------------------------------------------------------------
    def forward(self, x, precision="fp32", out=None, ws=None, stream=None):
        self._check_vol(x)
        out = torch.empty(self.data_shape, dtype=torch.complex64, device=self.device) if out is None else out
        self._check_data(out)
        ws = self._op_ws(ws)
        check("mpi3d_forward", _lib.load().mpi3d_forward(self._h, PRECISION[precision], _ptr(x), _ptr(out),
                                                          _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
        return out

    def adjoint(self, b, precision="fp32", out=None, ws=None, stream=None):
        self._check_data(b)
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check_vol(out)
        ws = self._op_ws(ws)
        check("mpi3d_adjoint", _lib.load().mpi3d_adjoint(self._h, PRECISION[precision], _ptr(b), _ptr(out),
                                                          _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
        return out

    def project(self, x, out=None, stream=None):
        self._check_vol(x)
        out = torch.empty(self.proj_shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check_f32(out, self.proj_shape, "projections")
        check("mpi3d_project", _lib.load().mpi3d_project(self._h, _ptr(x), _ptr(out), _stream(stream)))
        return out

    def backproject(self, rho, out=None, stream=None):
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check_vol(out)
        self._check_f32(rho, self.proj_shape, "projections")
        check("mpi3d_backproject", _lib.load().mpi3d_backproject(self._h, _ptr(rho), _ptr(out), _stream(stream)))
        return out

    def signal_fwd(self, rho, precision="fp32", out=None, ws=None, stream=None):
        out = torch.empty(self.data_shape, dtype=torch.complex64, device=self.device) if out is None else out
        self._check_data(out)
        self._check_f32(rho, self.lines_shape, "lines")
        ws = self._op_ws(ws)
        check("mpi3d_signal_fwd", _lib.load().mpi3d_signal_fwd(self._h, PRECISION[precision], _ptr(rho), _ptr(out),
                                                                _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
        return out

    def signal_adj(self, b, precision="fp32", out=None, ws=None, stream=None):
        self._check_data(b)
        out = torch.empty(self.lines_shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check_f32(out, self.lines_shape, "lines")
        ws = self._op_ws(ws)
        check("mpi3d_signal_adj", _lib.load().mpi3d_signal_adj(self._h, PRECISION[precision], _ptr(b), _ptr(out),
                                                                _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
        return out

    KERNELS = {"project": 0, "backproject": 1, "signal_fwd": 2, "signal_adj": 3,
               # the factored band DFT's kernels (FP32 plans with dft_cycles > 0)
               "fac_fwd": 4, "fac_fwd_out": 5, "fac_adj_in": 6, "fac_adj": 7}

    def time_kernel(self, kernel, repeats=10, precision="fp32", x=None, b=None, ws=None, stream=None):
        """Mean device time (ms) of one launch of an operator kernel, from HIP events."""
        x = torch.zeros(self.shape, dtype=torch.float32, device=self.device) if x is None else x
        b = torch.zeros(self.data_shape, dtype=torch.complex64, device=self.device) if b is None else b
        self._check_vol(x)
        self._check_data(b)
        ws = self._op_ws(ws)
        ms = ctypes.c_float()
        check("mpi3d_time_kernel", _lib.load().mpi3d_time_kernel(
            self._h, self.KERNELS[kernel], PRECISION[precision], repeats, _ptr(x), _ptr(b), _ptr(ws), ws.numel() * ws.element_size(),
            _stream(stream), ctypes.byref(ms)))
        return float(ms.value)

    # ---- solve ---------------------------------------------------------------
    def solve(self, b, lam, iters=0, x=None, precision="fp32", clamp_every=0, refine_sweeps=0, inner_iters=0,
              solver="cgls", reg="identity", tau=0.0, ws=None, history=None, report=True, stream=None):
        """min |Ax - b|^2 + lam |T x|^2 by CGLS (T = I) or the paper's momentum
        iteration (T = I or finite differences).  Returns (x, report or None)."""
        self._check_data(b)
        x0_zero = x is None
        if x is None:
            x = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        self._check_vol(x)
        ws = self.workspace("solve") if ws is None else ws
        if ws.device != self.device or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous tensor on %s" % self.device)
        o = _lib.SolveOpts()
        o.lam, o.iters, o.clamp_every = lam, iters, clamp_every
        o.precision = PRECISION[precision]
        o.refine_sweeps, o.inner_iters = refine_sweeps, inner_iters
        o.x0_is_zero = 1 if x0_zero else 0
        o.solver, o.reg, o.tau = SOLVER[solver], REG[reg], tau
        if history is not None and (history.dtype != torch.float64 or history.device != self.device
                                    or not history.is_contiguous()):
            raise ValueError("history must be a contiguous float64 tensor on %s" % self.device)
        rep = _lib.SolveReport() if report else None
        hptr = _ptr(history) if history is not None else ctypes.c_void_p()
        check("mpi3d_solve", _lib.load().mpi3d_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(o), _ptr(ws), ws.numel() * ws.element_size(),
                                                      hptr, ctypes.byref(rep) if rep is not None else None,
                                                      _stream(stream)))
        return x, rep


class State:
    """One CGLS solve advanced a step at a time by ``batch_step`` (serving).

    Owns (references) its data b, its volume x and its solver workspace; all
    of them stay on the device for the state's whole life.
    """

    def __init__(self, plan, b, lam, precision="fp32", iters=0, refine_sweeps=0, inner_iters=0, clamp_every=0,
                 x=None, ws=None):
        plan._check_data(b)
        self.plan = plan
        self.b = b
        self.x0_zero = x is None
        self.x = torch.empty(plan.shape, dtype=torch.float32, device=plan.device) if x is None else x
        plan._check_vol(self.x)
        self.ws = plan.workspace("solve") if ws is None else ws
        o = _lib.SolveOpts()
        o.lam, o.iters, o.clamp_every = lam, iters, clamp_every
        o.precision = PRECISION[precision]
        o.refine_sweeps, o.inner_iters = refine_sweeps, inner_iters
        o.x0_is_zero = 1 if self.x0_zero else 0
        h = ctypes.c_void_p()
        check("mpi3d_state_create", _lib.load().mpi3d_state_create(plan._h, _ptr(b), _ptr(self.x), ctypes.byref(o),
                                                                    _ptr(self.ws), self.ws.numel() * self.ws.element_size(), ctypes.byref(h)))
        self._h = h

    def progress(self):
        it = ctypes.c_int32()
        done = ctypes.c_int32()
        check("mpi3d_state_progress", _lib.load().mpi3d_state_progress(self._h, ctypes.byref(it), ctypes.byref(done)))
        return int(it.value), bool(done.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mpi3d_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step(states, stream=None):
    """One step (an iteration, or the restart opening a sweep) of every state."""
    if not states:
        return
    arr = (ctypes.c_void_p * len(states))(*[s._h for s in states])
    check("mpi3d_batch_step", _lib.load().mpi3d_batch_step(arr, len(states), _stream(stream)))
