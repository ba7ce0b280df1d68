"""ctypes binding of libmpi3d.so (argument marshalling only).

Every operator step runs in the library's HIP kernels; this module only turns
torch tensors into device pointers and sizes.  It raises if the shared
library has not been built -- there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpi3d.so")

MPI3D_FP32 = 0
MPI3D_MIXED = 1
MPI3D_PRECOMPOSED = 2

NOALLOC_SCRATCH_BYTES = 128 << 20      # MPI3D_NOALLOC_SCRATCH_BYTES

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTSUP", -5: "ENONFINITE"}


class Geometry(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("n_angles", ctypes.c_int32),
        ("theta_rad", ctypes.POINTER(ctypes.c_double)),
        ("n_u", ctypes.c_int32),
        ("n_t", ctypes.c_int32),
        ("drive_cycles", ctypes.c_double),
        ("drive_amp", ctypes.c_double),
        ("psf_width", ctypes.c_double),
        ("harm_lo", ctypes.c_int32), ("harm_hi", ctypes.c_int32),
        ("half_band", ctypes.c_int32),
        ("rx_filter", ctypes.POINTER(ctypes.c_float)),
        ("op_scale", ctypes.c_double),
        ("precisions", ctypes.c_int32),
        ("raster_sweep", ctypes.c_double),
        ("psf_rows", ctypes.c_int32),
        ("drive_axes", ctypes.c_int32),
        ("drive_amp_z", ctypes.c_double),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_vox", ctypes.c_int64), ("n_lines", ctypes.c_int64), ("n_bins", ctypes.c_int64),
        ("n_data_floats", ctypes.c_int64), ("n_proj_floats", ctypes.c_int64),
        ("op_ws_bytes", ctypes.c_int64), ("solve_ws_bytes", ctypes.c_int64),
        ("table_bytes", ctypes.c_int64), ("history_doubles", ctypes.c_int64),
        ("n_r", ctypes.c_int32), ("norm_iters", ctypes.c_int32), ("op_scale", ctypes.c_double),
        ("dft_cycles", ctypes.c_int32), ("dft_residues", ctypes.c_int32),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("lam", ctypes.c_double),
        ("iters", ctypes.c_int32), ("clamp_every", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("refine_sweeps", ctypes.c_int32), ("inner_iters", ctypes.c_int32), ("x0_is_zero", ctypes.c_int32),
        ("solver", ctypes.c_int32), ("reg", ctypes.c_int32), ("tau", ctypes.c_double),
    ]


class SolveReport(ctypes.Structure):
    _fields_ = [
        ("iters_done", ctypes.c_int32), ("status", ctypes.c_int32),
        ("gamma0", ctypes.c_double), ("gamma", ctypes.c_double),
    ]


# Every symbol include/mpi3d.h declares, with its ctypes signature.
_VP = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "mpi3d_plan_create": (_I, [ctypes.POINTER(Geometry), _I, ctypes.POINTER(_VP)]),
    "mpi3d_plan_destroy": (None, [_VP]),
    "mpi3d_plan_query": (_I, [_VP, ctypes.POINTER(PlanInfo)]),
    "mpi3d_forward": (_I, [_VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "mpi3d_adjoint": (_I, [_VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "mpi3d_forward_noalloc": (_I, [_VP, ctypes.c_int32, _VP, _VP, _VP]),
    "mpi3d_project": (_I, [_VP, _VP, _VP, _VP]),
    "mpi3d_backproject": (_I, [_VP, _VP, _VP, _VP]),
    "mpi3d_signal_fwd": (_I, [_VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "mpi3d_signal_adj": (_I, [_VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "mpi3d_solve": (_I, [_VP, _VP, _VP, ctypes.POINTER(SolveOpts), _VP, ctypes.c_size_t, _VP,
                         ctypes.POINTER(SolveReport), _VP]),
    "mpi3d_state_create": (_I, [_VP, _VP, _VP, ctypes.POINTER(SolveOpts), _VP, ctypes.c_size_t,
                                ctypes.POINTER(_VP)]),
    "mpi3d_batch_step": (_I, [ctypes.POINTER(_VP), ctypes.c_int32, _VP]),
    "mpi3d_state_progress": (_I, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "mpi3d_state_destroy": (None, [_VP]),
    "mpi3d_time_kernel": (_I, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_size_t,
                               _VP, ctypes.POINTER(ctypes.c_float)]),
    "mpi3d_strerror": (ctypes.c_char_p, [_I]),
}

_lib = None


def load():
    """Load libmpi3d.so; raise if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmpi3d.so is not built (run python -m paper_2511_06627_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class Mpi3dError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(status, "?"), status))
        self.status = status


def check(fn, status):
    if status != 0:
        raise Mpi3dError(fn, status)
    return status
