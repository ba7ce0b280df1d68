"""MI355X-native compressed 3D FFL MPI reconstruction (arXiv 2511.06627).

The operator A = blockdiag(A_DC) [P_theta] and its adjoint run as HIP kernels
for gfx950 in ``libmpi3d.so`` (C ABI in ``include/mpi3d.h``); ``Plan`` wraps
them for torch device buffers.  ``configs`` describes the scan workloads and
``phantoms`` draws seeded synthetic volumes.
"""
from . import configs, phantoms  # noqa: F401


def __getattr__(name):
    # Plan needs torch; import lazily so configs/phantoms stay light.
    if name == "Plan":
        from .plan import Plan
        return Plan
    raise AttributeError(name)
