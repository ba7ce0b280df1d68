"""Oracle finite-difference regulariser T of eq. nummodel, FP64.

Test infrastructure only (see ``oracle/__init__``).

The paper regularises with lambda ||T x||^2, T a finite-difference operator
(Sec. 3.3, after eq. nummodel), without fixing its stencil or boundary.
Reading taken here: T stacks the forward differences along x, y and z,

    (D_a x)[i] = x[i + e_a] - x[i]   for voxels i whose neighbour i + e_a is
                                     inside the grid (no term across the
                                     volume boundary),

so T^T T is the 7-point discrete Laplacian with Neumann (reflecting)
boundary, L_x (+) L_y (+) L_z as a Kronecker sum of 1D second-difference
matrices whose eigenvalues are 2 - 2 cos(pi k / n), k = 0..n-1.  Hence

    ||T^T T||_2 = sum over axes of (2 - 2 cos(pi (n_a - 1) / n_a)),

and T^T T annihilates constants.

Pins (tests/test_oracle_regularizer.py): T and T^T are exact adjoints; T^T T
on a small grid equals the Kronecker sum built from numpy's 1D matrices; its
largest eigenvalue (numpy.linalg.eigvalsh) equals the closed form; constants
are in its null space.
"""
import math

import numpy as np


def fd_forward(x):
    """T x: the three forward-difference fields (dx, dy, dz), each of shape
    (nz, ny, nx) with the last slab along its axis zero (no boundary term)."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    for axis in (2, 1, 0):           # x, y, z
        d = np.zeros_like(x)
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[axis] = slice(1, None)
        sl_lo[axis] = slice(0, -1)
        d[tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
        out.append(d)
    return out


def fd_adjoint(ds):
    """T^T applied to three difference fields (the exact transpose of fd_forward)."""
    res = np.zeros_like(np.asarray(ds[0], dtype=np.float64))
    for axis, d in zip((2, 1, 0), ds):
        d = np.asarray(d, dtype=np.float64)
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[axis] = slice(1, None)
        sl_lo[axis] = slice(0, -1)
        res[tuple(sl_hi)] += d[tuple(sl_lo)]
        res[tuple(sl_lo)] -= d[tuple(sl_lo)]
    return res


def fd_normal(x):
    """T^T T x."""
    return fd_adjoint(fd_forward(x))


def fd_normal_norm(shape):
    """||T^T T||_2 for a volume of shape (nz, ny, nx), closed form."""
    return float(sum(2.0 - 2.0 * math.cos(math.pi * (n - 1) / n) for n in shape if n > 1))
