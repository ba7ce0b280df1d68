"""Oracle geometry: voxel and detector grids, angles, ray samples, kept bins.

Test infrastructure only (see ``oracle/__init__``).

Readings of the paper used here (each listed in the design doc):
* Voxel centres X_i = i - (Nx-1)/2, Y_j = j - (Ny-1)/2 in voxel units; the
  FFL rotates about z (Sec. 2.2), so the volume is a stack of independent
  z-slices and z-line k of every angle is voxel row k.
* Detector (fast-axis) samples u_p = p - (Nu-1)/2.
* Angles theta_m = m pi / M, equally spaced over [0, 180) (Sec. 3.1).
* The line integral of eq. ptheta2 is a unit-step Riemann sum over ray samples
  y_q = q - (Nr-1)/2, Nr the smallest integer >= sqrt(Nx^2+Ny^2) with the
  parity of Ny, so that at theta = 0 every sample falls on a voxel centre.
* Tensor PSF coupling: FFL line (m, k) sees the rows k' with |k - k'| <= R
  (``psf_rows``) of the same angle's projection through the x-x tensor PSF at
  z-offset k - k' (rows one voxel apart); R >= Nz - 1 is the whole model, R = 0
  the collinear one.
* Dual drive (Sec. 3.1: every angle is scanned with the drive along x and
  again along z): the z-drive scan of angle m has one line per detector column
  p, running across the z-rows k with samples at z_k = k - (Nz-1)/2 and drive
  amplitude a_z (default Nz/2), through the same collinear PSF and bins.  Its
  lines follow the x-drive lines in the data, m-major: line M*Nz + m*Nu + p.
* Raster trajectory classes: every angle repeats one scan sequence (Sec. 2.2,
  before eq. modelF1); under a zig-zag raster (Sec. 3.1) the sweep direction
  alternates from line to line, so z-row k sweeps forward when k is even and
  backward when k is odd.
* Kept bins (eq. bcompress, Appendix A's set S): for harmonics k = k_lo..k_hi
  and offsets d = -D..D, omega_{k,d} = floor(k P + 1/2) + d, ordered k-major,
  positive frequencies only (the data are a real signal's spectrum).
"""
from dataclasses import dataclass, field
import math
import numpy as np


@dataclass
class Geometry:
    nx: int
    ny: int
    nz: int
    n_angles: int
    n_t: int
    drive_cycles: float
    psf_width: float
    harm_lo: int
    harm_hi: int
    half_band: int
    op_scale: float = 1.0
    drive_amp: float = None          # default Nu/2: the sweep spans the fast axis
    n_u: int = None                  # default Nx
    theta: np.ndarray = None         # default m*pi/M
    rx_filter: np.ndarray = None     # complex D_Gamma on the kept bins, None = 1
    raster_sweep: float = 0.0        # focus-field shift per line in voxels (0 = none)
    psf_rows: int = 0                # z-rows coupled by the tensor PSF on each side (0 = collinear)
    drive_axes: int = 1              # 1: x-drive scan; 2: x- and z-drive scans (dual drive)
    drive_amp_z: float = None        # z-drive amplitude in voxels, default Nz/2

    def __post_init__(self):
        if self.n_u is None:
            self.n_u = self.nx
        if self.drive_amp is None:
            self.drive_amp = self.n_u / 2.0
        if self.drive_amp_z is None:
            self.drive_amp_z = self.nz / 2.0
        assert self.drive_axes in (1, 2)
        if self.theta is None:
            self.theta = np.arange(self.n_angles, dtype=np.float64) * np.pi / self.n_angles
        self.theta = np.asarray(self.theta, dtype=np.float64)
        assert self.theta.shape == (self.n_angles,)

    # ---- derived sizes -------------------------------------------------
    @property
    def n_lines(self):
        return self.n_angles * self.nz

    @property
    def n_z_lines(self):
        """z-drive lines: one per angle and detector column (dual drive only)."""
        return self.n_angles * self.n_u if self.drive_axes == 2 else 0

    @property
    def n_data_lines(self):
        return self.n_lines + self.n_z_lines

    @property
    def n_bins(self):
        return (self.harm_hi - self.harm_lo + 1) * (2 * self.half_band + 1)

    @property
    def n_vox(self):
        return self.nx * self.ny * self.nz

    def with_scale(self, op_scale):
        g = Geometry(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        g.op_scale = float(op_scale)
        return g

    def slice_geometry(self):
        """The same scan on the fewest z-slices that hold every distinct slice
        operator: one slice, or two under a raster (even and odd rows sweep in
        opposite directions)."""
        g = Geometry(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        if self.psf_rows or self.drive_axes == 2:
            return g          # rows are coupled (tensor PSF, z-drive lines): no smaller equivalent
        g.nz = min(self.nz, 2) if self.raster_sweep else 1
        return g


def line_classes(g):
    """Trajectory class of every line l = m*Nz + k: k mod 2 under a raster, else 0."""
    k = np.tile(np.arange(g.nz, dtype=np.int64), g.n_angles)
    return k % 2 if g.raster_sweep else np.zeros_like(k)


def voxel_centres(n):
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def detector_grid(g):
    return np.arange(g.n_u, dtype=np.float64) - (g.n_u - 1) / 2.0


def ray_samples(g):
    nr = int(math.ceil(math.sqrt(g.nx * g.nx + g.ny * g.ny)))
    while nr * nr < g.nx * g.nx + g.ny * g.ny:
        nr += 1
    if (nr - g.ny) % 2:
        nr += 1
    return np.arange(nr, dtype=np.float64) - (nr - 1) / 2.0


def kept_bins(g):
    """omega_{k,d} = floor(k P + 1/2) + d, k-major; validated to lie in (0, T/2) and be distinct."""
    out = []
    for k in range(g.harm_lo, g.harm_hi + 1):
        c = math.floor(k * g.drive_cycles + 0.5)
        for d in range(-g.half_band, g.half_band + 1):
            out.append(c + d)
    out = np.asarray(out, dtype=np.int64)
    if out.min() <= 0 or out.max() >= g.n_t // 2 or len(set(out.tolist())) != len(out):
        raise ValueError("kept bins must be distinct and inside (0, T/2)")
    return out
