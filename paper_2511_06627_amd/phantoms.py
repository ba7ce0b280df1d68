"""Seeded synthetic phantoms (MNP density volumes) for the scan workloads.

Input generation only: this module draws random shapes and evaluates them at
voxel centres; it contains none of the reconstruction method's arithmetic.

Volumes are float64 arrays of shape (Nz, Ny, Nx), x fastest.  Index
coordinates: voxel (i, j, k) sits at (i, j, k).  All draws come from one
numpy PCG64 stream per phantom, in a fixed order, so a seed fixes the volume.

* Gaussian blobs: a * exp(-|r - c|^2 / (2 sigma^2)), point-sampled (as a
  product of its x, y and z factors); centre
  uniform in [lo*N, hi*N] per axis; sigma uniform; amplitude log-uniform.
* Ellipsoid: hard-edged indicator of amplitude ``amp`` with semi-axes
  U[0.12, 0.25] * (Nx, Ny, Nz) and centre uniform over the inner half.
* Faint satellites (high-dynamic-range scan): blobs whose centre lies a gap
  g ~ U[2, 5] voxels outside the ellipsoid surface, along the outward normal
  at a random surface point.
"""
import numpy as np


def _grid(shape):
    nz, ny, nx = shape
    return np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                       np.arange(nx, dtype=np.float64), indexing="ij")


def _blob(shape, c, sigma, amp):
    """Point-sampled isotropic Gaussian, evaluated as the outer product of its
    three axis factors (the same function, a fraction of the work)."""
    nz, ny, nx = shape
    f = [np.exp(-(np.arange(n, dtype=np.float64) - ci) ** 2 / (2.0 * sigma * sigma)) for n, ci in
         ((nx, c[0]), (ny, c[1]), (nz, c[2]))]
    return amp * (f[2][:, None, None] * (f[1][:, None] * f[0][None, :])[None, :, :])


def gaussian_blobs(shape, n_blobs, sigma_range, amp_log10_range, seed, centre_frac=(0.1, 0.9)):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    vol = np.zeros(shape)
    dims = np.array([nx, ny, nz], dtype=np.float64)
    for _ in range(n_blobs):
        c = rng.uniform(centre_frac[0], centre_frac[1], size=3) * dims
        sigma = rng.uniform(*sigma_range)
        amp = 10.0 ** rng.uniform(*amp_log10_range)
        vol += _blob(shape, c, sigma, amp)
    return vol


def ellipsoid(shape, seed, amp=1.0):
    """Returns (volume, centre, semi_axes) -- centre and axes in (x, y, z) order."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    dims = np.array([nx, ny, nz], dtype=np.float64)
    axes = rng.uniform(0.12, 0.25, size=3) * dims
    centre = rng.uniform(0.25, 0.75, size=3) * dims
    zz, yy, xx = _grid(shape)
    inside = (((xx - centre[0]) / axes[0]) ** 2 + ((yy - centre[1]) / axes[1]) ** 2
              + ((zz - centre[2]) / axes[2]) ** 2) <= 1.0
    return amp * inside.astype(np.float64), centre, axes


def organ_with_satellites(shape, n_blobs, sigma_range, amp_log10_range, gap_range, seed):
    """Bright ellipsoid plus faint blobs just outside its surface.

    Returns (volume, blobs) with blobs a list of (centre_xyz, sigma, amp) so a
    caller can measure recovered amplitudes.
    """
    vol, centre, axes = ellipsoid(shape, seed)
    rng = np.random.default_rng(seed + 7919)
    blobs = []
    for _ in range(n_blobs):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        t = 1.0 / np.sqrt(np.sum((d / axes) ** 2))
        surf = centre + t * d
        normal = (surf - centre) / axes ** 2
        normal /= np.linalg.norm(normal)
        gap = rng.uniform(*gap_range)
        sigma = rng.uniform(*sigma_range)
        amp = 10.0 ** rng.uniform(*amp_log10_range)
        c = surf + gap * normal
        vol += _blob(shape, c, sigma, amp)
        blobs.append((c, sigma, amp))
    return vol, blobs


def blobs_and_organ(shape, n_blobs, sigma_range, amp_log10_range, seed):
    """Blobs over the whole inner volume plus one bright ellipsoid (realistic scan)."""
    vol = gaussian_blobs(shape, n_blobs, sigma_range, amp_log10_range, seed)
    org, _, _ = ellipsoid(shape, seed + 104729)
    return vol + org
