"""Oracle signal model and harmonic compression, FP64.

Test infrastructure only (see ``oracle/__init__``).

Per FFL line l = (angle m, z-row k) with projection rho_theta[l, :]:

1. Time signal (eq. stheta1 with the collinear PSF of Appendix B eq. PSF,
   B = I):  s[l, n] = c_A v_n sum_p rho_theta[l, p] L'((xi_n - u_p)/w) / w,
   with xi and v those of the line's trajectory class (one class, or two
   under a raster: ``geometry.line_classes``).  With the tensor PSF coupling
   rows (``psf_rows`` = R > 0) the sum also runs over the rows k' of the same
   angle with |k - k'| <= R, through h_xx at z-offset k - k'
   (``physics.psf_xx``, ``kernel_row``, ``coupled_apply``).
2. Compression (eq. bcompress, eq. DCmodel, Appendix A):
   b[l, j] = D_Gamma[j] T^{-1/2} sum_n s[l, n] exp(+2 pi i omega_j n / T),
   the unitary DFT of Appendix A (plus sign, 1/sqrt(N)) restricted to the
   kept bins, with the receive filter as a diagonal on the kept bins.
3. Adjoint: the exact transpose of 1-2 in the real inner product
   <u, v> = Re(u^H v); the paper's projection onto real values (Sec. 3.3,
   after eq. iters) is what taking Re amounts to.

The DFT phase is formed from the exact integer product (omega_j n) mod T so no
large float argument reaches sin/cos.

``line_matrix`` precomposes C = D_Gamma F_S V K (shape nb x Nu) -- the same
operator associated differently -- used only to cross-check the time-domain
path and to speed up long FP64 reference solves; callers that use it say so.

Pins (tests/test_oracle_signal.py): DFT = sqrt(T) * numpy.fft.ifft; Parseval
over the full spectrum; |Re(F_S^H z)|^2 = |z|^2 / 2; half-wave symmetry
(even harmonics vanish) and empty side bins at integer P; adjoint identity;
precomposed vs time-domain path.
"""
import numpy as np

from .geometry import detector_grid, kept_bins, line_classes
from .physics import psf_kernel, psf_xx, trajectory

_LINE_BLOCK = 512  # lines per block, bounds the (lines x T) temporaries


def dft_matrix(g, bins=None):
    """E[n, j] = D_j exp(+2 pi i ((omega_j n) mod T) / T) / sqrt(T), shape (T, nb).

    ``bins`` overrides the kept set (used by the Parseval pin, which needs all
    T frequencies); the receive filter then is not applied.
    """
    w = kept_bins(g) if bins is None else np.asarray(bins, dtype=np.int64)
    n = np.arange(g.n_t, dtype=np.int64)
    phase = (n[:, None] * w[None, :]) % g.n_t
    e = np.exp(2j * np.pi * phase / g.n_t) / np.sqrt(g.n_t)
    if bins is None and g.rx_filter is not None:
        e = e * np.asarray(g.rx_filter, dtype=np.complex128)[None, :]
    return e


def kernel(g, cls=0):
    """K of trajectory class cls (1: the raster's backward sweep)."""
    direction = -1.0 if cls == 1 else 1.0
    return psf_kernel(g.n_t, g.drive_cycles, g.drive_amp, g.psf_width, detector_grid(g), g.op_scale,
                      g.raster_sweep, direction)


def kernel_row(g, d):
    """K_d[n, p] = c_A v_n h_xx(xi_n - u_p, d): the table coupling a line to
    the row d voxels away (tensor PSF; K_0 is the collinear ``kernel``)."""
    xi, v = trajectory(g.n_t, g.drive_cycles, g.drive_amp)
    du = xi[:, None] - detector_grid(g)[None, :]
    return g.op_scale * v[:, None] * psf_xx(du, d, g.psf_width)


def coupled_rows(g):
    return min(g.psf_rows, g.nz - 1)


def coupled_columns(g):
    """Detector columns coupled on each side to a z-drive line (tensor PSF)."""
    return min(g.psf_rows, g.n_u - 1)


def coupled_apply(g, rows, mats, adjoint=False, per=None):
    """The row-coupled map over the lines of every angle in line order, `per`
    lines an angle (default the z-rows): forward
    out[m, k] = sum_{|d| <= R} rows[m, k + d] @ mats[|d|].T, adjoint its
    transpose out[m, k + d] += rows[m, k] @ mats[|d|], R = len(mats) - 1."""
    per = g.nz if per is None else per
    R = len(mats) - 1
    rr = rows.reshape(g.n_angles, per, -1)
    width = mats[0].shape[1] if adjoint else mats[0].shape[0]
    out = np.zeros((g.n_angles, per, width), dtype=np.result_type(rows, mats[0]))
    for d in range(-R, R + 1):
        lo, hi = max(0, -d), min(per, per - d)
        if lo >= hi:
            continue
        M = mats[abs(d)]
        if adjoint:
            out[:, lo + d:hi + d] += rr[:, lo:hi] @ M
        else:
            out[:, lo:hi] += rr[:, lo + d:hi + d] @ M.T
    return out.reshape(g.n_angles * per, width)


def z_grid(g):
    """Sample positions of a z-drive line: the z-rows, centred."""
    return np.arange(g.nz, dtype=np.float64) - (g.nz - 1) / 2.0


def kernel_z(g):
    """K of the z-drive lines: c_A v_n L'((xi_n - z_k)/w)/w with amplitude a_z, shape (T, Nz)."""
    return psf_kernel(g.n_t, g.drive_cycles, g.drive_amp_z, g.psf_width, z_grid(g), g.op_scale)


def kernel_z_column(g, d):
    """K_z,d[n, k] = c_A v_n h(xi_n - z_k, d): a z-drive line's coupling to the
    detector column d voxels away under the tensor PSF.  With drive and
    receive coil along z, the entry of eq. PSF is the xx entry with the two
    axes exchanged: along-drive offset xi_n - z_k, transverse offset d
    (``physics.psf_xx``); K_z,0 is ``kernel_z``."""
    xi, v = trajectory(g.n_t, g.drive_cycles, g.drive_amp_z)
    dz = xi[:, None] - z_grid(g)[None, :]
    return g.op_scale * v[:, None] * psf_xx(dz, d, g.psf_width)


def z_column_matrices(g, precomposed):
    """The z-drive lines' tables per column offset d = 0..R (time domain), or
    precomposed with the band DFT: E^T K_z,d."""
    Ks = [kernel_z_column(g, d) for d in range(coupled_columns(g) + 1)]
    if not precomposed:
        return Ks
    E = dft_matrix(g)
    return [E.T @ K for K in Ks]


def z_lines(g, rho_theta):
    """z-drive lines of the projections rho_theta (M, Nz, Nu): line m*Nu + p is the
    column rho_theta[m, :, p], shape (M*Nu, Nz)."""
    r = np.asarray(rho_theta).reshape(g.n_angles, g.nz, g.n_u)
    return np.ascontiguousarray(r.transpose(0, 2, 1)).reshape(g.n_z_lines, g.nz)


def z_lines_transpose(g, zl):
    """Transpose of ``z_lines``: (M*Nu, Nz) -> (M, Nz, Nu)."""
    return np.ascontiguousarray(np.asarray(zl).reshape(g.n_angles, g.n_u, g.nz).transpose(0, 2, 1))


def classes_present(g):
    return (0, 1) if g.raster_sweep and g.nz > 1 else (0,)


def row_classes(g, n_rows):
    """Class of each of n_rows line rows: any number of rows of a one-class
    scan, or all L lines of a raster scan in line order."""
    if len(classes_present(g)) == 1:
        return np.zeros(n_rows, dtype=np.int64)
    assert n_rows == g.n_lines, "a raster scan's lines must be passed together"
    return line_classes(g)


def time_signal(g, rho_theta, K=None):
    """s[l, n], shape (rows, T): with K given, every row through K; else every
    line of the scan through its own class's K (rows must be all L lines when
    the scan has a raster)."""
    r = np.asarray(rho_theta, dtype=np.float64).reshape(-1, g.n_u)
    if K is not None:
        return r @ K.T
    if g.psf_rows:
        assert r.shape[0] == g.n_lines
        return coupled_apply(g, r, [kernel_row(g, d) for d in range(coupled_rows(g) + 1)])
    cl = row_classes(g, r.shape[0])
    out = np.empty((r.shape[0], g.n_t))
    for c in classes_present(g):
        idx = np.flatnonzero(cl == c)
        out[idx] = r[idx] @ kernel(g, c).T
    return out


def compress(g, s, E=None):
    """b[l, j] = sum_n s[l, n] E[n, j]."""
    E = dft_matrix(g) if E is None else E
    return np.asarray(s, dtype=np.float64) @ E


def forward(g, rho_theta):
    """Lines (L, Nu) -> compressed data (L, nb), time-domain path, block over lines."""
    r = np.asarray(rho_theta, dtype=np.float64).reshape(-1, g.n_u)
    E = dft_matrix(g)
    if g.psf_rows:
        assert r.shape[0] == g.n_lines and not g.raster_sweep
        s = coupled_apply(g, r, [kernel_row(g, d) for d in range(coupled_rows(g) + 1)])
        return compress(g, s, E)
    cl = row_classes(g, r.shape[0])
    out = np.empty((r.shape[0], g.n_bins), dtype=np.complex128)
    for c in classes_present(g):
        K = kernel(g, c)
        idx = np.flatnonzero(cl == c)
        for a in range(0, idx.size, _LINE_BLOCK):
            rows = idx[a:a + _LINE_BLOCK]
            out[rows] = compress(g, time_signal(g, r[rows], K), E)
    return out


def adjoint(g, y):
    """Compressed data (L, nb) -> lines (L, Nu): Re of the Hermitian transpose."""
    y = np.asarray(y, dtype=np.complex128).reshape(-1, g.n_bins)
    E = dft_matrix(g)
    if g.psf_rows:
        assert y.shape[0] == g.n_lines and not g.raster_sweep
        h = np.real(y @ np.ascontiguousarray(np.conj(E).T))
        return coupled_apply(g, h, [kernel_row(g, d) for d in range(coupled_rows(g) + 1)], adjoint=True)
    cl = row_classes(g, y.shape[0])
    out = np.empty((y.shape[0], g.n_u), dtype=np.float64)
    for c in classes_present(g):
        K = kernel(g, c)
        idx = np.flatnonzero(cl == c)
        for a in range(0, idx.size, _LINE_BLOCK):
            rows = idx[a:a + _LINE_BLOCK]
            h = np.real(y[rows] @ np.ascontiguousarray(np.conj(E).T))  # transpose of compress
            out[rows] = h @ K                                         # transpose of time_signal
    return out


def line_matrix(g, cls=0):
    """C[j, p] = sum_n E[n, j] K[n, p]: the per-line operator of class cls, precomposed."""
    return dft_matrix(g).T @ kernel(g, cls)


def row_matrices(g):
    """C_d = E^T K_d, d = 0..R: the coupled model precomposed per row offset."""
    E = dft_matrix(g)
    return [E.T @ kernel_row(g, d) for d in range(coupled_rows(g) + 1)]


def information_retained(s, bins):
    """I(s, S) = sqrt(sum_{w in S} |s_hat_w|^2) / |s| per row (Appendix A).

    Counts both the kept positive bins and their conjugate mirrors, which a
    real signal carries with the same magnitude.
    """
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    n = s.shape[1]
    sh = np.fft.ifft(s, axis=1) * np.sqrt(n)
    kept = np.zeros(n, dtype=bool)
    kept[np.asarray(bins)] = True
    kept[(n - np.asarray(bins)) % n] = True
    return np.sqrt((np.abs(sh[:, kept]) ** 2).sum(axis=1)) / np.linalg.norm(s, axis=1)
