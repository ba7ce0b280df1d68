"""Oracle full operator A = blockdiag(A_DC) [P_theta1; ...; P_thetaM], FP64.

Test infrastructure only (see ``oracle/__init__``).

* ``forward``  -- eq. modelF1 / the definition of A in Sec. 3.3: project every
                  angle, then apply A_DC (eq. DCmodel) to every FFL line.
* ``adjoint``  -- A^T = Re(A^H), the exact transpose in <u,v> = Re(u^H v).
* ``op_norm``  -- ||A||_2 by FP64 power iteration on A^T A.  The paper needs
                  ||A* A||_2 for its step size (after eq. iters) but does not
                  say how it is found.  A is block diagonal over z-slices (the
                  projector acts slice by slice) with the same block on every
                  slice of one trajectory class, so the norm is taken on one
                  slice, or on two under a raster.
* Dual drive -- the z-drive lines follow the x-drive lines (``geometry``);
                  A^T adds their transposed contributions to the projections.
                  Under the tensor PSF the x-drive lines couple across z-rows
                  and the z-drive lines across detector columns (the same
                  tensor entry with the drive axis exchanged).
* ``make_data`` -- synthetic compressed data: clean time signal of a phantom,
                  plus white Gaussian noise in the time domain with standard
                  deviation level * max|s_clean|, then compression.

Pins (tests/test_oracle_operator.py): adjoint identity to 1e-12; brute-force
dense A on 8^3 written from the element formula; precomposed vs time-domain;
exact z-separability; the one-slice norm equals the full-volume norm.
"""
import numpy as np

from . import projector, signal


def _per_class(g, rows_in, fn):
    """Apply fn(class, rows of that class) line by line class."""
    cl = signal.row_classes(g, rows_in.shape[0])
    out = None
    for c in signal.classes_present(g):
        idx = np.flatnonzero(cl == c)
        part = fn(c, rows_in[idx])
        if out is None:
            out = np.empty((rows_in.shape[0],) + part.shape[1:], dtype=part.dtype)
        out[idx] = part
    return out


def _dual_forward(g, rt, lines_fwd, z_fwd):
    """Dual drive: x-drive lines then z-drive lines, shape (L_x + L_z, nb)."""
    bx = lines_fwd(rt.reshape(g.n_lines, g.n_u))
    bz = z_fwd(signal.z_lines(g, rt))
    return np.concatenate([bx.reshape(g.n_lines, g.n_bins), bz.reshape(g.n_z_lines, g.n_bins)])


def _dual_adjoint(g, y, lines_adj, z_adj):
    y = np.asarray(y, dtype=np.complex128).reshape(g.n_data_lines, g.n_bins)
    lines = lines_adj(y[:g.n_lines]).reshape(g.n_angles, g.nz, g.n_u)
    return lines + signal.z_lines_transpose(g, z_adj(y[g.n_lines:]))


def forward(g, x, precomposed=False):
    if g.drive_axes == 2:
        return Operator(g, precomposed).forward(x)
    rt = projector.project(g, x).reshape(g.n_lines, g.n_u)
    if precomposed and g.psf_rows:
        return signal.coupled_apply(g, rt, signal.row_matrices(g)).reshape(g.n_angles, g.nz, g.n_bins)
    if precomposed:
        b = _per_class(g, rt, lambda c, r: r @ signal.line_matrix(g, c).T)
        return b.reshape(g.n_angles, g.nz, g.n_bins)
    return signal.forward(g, rt).reshape(g.n_angles, g.nz, g.n_bins)


def adjoint(g, y, precomposed=False):
    if g.drive_axes == 2:
        return Operator(g, precomposed).adjoint(y)
    y = np.asarray(y, dtype=np.complex128).reshape(g.n_lines, g.n_bins)
    if precomposed and g.psf_rows:
        lines = np.real(signal.coupled_apply(g, y, [np.conj(C) for C in signal.row_matrices(g)], adjoint=True))
    elif precomposed:
        lines = _per_class(g, y, lambda c, r: np.real(r @ np.conj(signal.line_matrix(g, c))))
    else:
        lines = signal.adjoint(g, y)
    return projector.backproject(g, lines.reshape(g.n_angles, g.nz, g.n_u))


class Operator:
    """A with its tables built once (C precomposed optional), per trajectory class."""

    def __init__(self, g, precomposed=False):
        self.g = g
        self.precomposed = precomposed
        self.classes = signal.classes_present(g)
        self.coupled = bool(g.psf_rows)
        self.dual = g.drive_axes == 2
        if self.dual:
            assert not g.raster_sweep
            if g.psf_rows:
                self.Mz = signal.z_column_matrices(g, precomposed)   # per column offset
            else:
                Kz = signal.kernel_z(g)
                if precomposed:
                    self.Cz = signal.dft_matrix(g).T @ Kz
                else:
                    self.Kz = Kz
        if self.coupled:
            assert not g.raster_sweep
            rows = range(signal.coupled_rows(g) + 1)
            if precomposed:
                self.Cd = signal.row_matrices(g)
            else:
                self.Kd = [signal.kernel_row(g, d) for d in rows]
        if precomposed:
            self.C = {c: signal.line_matrix(g, c) for c in self.classes}
        else:
            self.K = {c: signal.kernel(g, c) for c in self.classes}
            self.E = signal.dft_matrix(g)
            # real and imaginary parts kept apart so real signals meet real matrices
            self.E_re = np.ascontiguousarray(self.E.real)
            self.E_im = np.ascontiguousarray(self.E.imag)

    def _lines_fwd_class(self, c, rt):
        if self.precomposed:
            return rt @ self.C[c].T
        out = np.empty((rt.shape[0], self.g.n_bins), dtype=np.complex128)
        for a in range(0, rt.shape[0], 512):
            s = rt[a:a + 512] @ self.K[c].T
            out[a:a + 512] = (s @ self.E_re) + 1j * (s @ self.E_im)
        return out

    def _lines_adj_class(self, c, y):
        if self.precomposed:
            return np.real(y @ np.conj(self.C[c]))
        out = np.empty((y.shape[0], self.g.n_u), dtype=np.float64)
        for a in range(0, y.shape[0], 512):
            yb = y[a:a + 512]
            # Re(y conj(E)^T); contiguous copies keep numpy on its BLAS path
            h = np.ascontiguousarray(yb.real) @ self.E_re.T + np.ascontiguousarray(yb.imag) @ self.E_im.T
            out[a:a + 512] = h @ self.K[c]
        return out

    def _lines_fwd(self, rt):
        if self.coupled and self.precomposed:
            return signal.coupled_apply(self.g, rt, self.Cd)
        if self.coupled:
            s = signal.coupled_apply(self.g, rt, self.Kd)
            return (s @ self.E_re) + 1j * (s @ self.E_im)
        return _per_class(self.g, rt, self._lines_fwd_class)

    def _lines_adj(self, y):
        if self.coupled and self.precomposed:
            return np.real(signal.coupled_apply(self.g, y, [np.conj(C) for C in self.Cd], adjoint=True))
        if self.coupled:
            h = np.ascontiguousarray(y.real) @ self.E_re.T + np.ascontiguousarray(y.imag) @ self.E_im.T
            return signal.coupled_apply(self.g, h, self.Kd, adjoint=True)
        return _per_class(self.g, y, self._lines_adj_class)

    def _z_fwd(self, zl):
        g = self.g
        if self.coupled:   # z-drive lines coupled across the detector columns of their angle
            if self.precomposed:
                return signal.coupled_apply(g, zl, self.Mz, per=g.n_u)
            s = signal.coupled_apply(g, zl, self.Mz, per=g.n_u)
            return (s @ self.E_re) + 1j * (s @ self.E_im)
        if self.precomposed:
            return zl @ self.Cz.T
        s = zl @ self.Kz.T
        return (s @ self.E_re) + 1j * (s @ self.E_im)

    def _z_adj(self, y):
        g = self.g
        if self.coupled:
            if self.precomposed:
                return np.real(signal.coupled_apply(g, y, [np.conj(C) for C in self.Mz], adjoint=True, per=g.n_u))
            h = np.ascontiguousarray(y.real) @ self.E_re.T + np.ascontiguousarray(y.imag) @ self.E_im.T
            return signal.coupled_apply(g, h, self.Mz, adjoint=True, per=g.n_u)
        if self.precomposed:
            return np.real(y @ np.conj(self.Cz))
        h = np.ascontiguousarray(y.real) @ self.E_re.T + np.ascontiguousarray(y.imag) @ self.E_im.T
        return h @ self.Kz

    def forward(self, x):
        g = self.g
        rt = projector.project(g, x).reshape(g.n_lines, g.n_u)
        if self.dual:
            return _dual_forward(g, rt, self._lines_fwd, self._z_fwd)
        return self._lines_fwd(rt).reshape(g.n_angles, g.nz, g.n_bins)

    def adjoint(self, y):
        g = self.g
        if self.dual:
            return projector.backproject(g, _dual_adjoint(g, y, self._lines_adj, self._z_adj))
        y = np.asarray(y, dtype=np.complex128).reshape(g.n_lines, g.n_bins)
        lines = self._lines_adj(y)
        return projector.backproject(g, lines.reshape(g.n_angles, g.nz, g.n_u))


def op_norm(g, iters_min=100, iters_max=3000, rtol=1e-10, seed=12345, one_slice=True):
    """||A||_2 by power iteration on A^T A in FP64 (precomposed lines for speed)."""
    gs = g.slice_geometry() if one_slice else g
    op = Operator(gs, precomposed=True)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((gs.nz, gs.ny, gs.nx))
    x /= np.linalg.norm(x)
    lam_old = 0.0
    for it in range(iters_max):
        y = op.adjoint(op.forward(x))
        lam = float(np.vdot(x, y).real)
        x = y / np.linalg.norm(y)
        if it + 1 >= iters_min and abs(lam - lam_old) <= rtol * abs(lam):
            break
        lam_old = lam
    return float(np.sqrt(lam))


def normalised(g, **kw):
    """The geometry with c_A chosen so that ||A||_2 = 1."""
    return g.with_scale(1.0 / op_norm(g.with_scale(1.0), **kw))


def make_data(g, phantom, noise_level, noise_seed):
    """Compressed data b (M, Nz, nb) of a phantom with time-domain white noise
    ((L_x + L_z, nb) with the dual drive).

    Also returns the noise standard deviation used.  Noise is drawn line block
    by line block from one PCG64 stream, in line order, so the result does
    not depend on the block size.
    """
    op = Operator(g)
    rt = projector.project(g, phantom).reshape(g.n_lines, g.n_u)
    cl = signal.row_classes(g, g.n_lines)

    s_all = signal.coupled_apply(g, rt, op.Kd) if op.coupled else None
    if op.dual:   # x-drive lines, then z-drive lines
        zl = signal.z_lines(g, rt)
        if op.coupled:
            s_all = np.concatenate([s_all, signal.coupled_apply(g, zl, op.Mz, per=g.n_u)])
        else:
            s_all = np.concatenate([rt @ op.K[0].T, zl @ op.Kz.T])

    def clean(a):   # time signals of lines a .. a+511, each through its class's K
        if s_all is not None:
            return s_all[a:a + 512]
        s = np.empty((min(512, g.n_lines - a), g.n_t))
        for c in op.classes:
            m = cl[a:a + 512] == c
            s[m] = rt[a:a + 512][m] @ op.K[c].T
        return s

    s_max = 0.0
    n_rows = g.n_data_lines
    for a in range(0, n_rows, 512):
        s_max = max(s_max, float(np.abs(clean(a)).max()))
    sigma = noise_level * s_max
    rng = np.random.default_rng(noise_seed)
    b = np.empty((n_rows, g.n_bins), dtype=np.complex128)
    for a in range(0, n_rows, 512):
        s = clean(a)
        s = s + sigma * rng.standard_normal(s.shape)
        b[a:a + 512] = (s @ op.E_re) + 1j * (s @ op.E_im)
    if op.dual:
        return b, sigma
    return b.reshape(g.n_angles, g.nz, g.n_bins), sigma
