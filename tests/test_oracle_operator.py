"""Pins for oracle.operator: the full A and A^T."""
import math

import mpmath
import numpy as np
import pytest

from oracle import operator, projector
from oracle.geometry import Geometry


@pytest.fixture(autouse=True)
def _mp_precision():
    """30-digit mpmath for every test of this module, whatever other modules set."""
    with mpmath.workdps(30):
        yield


def _small():
    # 8^3 volume, 4 angles, T = 256 with P = 5.3333 and bands k = 1..6, +-1
    return Geometry(nx=8, ny=8, nz=8, n_angles=4, n_t=256, drive_cycles=5.3333, psf_width=1.5,
                    harm_lo=1, harm_hi=6, half_band=1, op_scale=0.8,
                    rx_filter=np.exp(0.3j * np.arange(18)) * (1 + 0.05 * np.arange(18)))


def _hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def _element_matrix(g):
    """A[(m,k,j), (k',y,x)] = delta_{kk'} sum_p W_m(p; x, y) C[j, p], written from scratch:

    W_m(p; x, y) = sum_q hat(X_pq - X_x) hat(Y_pq - Y_y)         (bilinear Riemann sum)
    C[j, p] = D_j T^{-1/2} sum_n e^{+2 pi i w_j n / T} c_A v_n L'((xi_n - u_p)/w)/w
    with L' from mpmath and the bins floor(k P + 1/2) + d.
    """
    n = g.nx
    nr = 12
    yq = np.arange(nr) - (nr - 1) / 2
    u = np.arange(n) - (n - 1) / 2
    W = []
    for t in g.theta:
        X = u[:, None] * math.cos(t) + yq[None, :] * math.sin(t)
        Y = -u[:, None] * math.sin(t) + yq[None, :] * math.cos(t)
        W.append(np.einsum("pqi,pqj->pji", _hat(X[:, :, None] - u[None, None, :]),
                           _hat(Y[:, :, None] - u[None, None, :])).reshape(n, n * n))
    T, P, a, w = g.n_t, g.drive_cycles, g.drive_amp, g.psf_width
    bins = [math.floor(k * P + 0.5) + d for k in range(g.harm_lo, g.harm_hi + 1)
            for d in range(-g.half_band, g.half_band + 1)]
    C = np.zeros((len(bins), n), dtype=complex)
    for nn in range(T):
        ph = 2 * math.pi * P * nn / T
        xi, v = a * math.sin(ph), a * 2 * math.pi * P / T * math.cos(ph)
        k_row = np.array([float(1 / mpmath.mpf((xi - up) / w) ** 2 - 1 / mpmath.sinh((xi - up) / w) ** 2)
                          if abs(xi - up) > 1e-12 else 1 / 3 for up in u])
        k_row *= g.op_scale * v / w
        e = np.exp(2j * math.pi * ((np.array(bins) * nn) % T) / T) / math.sqrt(T)
        C += e[:, None] * k_row[None, :]
    C *= np.asarray(g.rx_filter)[:, None]
    nb = len(bins)
    A = np.zeros((g.n_angles, g.nz, nb, g.nz, n * n), dtype=complex)
    for m in range(g.n_angles):
        blk = C @ W[m]                                   # (nb, n*n)
        for k in range(g.nz):
            A[m, k, :, k, :] = blk
    return A.reshape(g.n_angles * g.nz * nb, g.nz * n * n)


def test_brute_force_dense_forward_and_adjoint():
    g = _small()
    A = _element_matrix(g)
    op = operator.Operator(g)
    cols = np.empty_like(A)
    for c in range(A.shape[1]):
        e = np.zeros(A.shape[1])
        e[c] = 1.0
        cols[:, c] = op.forward(e.reshape(g.nz, g.ny, g.nx)).ravel()
    assert np.max(np.abs(cols - A)) <= 1e-13 * np.max(np.abs(A))
    rng = np.random.default_rng(3)
    y = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    want = np.real(np.conj(A).T @ y)
    got = op.adjoint(y.reshape(g.n_angles, g.nz, g.n_bins)).ravel()
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_adjoint_identity_1e12():
    """<A x, y> = <x, A^T y> in the inner product Re(u^H v)."""
    for g in (_small(),
              Geometry(nx=32, ny=32, nz=32, n_angles=8, n_t=2048, drive_cycles=2048 / 256 + 1 / 3,
                       psf_width=2.0, harm_lo=1, harm_hi=15, half_band=2, op_scale=0.02)):
        rng = np.random.default_rng(21)
        x = rng.standard_normal((g.nz, g.ny, g.nx))
        y = rng.standard_normal((g.n_angles, g.nz, g.n_bins)) + 1j * rng.standard_normal((g.n_angles, g.nz, g.n_bins))
        lhs = np.vdot(operator.forward(g, x), y).real
        rhs = np.vdot(x, operator.adjoint(g, y))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_precomposed_equals_time_domain():
    g = _small()
    rng = np.random.default_rng(4)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    a = operator.forward(g, x)
    b = operator.forward(g, x, precomposed=True)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_z_separability_exact_zeros():
    g = _small()
    x = np.zeros((g.nz, g.ny, g.nx))
    x[3] = np.random.default_rng(5).uniform(0, 1, (g.ny, g.nx))
    b = operator.forward(g, x)
    assert np.all(b[:, [0, 1, 2, 4, 5, 6, 7], :] == 0)
    assert np.all(np.abs(b[:, 3, :]) > 0)


def test_one_slice_norm_equals_full_norm():
    g = _small()
    a = operator.op_norm(g, one_slice=True)
    b = operator.op_norm(g, one_slice=False)
    assert abs(a - b) <= 1e-9 * a
    gn = operator.normalised(g)
    assert abs(operator.op_norm(gn) - 1.0) <= 1e-9


def test_make_data_noise_free_equals_forward():
    g = _small()
    rng = np.random.default_rng(6)
    x = rng.uniform(0, 1, (g.nz, g.ny, g.nx))
    b, sigma = operator.make_data(g, x, 0.0, 1)
    assert sigma == 0.0
    a = operator.forward(g, x)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_raster_operator_adjoint_and_two_slice_norm():
    """Raster scan (odd nz): adjoint identity to 1e-12, the precomposed and
    time-domain paths agree, and the norm on two slices (one per sweep
    direction) equals the full-volume norm."""
    g = _small()
    g = Geometry(**{**{k: getattr(g, k) for k in g.__dataclass_fields__}, "nz": 5, "raster_sweep": 7.0})
    rng = np.random.default_rng(21)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    y = rng.standard_normal((g.n_angles, g.nz, g.n_bins)) + 1j * rng.standard_normal((g.n_angles, g.nz, g.n_bins))
    ax = operator.forward(g, x)
    lhs = np.vdot(ax, y).real
    rhs = np.vdot(x, operator.adjoint(g, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.max(np.abs(operator.forward(g, x, precomposed=True) - ax)) <= 1e-12 * np.max(np.abs(ax))
    a = operator.op_norm(g, one_slice=True)
    b = operator.op_norm(g, one_slice=False)
    assert abs(a - b) <= 1e-9 * a


def test_tensor_operator_adjoint_and_precomposed():
    """Rows coupled by the tensor PSF: adjoint identity to 1e-12 and the
    precomposed per-offset form equal to the time-domain one."""
    g = _small()
    g = Geometry(**{**{k: getattr(g, k) for k in g.__dataclass_fields__}, "nz": 5, "psf_rows": 2})
    rng = np.random.default_rng(22)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    y = rng.standard_normal((g.n_angles, g.nz, g.n_bins)) + 1j * rng.standard_normal((g.n_angles, g.nz, g.n_bins))
    ax = operator.forward(g, x)
    assert abs(np.vdot(ax, y).real - np.vdot(x, operator.adjoint(g, y))) <= 1e-12 * abs(np.vdot(ax, y).real)
    assert np.max(np.abs(operator.forward(g, x, precomposed=True) - ax)) <= 1e-12 * np.max(np.abs(ax))
    ya = operator.adjoint(g, y)
    assert np.max(np.abs(operator.adjoint(g, y, precomposed=True) - ya)) <= 1e-12 * np.max(np.abs(ya))
    op = operator.Operator(g)
    assert np.max(np.abs(op.forward(x) - ax)) <= 1e-12 * np.max(np.abs(ax))


def _dual(nz=5, **kw):
    g = _small()
    return Geometry(**{**{k: getattr(g, k) for k in g.__dataclass_fields__}, "nz": nz, "drive_axes": 2,
                       "drive_amp_z": None, **kw})


def test_dual_drive_lines_are_derivatives_of_their_magnetisation():
    """Every x-drive line's signal is dm/dt along u of row (m, k); every z-drive
    line's is dm/dt along z of column (m, p) with amplitude a_z, at data line
    M*Nz + m*Nu + p (complex step): pins the z-lines' layout and their PSF."""
    from oracle import physics, signal
    from oracle.geometry import detector_grid
    g = _dual(nz=6)
    rng = np.random.default_rng(23)
    rt = rng.uniform(0, 1, (g.n_angles, g.nz, g.n_u))
    op = operator.Operator(g)
    s = np.concatenate([rt.reshape(g.n_lines, g.n_u) @ op.K[0].T, signal.z_lines(g, rt) @ op.Kz.T])
    h = 1e-30
    t = np.arange(g.n_t) + 1j * h
    zg = np.arange(g.nz) - (g.nz - 1) / 2.0
    for m in range(g.n_angles):
        for k in range(g.nz):
            dm = physics.magnetisation(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, detector_grid(g),
                                       rt[m, k], g.op_scale).imag / h
            assert np.max(np.abs(s[m * g.nz + k] - dm)) <= 1e-12 * np.max(np.abs(dm))
        for p in range(g.n_u):
            dm = physics.magnetisation(t, g.drive_cycles, g.n_t, g.nz / 2.0, g.psf_width, zg, rt[m, :, p],
                                       g.op_scale).imag / h
            assert np.max(np.abs(s[g.n_lines + m * g.n_u + p] - dm)) <= 1e-12 * np.max(np.abs(dm))


def test_dual_drive_adjoint_precomposed_and_data():
    g = _dual(nz=5)
    rng = np.random.default_rng(24)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    y = rng.standard_normal((g.n_data_lines, g.n_bins)) + 1j * rng.standard_normal((g.n_data_lines, g.n_bins))
    ax = operator.forward(g, x)
    assert ax.shape == (g.n_data_lines, g.n_bins)
    lhs = np.vdot(ax, y).real
    assert abs(lhs - np.vdot(x, operator.adjoint(g, y))) <= 1e-12 * abs(lhs)
    assert np.max(np.abs(operator.forward(g, x, precomposed=True) - ax)) <= 1e-12 * np.max(np.abs(ax))
    b, sigma = operator.make_data(g, np.abs(x), 0.0, 1)
    assert sigma == 0.0 and np.max(np.abs(b - operator.forward(g, np.abs(x)))) <= 1e-12 * np.max(np.abs(b))
    # the x-drive half is the single-drive operator
    g1 = _dual(nz=5, drive_axes=1)
    ax1 = operator.forward(g1, x).reshape(g.n_lines, g.n_bins)
    assert np.max(np.abs(ax[:g.n_lines] - ax1)) <= 1e-13 * np.max(np.abs(ax1))


def test_dual_drive_tensor_lines_are_derivatives_of_their_magnetisation():
    """Both scans under the tensor PSF (Sec. 3.1 with Appendix B eq. PSF): every
    x-drive line's signal is the time derivative of the x-magnetisation of the
    z-rows within R of it, and every z-drive line's (m, p) that of the
    z-magnetisation of the detector columns within R of p -- the same tensor
    entry with the drive axis exchanged, m_z = c_A sum rho L(r/w) dz/r,
    r = |(xi_z - z_k, p' - p)| -- at data line M*Nz + m*Nu + p (complex step)."""
    from oracle import physics, signal
    from oracle.geometry import detector_grid
    for R in (2, 7):
        g = _dual(nz=5, psf_rows=R)
        rng = np.random.default_rng(31)
        rt = rng.uniform(0, 1, (g.n_angles, g.nz, g.n_u))
        op = operator.Operator(g)
        s_x = signal.coupled_apply(g, rt.reshape(g.n_lines, g.n_u), op.Kd)
        s_z = signal.coupled_apply(g, signal.z_lines(g, rt), op.Mz, per=g.n_u)
        h = 1e-30
        t = np.arange(g.n_t) + 1j * h
        zg = np.arange(g.nz) - (g.nz - 1) / 2.0
        Rx, Rz = min(R, g.nz - 1), min(R, g.n_u - 1)
        for m in range(g.n_angles):
            for k in range(g.nz):
                dm = sum(physics.magnetisation_x(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, detector_grid(g),
                                                 rt[m, k2], g.op_scale, k - k2).imag / h
                         for k2 in range(g.nz) if abs(k - k2) <= Rx)
                assert np.max(np.abs(s_x[m * g.nz + k] - dm)) <= 1e-12 * np.max(np.abs(dm))
            for p in range(g.n_u):
                dm = sum(physics.magnetisation_x(t, g.drive_cycles, g.n_t, g.nz / 2.0, g.psf_width, zg,
                                                 rt[m, :, p2], g.op_scale, p - p2).imag / h
                         for p2 in range(g.n_u) if abs(p - p2) <= Rz)
                assert np.max(np.abs(s_z[m * g.n_u + p] - dm)) <= 1e-12 * np.max(np.abs(dm)), (R, m, p)


def test_dual_drive_tensor_operator():
    """Both scans under the tensor PSF: adjoint identity to 1e-12, precomposed =
    time-domain, noise-free data = A x, the x-drive half equal to the
    single-drive tensor operator, and the z-drive table at zero column offset
    the collinear z-drive PSF (closed form h(along, 0) = L'(along/w)/w); the
    coupling across columns is not negligible."""
    from oracle import signal
    g = _dual(nz=5, psf_rows=2)
    rng = np.random.default_rng(32)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    y = rng.standard_normal((g.n_data_lines, g.n_bins)) + 1j * rng.standard_normal((g.n_data_lines, g.n_bins))
    ax = operator.forward(g, x)
    lhs = np.vdot(ax, y).real
    assert abs(lhs - np.vdot(x, operator.adjoint(g, y))) <= 1e-12 * abs(lhs)
    assert np.max(np.abs(operator.forward(g, x, precomposed=True) - ax)) <= 1e-12 * np.max(np.abs(ax))
    ya = operator.adjoint(g, y)
    assert np.max(np.abs(operator.adjoint(g, y, precomposed=True) - ya)) <= 1e-12 * np.max(np.abs(ya))
    b, sigma = operator.make_data(g, np.abs(x), 0.0, 1)
    assert sigma == 0.0 and np.max(np.abs(b - operator.forward(g, np.abs(x)))) <= 1e-12 * np.max(np.abs(b))
    gx = _small()
    gx = Geometry(**{**{k: getattr(gx, k) for k in gx.__dataclass_fields__}, "nz": 5, "psf_rows": 2})
    ax1 = operator.forward(gx, x).reshape(g.n_lines, g.n_bins)
    assert np.max(np.abs(ax[:g.n_lines] - ax1)) <= 1e-13 * np.max(np.abs(ax1))
    Kz0 = signal.kernel_z_column(g, 0)
    assert np.max(np.abs(Kz0 - signal.kernel_z(g))) <= 1e-14 * np.max(np.abs(Kz0))
    g0 = _dual(nz=5)
    az0 = operator.forward(g0, x)[g.n_lines:]
    assert np.linalg.norm(ax[g.n_lines:] - az0) > 1e-3 * np.linalg.norm(az0)
