"""Pins for oracle.physics: Langevin L, L', trajectory/velocity, PSF shape."""
import mpmath
import numpy as np
import pytest

from oracle import physics, signal
from oracle.geometry import Geometry, detector_grid


@pytest.fixture(autouse=True)
def _mp_precision():
    """40-digit mpmath for every test of this module, whatever other modules set."""
    with mpmath.workdps(40):
        yield


def _mp_L(x):
    x = mpmath.mpf(x)
    if x == 0:
        return mpmath.mpf(0)
    return mpmath.coth(x) - 1 / x


def _mp_Lp(x):
    x = mpmath.mpf(x)
    if x == 0:
        return mpmath.mpf(1) / 3
    return 1 / x ** 2 - 1 / mpmath.sinh(x) ** 2


GRID = np.concatenate([
    np.linspace(-30, 30, 601),
    [0.0, 1e-12, -1e-9, 1e-6, -1e-6, 3e-4, 0.0999999, 0.1, 0.1000001, 0.5, 0.999999, 1.0, 1.000001, 700.0, -800.0],
    np.geomspace(1e-8, 25, 97),
])


def test_langevin_derivative_vs_mpmath():
    got = physics.langevin_deriv(GRID)
    want = np.array([float(_mp_Lp(x)) for x in GRID])
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() <= 1e-14, (GRID[rel.argmax()], rel.max())


def test_langevin_vs_mpmath():
    grid = GRID[np.abs(GRID) > 0]
    got = physics.langevin(grid)
    want = np.array([float(_mp_L(x)) for x in grid])
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() <= 1e-14, (grid[rel.argmax()], rel.max())


def test_langevin_is_odd_derivative_is_even():
    x = np.linspace(0.01, 20, 333)
    assert np.array_equal(physics.langevin(-x), -physics.langevin(x))
    assert np.array_equal(physics.langevin_deriv(-x), physics.langevin_deriv(x))


def test_velocity_psf_chain_is_time_derivative_of_magnetisation():
    """s_n must equal dm/dt at t_n, m(t) = c_A sum_p rho_p L((xi(t)-u_p)/w).

    Complex-step derivative: Im m(t + i h) / h is exact to rounding, so this
    checks v = xi' (velocity operator V), the 1/w PSF scale and L' against L.
    """
    g = Geometry(nx=24, ny=24, nz=1, n_angles=1, n_t=512, drive_cycles=3.7, psf_width=2.5,
                 harm_lo=1, harm_hi=5, half_band=1, op_scale=1.7)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.0, 1.0, g.n_u)
    u = detector_grid(g)
    s = signal.time_signal(g, rho[None, :])[0]
    h = 1e-30
    t = np.arange(g.n_t) + 1j * h
    dm = physics.magnetisation(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, u, rho,
                               g.op_scale).imag / h
    assert np.max(np.abs(s - dm)) <= 1e-12 * np.max(np.abs(dm))


def test_psf_single_source_and_fwhm():
    """A single source gives s_n / v_n = c_A L'((xi_n - u)/w)/w; FWHM of L' is 4.1610 w."""
    w = 2.0
    x_half = mpmath.findroot(lambda x: _mp_Lp(x) - mpmath.mpf(1) / 6, 2.0)
    fwhm = 2 * float(x_half)
    assert abs(fwhm - 4.1610) < 1e-4
    # the oracle's L' agrees with the half-maximum point to 1e-14
    assert abs(physics.langevin_deriv(np.array([float(x_half)]))[0] - 1 / 6) < 1e-14
    g = Geometry(nx=16, ny=16, nz=1, n_angles=1, n_t=1024, drive_cycles=4.3333, psf_width=w,
                 harm_lo=1, harm_hi=3, half_band=1, op_scale=0.9)
    rho = np.zeros(g.n_u)
    rho[5] = 1.0
    s = signal.time_signal(g, rho[None, :])[0]
    xi, v = physics.trajectory(g.n_t, g.drive_cycles, g.drive_amp)
    u5 = detector_grid(g)[5]
    ok = np.abs(v) > 1e-3
    want = g.op_scale * np.array([float(_mp_Lp((a - u5) / w)) for a in xi[ok]]) / w
    assert np.max(np.abs(s[ok] / v[ok] - want)) <= 1e-12 * np.max(np.abs(want))


def test_trajectory_sweep():
    xi, v = physics.trajectory(4096, 16.0, 8.0)
    assert abs(xi.max() - 8.0) < 1e-12 and abs(xi.min() + 8.0) < 1e-12
    # closed-form velocity: a * 2 pi P / T at phase 0
    assert abs(v[0] - 8.0 * 2 * np.pi * 16.0 / 4096) < 1e-15


def test_raster_velocity_psf_chain_is_time_derivative_of_magnetisation():
    """With the raster's focus-field shift c(t) = +-S (t/T - 1/2) added to the
    drive, s_n must still be dm/dt (complex step): this pins the shift and its
    constant speed +-S/T in v, for both sweep directions."""
    for direction in (1.0, -1.0):
        g = Geometry(nx=24, ny=24, nz=1, n_angles=1, n_t=512, drive_cycles=3.7, psf_width=2.5,
                     harm_lo=1, harm_hi=5, half_band=1, op_scale=1.3, drive_amp=4.0, raster_sweep=17.0)
        rng = np.random.default_rng(11)
        rho = rng.uniform(0.0, 1.0, g.n_u)
        u = detector_grid(g)
        K = physics.psf_kernel(g.n_t, g.drive_cycles, g.drive_amp, g.psf_width, u, g.op_scale,
                               g.raster_sweep, direction)
        s = rho @ K.T
        h = 1e-30
        t = np.arange(g.n_t) + 1j * h
        dm = physics.magnetisation(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, u, rho,
                                   g.op_scale, g.raster_sweep, direction).imag / h
        assert np.max(np.abs(s - dm)) <= 1e-12 * np.max(np.abs(dm))


def test_raster_trajectory_closed_form():
    """Centre -S/2 at n = 0 moving at S/T per sample (forward), mirrored backward."""
    T, S = 4096, 40.0
    xi0, v0 = physics.trajectory(T, 16.0, 8.0)
    xi_f, v_f = physics.trajectory(T, 16.0, 8.0, S, 1.0)
    xi_b, v_b = physics.trajectory(T, 16.0, 8.0, S, -1.0)
    n = np.arange(T)
    assert np.max(np.abs(xi_f - xi0 - S * (n / T - 0.5))) < 1e-12
    assert np.max(np.abs(xi_b - xi0 + S * (n / T - 0.5))) < 1e-12
    assert abs(xi_f[0] - (xi0[0] - S / 2)) < 1e-12
    assert np.max(np.abs(v_f - v0 - S / T)) < 1e-15 and np.max(np.abs(v_b - v0 + S / T)) < 1e-15


def test_tensor_psf_is_derivative_of_magnetisation_x():
    """Rows dz away from the line: s_n = c_A v_n sum_p rho_p h_xx(xi_n - u_p, dz)
    must be d/dt of the x-component of the magnetisation c_A sum rho L(|d|/w)
    d_x/|d| (complex step), which pins both terms of eq. PSF's xx entry."""
    g = Geometry(nx=24, ny=24, nz=1, n_angles=1, n_t=512, drive_cycles=3.7, psf_width=2.5,
                 harm_lo=1, harm_hi=5, half_band=1, op_scale=1.1)
    rng = np.random.default_rng(14)
    rho = rng.uniform(0.0, 1.0, g.n_u)
    u = detector_grid(g)
    h = 1e-30
    t = np.arange(g.n_t) + 1j * h
    for dz in (0, 1, 2, 5, 9):
        s = rho @ signal.kernel_row(g, dz).T
        dm = physics.magnetisation_x(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, u, rho,
                                     g.op_scale, dz).imag / h
        assert np.max(np.abs(s - dm)) <= 1e-12 * np.max(np.abs(dm)), dz


def test_tensor_psf_closed_forms():
    """h_xx(0, dz) = L(|dz|/w)/|dz| (only the transverse term), symmetry in du
    and dz, the collinear kernel on the row itself, and the saturated far
    field h_xx(0, dz) -> 1/|dz|."""
    w = 2.0
    for dz in (1, 3, 7):
        want = float(_mp_L(dz / w)) / dz
        assert abs(physics.psf_xx(np.array([0.0]), dz, w)[0] - want) <= 1e-14 * want
        assert abs(physics.psf_xx(np.array([0.0]), -dz, w)[0] - want) <= 1e-14 * want
    du = np.linspace(-9, 9, 37)
    assert np.array_equal(physics.psf_xx(du, 2, w), physics.psf_xx(-du, 2, w))
    assert np.max(np.abs(physics.psf_xx(du, 0, w) - physics.langevin_deriv(du / w) / w)) == 0.0
    far = physics.psf_xx(np.array([0.0]), 400, w)[0]
    assert abs(far * 400 - 1.0) < 2 * w / 400
