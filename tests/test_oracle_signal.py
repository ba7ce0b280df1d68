"""Pins for oracle.signal: band DFT, Parseval, adjoint, harmonic structure."""
import numpy as np

from oracle import signal
from oracle.geometry import Geometry, kept_bins, detector_grid


def _geom(**kw):
    base = dict(nx=32, ny=32, nz=1, n_angles=1, n_t=2048, drive_cycles=2048 / 256 + 1 / 3,
                psf_width=2.0, harm_lo=1, harm_hi=15, half_band=2, op_scale=1.0)
    base.update(kw)
    return Geometry(**base)


def test_dft_equals_scaled_numpy_ifft():
    """Appendix A: s_hat_w = T^{-1/2} sum_j s_j e^{+i 2 pi w j / T} = sqrt(T) ifft(s)[w]."""
    g = _geom()
    rng = np.random.default_rng(1)
    s = rng.standard_normal((7, g.n_t))
    got = signal.compress(g, s)
    want = np.sqrt(g.n_t) * np.fft.ifft(s, axis=1)[:, kept_bins(g)]
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_parseval_full_spectrum():
    g = _geom(n_t=512, drive_cycles=5.3333, harm_hi=3)
    rng = np.random.default_rng(2)
    s = rng.standard_normal((3, g.n_t))
    E = signal.dft_matrix(g, bins=np.arange(g.n_t))
    sh = s @ E
    assert np.allclose((np.abs(sh) ** 2).sum(axis=1), (s ** 2).sum(axis=1), rtol=1e-13, atol=0)


def test_real_adjoint_of_band_dft_halves_energy():
    """For kept bins strictly inside (0, T/2): |Re(F_S^H z)|^2 = |z|^2 / 2."""
    g = _geom()
    rng = np.random.default_rng(3)
    z = rng.standard_normal(g.n_bins) + 1j * rng.standard_normal(g.n_bins)
    E = signal.dft_matrix(g)
    h = np.real(z[None, :] @ np.conj(E).T)[0]
    assert abs((h ** 2).sum() / (0.5 * (np.abs(z) ** 2).sum()) - 1.0) <= 1e-13


def _symmetric_source(g):
    rho = np.zeros(g.n_u)
    u = detector_grid(g)
    rho[np.argmin(np.abs(u - 0.5))] = 1.0
    rho[np.argmin(np.abs(u + 0.5))] = 1.0
    rho[np.argmin(np.abs(u - 6.5))] = 0.3
    rho[np.argmin(np.abs(u + 6.5))] = 0.3
    return rho


def test_half_wave_symmetry_even_harmonics_vanish():
    """Integer P and a source symmetric about u = 0: s(t + T/2P) = -s(t), so the
    spectrum holds odd harmonics only."""
    g = _geom(drive_cycles=8.0, half_band=0)
    b = signal.forward(g, _symmetric_source(g)[None, :])[0]
    harm = np.arange(g.harm_lo, g.harm_hi + 1)
    odd, even = np.abs(b[harm % 2 == 1]), np.abs(b[harm % 2 == 0])
    assert even.max() <= 1e-13 * odd.max()
    assert odd.min() > 1e-6 * odd.max()


def test_integer_drive_periods_leave_side_bins_empty():
    g = _geom(drive_cycles=8.0, half_band=2)
    rng = np.random.default_rng(4)
    b = signal.forward(g, rng.uniform(0, 1, (1, g.n_u)))[0].reshape(-1, 5)
    assert np.abs(b[:, [0, 1, 3, 4]]).max() <= 1e-13 * np.abs(b[:, 2]).max()


def test_non_integer_drive_periods_fill_side_bins():
    g = _geom()
    rng = np.random.default_rng(4)
    b = signal.forward(g, rng.uniform(0, 1, (1, g.n_u)))[0].reshape(-1, 5)
    assert np.abs(b[:3, [0, 1, 3, 4]]).max() > 1e-2 * np.abs(b[:3, 2]).max()


def test_signal_adjoint_identity():
    g = _geom(op_scale=0.37, rx_filter=np.exp(1j * np.linspace(0, 3, 75)) * np.linspace(0.5, 1.5, 75))
    rng = np.random.default_rng(6)
    r = rng.standard_normal((5, g.n_u))
    y = rng.standard_normal((5, g.n_bins)) + 1j * rng.standard_normal((5, g.n_bins))
    lhs = np.vdot(signal.forward(g, r), y).real
    rhs = np.vdot(r, signal.adjoint(g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_precomposed_line_matrix_equals_time_domain_path():
    g = _geom(op_scale=2.0)
    rng = np.random.default_rng(7)
    r = rng.standard_normal((9, g.n_u))
    a = signal.forward(g, r)
    b = r @ signal.line_matrix(g).T
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_receive_filter_is_fourier_diagonal():
    """Gamma = F^-1 D F (eq. DCmodel): filtering the time signal by the circular
    convolution whose spectrum is D, then compressing, equals compressing and
    multiplying the kept bins by D."""
    g = _geom(n_t=1024, drive_cycles=1024 / 256 + 1 / 3, harm_hi=8, half_band=1)
    rng = np.random.default_rng(8)
    s = rng.standard_normal(g.n_t)
    D = np.ones(g.n_t, dtype=complex)
    bins = kept_bins(g)
    Dk = np.exp(1j * rng.uniform(0, 2 * np.pi, len(bins))) * rng.uniform(0.5, 1.5, len(bins))
    D[bins] = Dk
    D[(g.n_t - bins) % g.n_t] = np.conj(Dk)        # real filter: Hermitian spectrum
    s_filt = np.real(np.fft.fft(np.fft.ifft(s) * D))  # the filter in the paper's +i convention
    g.rx_filter = Dk
    a = signal.compress(g, s)
    g.rx_filter = None
    b = signal.compress(g, s_filt)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_information_retained_in_unit_interval():
    g = _geom()
    rng = np.random.default_rng(9)
    s = signal.time_signal(g, rng.uniform(0, 1, (4, g.n_u)))
    info = signal.information_retained(s, kept_bins(g))
    assert np.all(info > 0.9) and np.all(info <= 1.0)


def test_raster_lines_follow_their_own_sweep_direction():
    """Every line's time signal is the derivative of its own magnetisation, with
    the sweep forward on even z-rows and backward on odd ones (the zig-zag,
    repeated for every angle): pins the class of each line independently of
    the kernel tables."""
    from oracle import physics
    g = _geom(nz=3, n_angles=2, n_t=512, drive_cycles=3.7, harm_hi=5, half_band=1,
              drive_amp=6.0, raster_sweep=11.0, op_scale=0.8)
    rng = np.random.default_rng(12)
    rho = rng.uniform(0.0, 1.0, (g.n_lines, g.n_u))
    s = signal.time_signal(g, rho)
    u = detector_grid(g)
    h = 1e-30
    t = np.arange(g.n_t) + 1j * h
    for line in range(g.n_lines):
        k = line % g.nz
        direction = 1.0 if k % 2 == 0 else -1.0
        dm = physics.magnetisation(t, g.drive_cycles, g.n_t, g.drive_amp, g.psf_width, u, rho[line],
                                   g.op_scale, g.raster_sweep, direction).imag / h
        assert np.max(np.abs(s[line] - dm)) <= 1e-12 * np.max(np.abs(dm))
    # the two directions really differ
    assert np.max(np.abs(signal.kernel(g, 0) - signal.kernel(g, 1))) > 1e-3 * np.max(np.abs(signal.kernel(g, 0)))


def test_raster_signal_adjoint_identity_and_precomposed():
    g = _geom(nz=4, n_angles=2, raster_sweep=9.0, op_scale=0.6)
    rng = np.random.default_rng(13)
    r = rng.standard_normal((g.n_lines, g.n_u))
    y = rng.standard_normal((g.n_lines, g.n_bins)) + 1j * rng.standard_normal((g.n_lines, g.n_bins))
    fr = signal.forward(g, r)
    lhs = np.vdot(fr, y).real
    rhs = np.vdot(r, signal.adjoint(g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    cl = np.tile(np.arange(g.nz) % 2, g.n_angles)
    pre = np.where((cl == 0)[:, None], r @ signal.line_matrix(g, 0).T, r @ signal.line_matrix(g, 1).T)
    assert np.max(np.abs(fr - pre)) <= 1e-13 * np.max(np.abs(fr))


def _brute_coupled_time_signal(g, rho):
    """s[m, k, n] = c_A v_n sum_{k', p} rho[m, k', p] h_xx(xi_n - u_p, k - k'),
    |k - k'| <= R, written out element by element."""
    from oracle import physics
    xi, v = physics.trajectory(g.n_t, g.drive_cycles, g.drive_amp)
    u = detector_grid(g)
    R = min(g.psf_rows, g.nz - 1)
    s = np.zeros((g.n_angles, g.nz, g.n_t))
    for m in range(g.n_angles):
        for k in range(g.nz):
            for k2 in range(g.nz):
                if abs(k - k2) > R:
                    continue
                for p in range(g.n_u):
                    h = physics.psf_xx(xi - u[p], k - k2, g.psf_width)
                    s[m, k] += g.op_scale * v * h * rho[m, k2, p]
    return s.reshape(g.n_lines, g.n_t)


def test_tensor_coupled_time_signal_brute_force():
    """The row-coupled time signal against the element formula, for the whole
    model (R >= nz - 1) and a truncated one; R = 0 is the collinear signal."""
    for R in (4, 1):
        g = _geom(nx=8, ny=8, nz=4, n_angles=2, n_t=128, drive_cycles=128 / 32 + 1 / 3, harm_hi=3,
                  half_band=1, psf_rows=R, op_scale=0.9)
        rho = np.random.default_rng(15).uniform(0, 1, (g.n_angles, g.nz, g.n_u))
        got = signal.time_signal(g, rho.reshape(g.n_lines, g.n_u))
        want = _brute_coupled_time_signal(g, rho)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), R
    g0 = _geom(nx=8, ny=8, nz=4, n_angles=2, n_t=128, drive_cycles=128 / 32 + 1 / 3, harm_hi=3, half_band=1)
    g1 = _geom(nx=8, ny=8, nz=4, n_angles=2, n_t=128, drive_cycles=128 / 32 + 1 / 3, harm_hi=3, half_band=1,
               psf_rows=1)
    rho = np.random.default_rng(16).uniform(0, 1, (g0.n_lines, g0.n_u))
    s0 = signal.time_signal(g0, rho)
    s1 = signal.time_signal(g1, rho)
    assert np.max(np.abs(s1 - s0)) > 1e-3 * np.max(np.abs(s0))      # the coupling is not negligible


def test_tensor_coupled_adjoint_and_precomposed():
    g = _geom(nz=6, n_angles=2, psf_rows=2, op_scale=0.5)
    rng = np.random.default_rng(17)
    r = rng.standard_normal((g.n_lines, g.n_u))
    y = rng.standard_normal((g.n_lines, g.n_bins)) + 1j * rng.standard_normal((g.n_lines, g.n_bins))
    fr = signal.forward(g, r)
    lhs = np.vdot(fr, y).real
    rhs = np.vdot(r, signal.adjoint(g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    pre = signal.coupled_apply(g, r, signal.row_matrices(g))
    assert np.max(np.abs(fr - pre)) <= 1e-13 * np.max(np.abs(fr))
