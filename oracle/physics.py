"""Oracle physics: Langevin function, its derivative, FFL trajectory.

Test infrastructure only (see ``oracle/__init__``).

Passages followed
-----------------
* Langevin function L(x) = coth(x) - 1/x: Appendix B (notation list).
* Magnetisation M = m rho L(beta |H|) H/|H| and the received signal
  s0 = d/dt int b^T M: Sec. 1.2, eq. s01; its evaluated form
  s0 = m int rho b^T h(xi(t) - x) v(t) dx with v = xi': eq. reals0.
* Tensor PSF h(x): Appendix B, eq. PSF.  On the FFL's own row, with drive and
  receive coil along the fast axis, G x is parallel to the drive direction, so
  the transverse L(.)/|Gx| term is zero and the PSF reduces to the scalar
  h(u) = L'(u/w)/w with w = H_sat/G0 in voxels (collinear reduction).
* Sinusoidal drive H_D = A sin(2 pi f0 t): eq. HD; FFL position
  xi(t) = a sin(phi(t)) follows from eq. H1 (H = G(xi - x)).
* Tensor PSF across z-rows (Appendix B, eq. PSF, in the xz-plane where the 2D
  FFL model of Sec. 2.2 acts): with the in-plane gradient of equal magnitude g
  on both axes (zero trace with the FFL direction's zero gradient; the sign
  pattern does not change the xx entry), drive and receive coil along the fast
  axis, and d = (du, dz) the offset of the line centre from a point,
  h_xx(d) = L'(r/w)/w du^2/r^2 + L(r/w) dz^2/r^3 with r = |d| and w = H_sat/g.
  On the line's own row (dz = 0) it is the collinear L'(|du|/w)/w.
* Raster (Sec. 3.1, the scanner's acquisition): a slow focus field moves the
  line across the field of view in a zig-zag, back and forth along the fast
  axis.  Reading: during one FFL line the centre moves at constant speed over
  ``sweep`` voxels, c(t) = direction * sweep * (t/T - 1/2), in the direction
  that alternates from line to line, and adds to the drive.

Pins (tests/test_oracle_physics.py): L and L' against mpmath at 40 digits;
the velocity and PSF chain against a complex-step derivative of the
magnetisation; the PSF full width at half maximum.
"""
import numpy as np

# Series coefficients of L'(x) = 1/3 - x^2/15 + 2x^4/189 - x^6/675 + 2x^8/10395,
# i.e. the term-by-term derivative of L(x) = sum_n 2^{2n} B_{2n} x^{2n-1}/(2n)!.
_LP_SERIES = (1.0 / 3.0, -1.0 / 15.0, 2.0 / 189.0, -1.0 / 675.0, 2.0 / 10395.0)
_L_SERIES = (1.0 / 3.0, -1.0 / 45.0, 2.0 / 945.0, -1.0 / 4725.0, 2.0 / 93555.0)
_SERIES_CUT = 0.1


def langevin(x):
    """L(x) = coth(x) - 1/x, real or complex argument (Appendix B).

    |x| < 0.1 uses the odd Taylor series (relative error below 1e-14 there);
    0.1 <= |x| < 2 the ratio (x cosh x - sinh x)/(x sinh x) with a series
    numerator (no cancellation); elsewhere coth x - 1/x.  Complex arguments are supported so that the
    complex-step derivative test can differentiate it.
    """
    x = np.asarray(x)
    out = np.empty(x.shape, dtype=np.result_type(x.dtype, np.float64))
    small = np.abs(x) < _SERIES_CUT
    xs = x[small]
    x2 = xs * xs
    acc = np.zeros_like(xs)
    for c in reversed(_L_SERIES):
        acc = acc * x2 + c
    out[small] = xs * acc
    mid = (~small) & (np.abs(x) < 2.0)
    xm = x[mid]
    out[mid] = _xcosh_minus_sinh(xm) / (xm * np.sinh(xm))
    big = np.abs(x) >= 2.0
    xl = x[big]
    out[big] = 1.0 / np.tanh(xl) - 1.0 / xl
    return out


def _xcosh_minus_sinh(x):
    """x cosh x - sinh x = sum_{n>=1} 2n x^{2n+1} / (2n+1)!, free of cancellation."""
    x2 = x * x
    term = x * x2 / 6.0          # x^3 / 3!
    acc = 2.0 * term
    n = 1
    while True:
        term = term * x2 / ((2 * n + 2) * (2 * n + 3))
        n += 1
        acc = acc + 2 * n * term
        if np.all(np.abs(2 * n * term) <= 1e-18 * np.abs(acc)):
            return acc


def _sinh_minus_x(x):
    """sinh(x) - x summed from its Taylor series x^3/3! + x^5/5! + ... (|x| < 1)."""
    x2 = x * x
    term = x * x2 / 6.0
    acc = term.copy()
    n = 3
    while True:
        term = term * x2 / ((n + 1) * (n + 2))
        n += 2
        acc = acc + term
        if np.all(np.abs(term) <= 1e-18 * np.abs(acc)):
            return acc


def langevin_deriv(x):
    """L'(x) = 1/x^2 - 1/sinh^2(x), evaluated without cancellation.

    * |x| < 0.1: even Taylor series (five terms, relative error <= 7e-15).
    * 0.1 <= |x| < 1: (sinh x - x)(sinh x + x) / (x^2 sinh^2 x), with
      sinh x - x from its own series, so nothing cancels.
    * |x| >= 1: 1/x^2 - 4 e^{-2|x|} / (1 - e^{-2|x|})^2 (no overflow).
    L' is even, so the work is done on |x|.
    """
    x = np.abs(np.asarray(x, dtype=np.float64))
    out = np.empty_like(x)
    a = x < _SERIES_CUT
    x2 = x[a] ** 2
    acc = np.zeros_like(x2)
    for c in reversed(_LP_SERIES):
        acc = acc * x2 + c
    out[a] = acc
    b = (x >= _SERIES_CUT) & (x < 1.0)
    xb = x[b]
    sh = np.sinh(xb)
    out[b] = _sinh_minus_x(xb) * (sh + xb) / (xb * xb * sh * sh)
    c = x >= 1.0
    xc = x[c]
    e = np.exp(-2.0 * xc)
    out[c] = 1.0 / (xc * xc) - 4.0 * e / (1.0 - e) ** 2
    return out


def psf_xx(du, dz, psf_width):
    """h_xx(du, dz) of the tensor PSF (see the module notes), real du, one dz."""
    du = np.asarray(du, dtype=np.float64)
    w = psf_width
    if dz == 0:
        return langevin_deriv(du / w) / w
    r2 = du * du + float(dz) * float(dz)
    r = np.sqrt(r2)
    return langevin_deriv(r / w) / w * (du * du / r2) + langevin(r / w) * (float(dz) * float(dz) / (r2 * r))


def magnetisation_x(t, drive_cycles, n_t, drive_amp, psf_width, u, rho_line, op_scale, dz):
    """x-component of the magnetisation of a row dz away from the line,
    m_x(t) = c_A sum_p rho_p L(|d|/w) du/|d|, d = (xi(t) - u_p, dz): the unit
    vector G d/|G d| of eq. PSF's derivation in the xz-plane.  t real or
    complex; used only to pin psf_xx through s0 = dm/dt (eq. s01)."""
    t = np.asarray(t)
    omega = 2.0 * np.pi * drive_cycles / n_t
    du = drive_amp * np.sin(omega * t)[..., None] - np.asarray(u)[None, :]
    if dz == 0:
        return op_scale * (langevin(du / psf_width) * np.asarray(rho_line)[None, :]).sum(axis=-1)
    r = np.sqrt(du * du + float(dz) * float(dz))
    return op_scale * (langevin(r / psf_width) * du / r * np.asarray(rho_line)[None, :]).sum(axis=-1)


def trajectory(n_t, drive_cycles, drive_amp, sweep=0.0, direction=1.0):
    """FFL position xi_n and velocity v_n at samples n = 0..T-1.

    phi_n = 2 pi P n / T, xi_n = a sin(phi_n), v_n = a (2 pi P / T) cos(phi_n):
    the sinusoidal drive of eq. HD moves the line as xi(t) (eq. H1), and the
    velocity multiplier V of Table 1 is v = xi' (eq. reals0), with time in
    units of one sample.  A raster adds the focus-field shift
    c_n = direction * sweep * (n/T - 1/2) to xi_n and its constant speed
    direction * sweep / T to v_n.
    """
    n = np.arange(n_t, dtype=np.float64)
    omega = 2.0 * np.pi * drive_cycles / n_t
    xi = drive_amp * np.sin(omega * n) + direction * sweep * (n / n_t - 0.5)
    v = drive_amp * omega * np.cos(omega * n) + direction * sweep / n_t
    return xi, v


def psf_kernel(n_t, drive_cycles, drive_amp, psf_width, u, op_scale, sweep=0.0, direction=1.0):
    """K[n, p] = c_A * v_n * L'((xi_n - u_p)/w) / w, shape (T, Nu).

    The matrix of the fused E H V operators of eq. svecHPF restricted to one
    FFL row (collinear PSF), with B = I and all physical constants in c_A.
    """
    xi, v = trajectory(n_t, drive_cycles, drive_amp, sweep, direction)
    arg = (xi[:, None] - np.asarray(u, dtype=np.float64)[None, :]) / psf_width
    return op_scale * v[:, None] * langevin_deriv(arg) / psf_width


def magnetisation(t, drive_cycles, n_t, drive_amp, psf_width, u, rho_line, op_scale, sweep=0.0, direction=1.0):
    """m(t) = c_A * sum_p rho_p L((xi(t) - u_p)/w), t real or complex.

    Used only to pin the signal chain: s0 = dm/dt (eq. s01 -> eq. reals0).
    """
    t = np.asarray(t)
    omega = 2.0 * np.pi * drive_cycles / n_t
    xi = drive_amp * np.sin(omega * t) + direction * sweep * (t / n_t - 0.5)
    arg = (xi[..., None] - np.asarray(u)[None, :]) / psf_width
    return op_scale * (langevin(arg) * np.asarray(rho_line)[None, :]).sum(axis=-1)
