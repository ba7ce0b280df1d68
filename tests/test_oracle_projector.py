"""Pins for oracle.projector: Gaussian closed form, convergence order, adjoint."""
import math

import numpy as np
import pytest

from oracle import projector
from oracle.geometry import Geometry, detector_grid, voxel_centres


def _geom(n, theta, nz=1):
    return Geometry(nx=n, ny=n, nz=nz, n_angles=len(theta), n_t=512, drive_cycles=3.3333,
                    psf_width=2.0, harm_lo=1, harm_hi=3, half_band=1, theta=np.asarray(theta, float))


def _gauss_volume(g, c, sigma, amp=1.0, zc=None):
    X = voxel_centres(g.nx)[None, None, :]
    Y = voxel_centres(g.ny)[None, :, None]
    Z = np.arange(g.nz, dtype=float)[:, None, None]
    zc = 0.0 if zc is None else zc
    return amp * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - zc) ** 2) / (2 * sigma ** 2))


def _closed_form(g, c, sigma, amp=1.0, zc=None):
    """Line integral of the isotropic Gaussian along the ray through detector u at angle theta:
    a sqrt(2 pi) sigma exp(-(u - u_c)^2 / 2 sigma^2) with u_c = c_X cos t - c_Y sin t."""
    u = detector_grid(g)
    Z = np.arange(g.nz, dtype=float)
    zc = 0.0 if zc is None else zc
    out = np.empty((g.n_angles, g.nz, g.n_u))
    for m, t in enumerate(g.theta):
        uc = c[0] * math.cos(t) - c[1] * math.sin(t)
        prof = amp * math.sqrt(2 * math.pi) * sigma * np.exp(-(u - uc) ** 2 / (2 * sigma ** 2))
        out[m] = np.exp(-(Z - zc) ** 2 / (2 * sigma ** 2))[:, None] * prof[None, :]
    return out


@pytest.mark.parametrize("theta", [0.0, math.pi / 2])
def test_gaussian_exact_on_axis_angles(theta):
    """At 0 and 90 degrees the samples sit on voxel centres: the Riemann sum of a
    Gaussian with >= 8 sigma of room equals its integral to ~1e-14."""
    g = _geom(48, [theta], nz=3)
    c, sigma = (0.37, -1.21), 2.0
    vol = _gauss_volume(g, c, sigma, zc=1.0)
    got = projector.project(g, vol)
    want = _closed_form(g, c, sigma, zc=1.0)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_gaussian_second_order_at_oblique_angles():
    """Bilinear sampling converges at second order: doubling sigma and N (one grid
    refinement) divides the relative L2 error by about 4."""
    thetas = [math.pi / 7, 0.3 * math.pi, 0.61 * math.pi]
    errs = []
    for n, sigma in ((32, 1.5), (64, 3.0), (128, 6.0)):
        g = _geom(n, thetas)
        c = (0.11 * n / 32, -0.07 * n / 32)
        got = projector.project(g, _gauss_volume(g, c, sigma))
        want = _closed_form(g, c, sigma)
        errs.append(np.linalg.norm(got - want) / np.linalg.norm(want))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 <= r1 <= 4.5 and 3.5 <= r2 <= 4.5, errs


def test_projector_adjoint_identity():
    rng = np.random.default_rng(11)
    g = Geometry(nx=37, ny=29, nz=4, n_angles=7, n_t=512, drive_cycles=3.3333, psf_width=2.0,
                 harm_lo=1, harm_hi=3, half_band=1)
    x = rng.standard_normal((g.nz, g.ny, g.nx))
    y = rng.standard_normal((g.n_angles, g.nz, g.n_u))
    lhs = np.vdot(projector.project(g, x), y)
    rhs = np.vdot(x, projector.backproject(g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def test_projector_brute_force_dense():
    """Column by column on an 8x8 slice against W(p; i, j) = sum_q hat(X_pq - X_i) hat(Y_pq - Y_j),
    the bilinear weight written from the hat-function form of interpolation."""
    g = Geometry(nx=8, ny=8, nz=1, n_angles=5, n_t=256, drive_cycles=3.3333, psf_width=1.5,
                 harm_lo=1, harm_hi=3, half_band=1)
    nr = 12  # smallest integer >= sqrt(128) = 11.31 with the parity of 8
    yq = np.arange(nr) - (nr - 1) / 2
    u = np.arange(8) - 3.5
    Xi = np.arange(8) - 3.5
    for m, t in enumerate(g.theta):
        X = u[:, None] * math.cos(t) + yq[None, :] * math.sin(t)     # (p, q)
        Y = -u[:, None] * math.sin(t) + yq[None, :] * math.cos(t)
        W = np.einsum("pqi,pqj->pji", _hat(X[:, :, None] - Xi[None, None, :]),
                      _hat(Y[:, :, None] - Xi[None, None, :]))      # (p, j, i)
        for col in range(64):
            e = np.zeros((1, 8, 8))
            e.flat[col] = 1.0
            got = projector.project(g, e)[m, 0]
            assert np.max(np.abs(got - W.reshape(8, 64)[:, col])) <= 1e-13
