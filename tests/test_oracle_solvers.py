"""Pins for oracle.solvers against dense linear algebra on 8^3 problems."""
import numpy as np
import pytest

from oracle import operator, solvers
from oracle.geometry import Geometry


@pytest.fixture(scope="module")
def problem():
    g = Geometry(nx=8, ny=8, nz=8, n_angles=4, n_t=256, drive_cycles=5.3333, psf_width=1.5,
                 harm_lo=1, harm_hi=6, half_band=1)
    g = operator.normalised(g)
    op = operator.Operator(g)
    n = g.n_vox
    cols = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        cols.append(op.forward(e.reshape(g.nz, g.ny, g.nx)).ravel())
    A = np.stack(cols, axis=1)
    rng = np.random.default_rng(2)
    xt = rng.uniform(0, 1, (g.nz, g.ny, g.nx))
    b = op.forward(xt) + 0.01 * (rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])).reshape(
        g.n_angles, g.nz, g.n_bins)
    lam = 1e-3
    N = np.real(np.conj(A).T @ A) + lam * np.eye(n)
    xs = np.linalg.solve(N, np.real(np.conj(A).T @ b.ravel()))
    return g, op, A, b, lam, xs.reshape(g.nz, g.ny, g.nx)


def test_cgls_converges_to_dense_normal_equations(problem):
    g, op, A, b, lam, xs = problem
    # well past convergence (about 60 iterations here) but short of the long
    # post-convergence drift that plain CGLS shows in floating point
    x = solvers.cgls(op, b, lam, 120)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_reference_minimiser(problem):
    g, op, A, b, lam, xs = problem
    x, it = solvers.reference_minimiser(op, b, lam, tol=1e-13)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert it < 5000


def test_cgls_objective_monotone(problem):
    g, op, A, b, lam, xs = problem
    vals = [solvers.objective(op, b, solvers.cgls(op, b, lam, k), lam) for k in range(0, 25)]
    assert all(b2 <= a2 * (1 + 1e-14) for a2, b2 in zip(vals, vals[1:]))


def test_cgls_first_step_is_exact_line_search(problem):
    """After one iteration from 0, x = alpha s0 with alpha minimising the objective along s0."""
    g, op, A, b, lam, xs = problem
    s0 = np.real(np.conj(A).T @ b.ravel())
    As0 = A @ s0
    alpha = (s0 @ s0) / (np.vdot(As0, As0).real + lam * s0 @ s0)
    x1 = solvers.cgls(op, b, lam, 1).ravel()
    assert np.max(np.abs(x1 - alpha * s0)) <= 1e-13 * np.max(np.abs(x1))


def test_restart_schedules(problem):
    g, op, A, b, lam, xs = problem
    plain = solvers.cgls(op, b, lam, 20)
    once = solvers.cgls_restarted(op, b, lam, 20, every=20)
    assert np.array_equal(plain, once)
    manual = solvers.cgls(op, b, lam, 10, x0=solvers.cgls(op, b, lam, 10))
    two = solvers.cgls_restarted(op, b, lam, 20, every=10)
    assert np.max(np.abs(manual - two)) == 0.0
    clamped = solvers.cgls_restarted(op, b, lam, 30, every=10, clamp=True)
    assert clamped.min() >= 0.0


def test_clamp_inactive_reduces_to_restarted(problem):
    """With data of a strongly positive image and a large offset, the clamp never acts."""
    g, op, A, b, lam, xs = problem
    xt = 5.0 + np.random.default_rng(9).uniform(0, 1, (g.nz, g.ny, g.nx))
    bb = op.forward(xt)
    a = solvers.cgls_restarted(op, bb, lam, 30, every=10, clamp=False)
    if a.min() <= 0:
        pytest.skip("iterate not positive; clamp would be active")
    c = solvers.cgls_restarted(op, bb, lam, 30, every=10, clamp=True)
    assert np.array_equal(a, c)


def test_momentum_gradient_converges_to_minimiser(problem):
    g, op, A, b, lam, xs = problem
    tau = 1.0 / (1.0 + lam)        # ||A^* A|| = 1 after normalisation, ||T^* T|| = 1 for T = I
    e = [np.linalg.norm(solvers.momentum_gradient(op, b, lam, k, tau, nonneg=False) - xs)
         / np.linalg.norm(xs) for k in (300, 3000)]
    # accelerated gradient: sublinear, but steadily toward the same minimiser
    assert e[1] <= 5e-5 and e[1] < 0.2 * e[0], e


def test_momentum_gradient_projection_keeps_nonnegative(problem):
    g, op, A, b, lam, xs = problem
    x = solvers.momentum_gradient(op, b, lam, 50, 1.0 / (1.0 + lam), nonneg=True)
    assert x.min() >= 0.0


def test_momentum_gradient_with_finite_differences(problem):
    """With T the finite differences of oracle.regularizer the paper's iteration
    heads to the minimiser of ||Ax-b||^2 + lam ||Tx||^2, written out densely."""
    from oracle import regularizer
    g, op, A, b, lam, _ = problem
    n = g.n_vox
    cols = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        cols.append(regularizer.fd_normal(e.reshape(g.nz, g.ny, g.nx)).ravel())
    TT = np.stack(cols, axis=1)
    lam_fd = 1e-2
    N = np.real(np.conj(A).T @ A) + lam_fd * TT
    xs = np.linalg.solve(N, np.real(np.conj(A).T @ b.ravel())).reshape(g.nz, g.ny, g.nx)
    tau = solvers.paper_tau(1.0, lam_fd, "fd", (g.nz, g.ny, g.nx))
    assert tau == 1.0 / (1.0 + lam_fd * regularizer.fd_normal_norm((g.nz, g.ny, g.nx)))
    e = [np.linalg.norm(solvers.momentum_gradient(op, b, lam_fd, k, tau, nonneg=False, reg="fd") - xs)
         / np.linalg.norm(xs) for k in (200, 2000)]
    assert e[1] <= 1e-3 and e[1] < 0.2 * e[0], e
