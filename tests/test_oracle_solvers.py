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


def test_op_norm_equals_dense_spectral_norm(problem):
    """The power-iteration norm against the dense matrix's largest singular
    value: the normalised operator has ||A||_2 = 1 (Sec. 3.3).  A maps real
    volumes to complex data and its norm is taken in the real inner product
    Re(u^H v), so the matrix is [Re A; Im A] (the complex matrix's own 2-norm,
    a maximum over complex x, is larger)."""
    g, op, A, b, lam, xs = problem
    assert abs(np.linalg.norm(np.concatenate([A.real, A.imag]), 2) - 1.0) <= 1e-9
    # and the raw operator's norm is the reciprocal of the scale that normalised it
    assert abs(operator.op_norm(g.with_scale(1.0)) * g.op_scale - 1.0) <= 1e-9


def test_refinement_with_exact_inner_operator_is_restarted_cgls(problem):
    """Refinement in correction form reduces to CGLS restarted every sweep when
    the inner operator is the outer one (with and without the clamp).  The two
    forms round differently: from the second sweep on, the restart gradient
    A^T r0 - lam x is small next to its terms, so rounding differences of
    relative size 1e-16 in it are amplified by CGLS (measured: 9e-12 after one
    sweep of 4, 2e-4 after two).  So one sweep is compared at 1e-10, and
    several sweeps at convergence against the dense minimiser."""
    g, op, A, b, lam, xs = problem
    for clamp in (False, True):
        a = solvers.cgls_restarted(op, b, lam, 4, every=4, clamp=clamp)
        r = solvers.refine(op, op, b, lam, 1, 4, clamp=clamp)
        assert np.linalg.norm(r - a) <= 1e-10 * np.linalg.norm(a), clamp
    x = solvers.refine(op, op, b, lam, 4, 40)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_refinement_reaches_minimiser_with_rounded_inner_operator(problem):
    """An inner operator carrying 1e-3 relative errors still converges to the
    exact minimiser: the outer residual is exact, so only the rate suffers."""
    g, op, A, b, lam, xs = problem

    class Rounded:
        def __init__(self, o):
            self.g, self.o, self.rng = o.g, o, np.random.default_rng(5)

        def forward(self, x):
            y = self.o.forward(x)
            return y * (1 + 1e-3 * self.rng.standard_normal(y.shape))

        def adjoint(self, y):
            x = self.o.adjoint(y)
            return x * (1 + 1e-3 * self.rng.standard_normal(x.shape))

    x = solvers.refine(op, Rounded(op), b, lam, 12, 15)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


class _Dense2:
    """A 2 x 2 real operator in the oracle's operator interface (one 1 x 2 slice)."""

    class g:
        nz, ny, nx = 1, 1, 2

    A = np.array([[1.0, 0.5], [-0.25, 1.0]])

    def forward(self, x):
        return (self.A @ x.reshape(2)).astype(np.complex128).reshape(1, 1, 2)

    def adjoint(self, y):
        return np.real(self.A.T @ np.asarray(y).reshape(2)).reshape(1, 1, 2)


def test_momentum_first_three_iterates_by_hand():
    """eq. iters step by step on a 2 x 2 problem: x^0 = x^1 = 0, momentum
    weights (k-1)/(k+2) = 0, 1/4, 2/5 for k = 1, 2, 3, gradient of
    |Ay - b|^2 / 2 + lam |y|^2 / 2, then the projection onto x >= 0."""
    op = _Dense2()
    A = op.A
    b = np.array([1.0, -0.5])
    lam, tau = 0.1, 0.5

    def step(y):
        return np.maximum(y - tau * (A.T @ (A @ y - b) + lam * y), 0.0)

    x1 = np.zeros(2)
    x2 = step(x1 + 0.0 * (x1 - x1))
    x3 = step(x2 + 0.25 * (x2 - x1))
    x4 = step(x3 + 0.4 * (x3 - x2))
    bc = b.astype(np.complex128).reshape(1, 1, 2)
    for k, want in ((1, x2), (2, x3), (3, x4)):
        got = solvers.momentum_gradient(op, bc, lam, k, tau, nonneg=True).reshape(2)
        assert np.max(np.abs(got - want)) <= 1e-15, (k, got, want)
    # the clamp acts here (the second unknown would go negative), so the
    # nonnegative and unconstrained runs must differ
    free = solvers.momentum_gradient(op, bc, lam, 3, tau, nonneg=False).reshape(2)
    assert free.min() < 0.0 and x4.min() >= 0.0
