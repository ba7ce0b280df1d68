"""Pins for oracle.regularizer: the finite-difference T of eq. nummodel."""
import numpy as np

from oracle import regularizer as reg


def _dense_normal(shape):
    nz, ny, nx = shape
    n = nz * ny * nx
    cols = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        cols.append(reg.fd_normal(e.reshape(shape)).ravel())
    return np.stack(cols, axis=1)


def _lap1d(n):
    """1D second-difference matrix with reflecting ends, written from its stencil."""
    m = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            m[i, i] += 1.0
            m[i, i - 1] -= 1.0
        if i < n - 1:
            m[i, i] += 1.0
            m[i, i + 1] -= 1.0
    return m


def test_adjoint_identity():
    """<T x, d> = <x, T^T d> for arbitrary difference fields (the slab T x
    leaves at zero is ignored by T^T too)."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7))
    ds = [rng.standard_normal((5, 6, 7)) for _ in range(3)]
    lhs = sum(float(np.vdot(a, b)) for a, b in zip(reg.fd_forward(x), ds))
    rhs = float(np.vdot(x, reg.fd_adjoint(ds)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_normal_is_kronecker_sum_of_1d_laplacians():
    shape = (3, 4, 5)
    nz, ny, nx = shape
    got = _dense_normal(shape)
    Lx, Ly, Lz = _lap1d(nx), _lap1d(ny), _lap1d(nz)
    want = (np.kron(np.kron(np.eye(nz), np.eye(ny)), Lx) + np.kron(np.kron(np.eye(nz), Ly), np.eye(nx))
            + np.kron(np.kron(Lz, np.eye(ny)), np.eye(nx)))
    assert np.array_equal(got, want)


def test_norm_closed_form_matches_eigenvalues():
    for shape in ((3, 4, 5), (2, 6, 6), (4, 4, 4)):
        ev = np.linalg.eigvalsh(_dense_normal(shape))
        assert abs(ev.max() - reg.fd_normal_norm(shape)) <= 1e-12 * ev.max()
        assert abs(ev.min()) <= 1e-12


def test_constants_in_null_space():
    x = np.full((4, 5, 6), 3.25)
    assert np.abs(reg.fd_normal(x)).max() == 0.0
