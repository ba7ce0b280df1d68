"""Oracle solvers for the Tikhonov problem of eq. nummodel, FP64.

Test infrastructure only (see ``oracle/__init__``).

Objective (Sec. 3.3, eq. nummodel):  min_x ||A x - b||^2 + lam ||T x||^2,
here with T = I.  Norms of complex data are sums of squared moduli.

* ``cgls``          -- conjugate gradients on the normal equations
                       (A^T A + lam I) x = A^T b in the least-squares form:
                         r = b - A x, s = A^T r - lam x, p = s, gamma = |s|^2
                         loop: q = A p, delta = |q|^2 + lam |p|^2,
                               alpha = gamma / delta, x += alpha p,
                               r -= alpha q, s = A^T r - lam x,
                               gamma' = |s|^2, beta = gamma'/gamma,
                               p = s + beta p.
* ``cgls_restarted`` -- the same, restarted every ``every`` iterations from
                       the current x with freshly formed r, s, p; optionally
                       clamping x >= 0 before each restart (the nonnegativity
                       the paper imposes, Sec. 3.3 after eq. iters).  With an
                       exact operator, iterative refinement sweeps reduce to
                       exactly this schedule.
* ``momentum_gradient`` -- the paper's own method, eq. iters: fixed step
                       tau = 1/(||A*A|| + lam ||T*T||) with the momentum
                       weight (k-1)/(k+2), projecting onto real nonnegative
                       values every iteration; T = I or the finite
                       differences of ``oracle.regularizer``.
* ``refine``        -- iterative refinement in correction form: each sweep
                       forms r0 = b - A x and g0 = A^T r0 - lam x with the
                       outer operator, then runs CGLS with the inner operator
                       on the correction d of min |A' d - r0|^2 + lam |x + d|^2
                       (from d = 0), sets x += d and optionally clamps x >= 0.
                       With the inner operator equal to the outer one this is
                       CGLS restarted every sweep (the same iterates in exact
                       arithmetic); it is the schedule of a mixed-precision
                       solve whose inner operator is a rounded copy of A.
* ``reference_minimiser`` -- x* = argmin, from CGLS run until
                       |s_k| <= tol |s_0|.

Pins (tests/test_oracle_solvers.py): on 8^3 problems CGLS matches
numpy.linalg.solve of the dense normal equations; the objective is monotone;
restarted CGLS with an inactive clamp equals restarted CGLS; refinement with
the exact operator inside reproduces restarted CGLS; the momentum method
converges to the same minimiser when the clamp is inactive, and its first
three iterates on a 2 x 2 problem match the recurrence written out by hand.
"""
import numpy as np


def _sq(v):
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return float(np.sum(v.real * v.real + v.imag * v.imag))
    return float(np.sum(v * v))


def objective(op, b, x, lam):
    return _sq(op.forward(x) - b) + lam * _sq(x)


def cgls(op, b, lam, iters, x0=None, history=None):
    """Plain CGLS; ``history`` (list) receives (gamma, delta, alpha, beta) per iteration."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx)) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - op.forward(x)
    s = op.adjoint(r) - lam * x
    p = s.copy()
    gamma = _sq(s)
    for _ in range(iters):
        q = op.forward(p)
        delta = _sq(q) + lam * _sq(p)
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = op.adjoint(r) - lam * x
        gamma_new = _sq(s)
        beta = gamma_new / gamma
        p = s + beta * p
        if history is not None:
            history.append((gamma, delta, alpha, beta))
        gamma = gamma_new
    return x


def cgls_restarted(op, b, lam, iters, every, clamp=False, x0=None):
    """CGLS restarted every ``every`` iterations (and clamped x >= 0 first if asked).

    The clamp, when asked, is applied after iterations every, 2*every, ...,
    including the last one.
    """
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx)) if x0 is None else np.array(x0, dtype=np.float64)
    done = 0
    while done < iters:
        n = min(every, iters - done)
        x = cgls(op, b, lam, n, x0=x)
        done += n
        if clamp:
            x = np.maximum(x, 0.0)
    return x


def refine(op, op_inner, b, lam, sweeps, inner_iters, clamp=False, x0=None):
    """Refinement sweeps in correction form (see the module docstring).

    Within a sweep x is fixed; CGLS runs on d with r = r0 - A' d and the
    gradient s = g0 - A'^T A' d - lam d, i.e. s = g0 + A'^T r_d - lam d where
    r_d = -A' d is carried as the data-space residual of the correction.
    """
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx)) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(sweeps):
        r0 = b - op.forward(x)
        g0 = op.adjoint(r0) - lam * x
        d = np.zeros_like(x)
        rd = np.zeros_like(r0)          # -A' d
        s = g0.copy()
        p = s.copy()
        gamma = _sq(s)
        for _ in range(inner_iters):
            q = op_inner.forward(p)
            alpha = gamma / (_sq(q) + lam * _sq(p))
            d = d + alpha * p
            rd = rd - alpha * q
            s = g0 + op_inner.adjoint(rd) - lam * d
            gamma_new = _sq(s)
            p = s + (gamma_new / gamma) * p
            gamma = gamma_new
        x = x + d
        if clamp:
            x = np.maximum(x, 0.0)
    return x


def reference_minimiser(op, b, lam, tol=1e-13, max_iters=5000):
    """x* by CGLS until |A^T r - lam x| <= tol |A^T b| (x0 = 0)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx))
    r = b.copy()
    s = op.adjoint(r)
    p = s.copy()
    gamma = gamma0 = _sq(s)
    it = 0
    while it < max_iters and gamma > (tol ** 2) * gamma0:
        q = op.forward(p)
        alpha = gamma / (_sq(q) + lam * _sq(p))
        x = x + alpha * p
        r = r - alpha * q
        s = op.adjoint(r) - lam * x
        gamma_new = _sq(s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        it += 1
    return x, it


def momentum_gradient(op, b, lam, iters, tau, x0=None, nonneg=True, reg="identity"):
    """The paper's iteration (eq. iters).

    y^{k+1} = x^k + (k-1)/(k+2) (x^k - x^{k-1})
    x^{k+1} = P( y^{k+1} - tau [A^*(A y^{k+1} - b) + lam T^*T y^{k+1}] )
    where P keeps the real part (A^T = Re A^H already) and, if ``nonneg``,
    clamps to >= 0.  Iterations are numbered k = 1, 2, ...; x^0 = x^1 = x0.
    ``reg``: "identity" (T = I) or "fd" (the finite differences of
    oracle.regularizer).
    """
    from .regularizer import fd_normal
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx)) if x0 is None else np.array(x0, dtype=np.float64)
    x_prev = x.copy()
    for k in range(1, iters + 1):
        y = x + (k - 1.0) / (k + 2.0) * (x - x_prev)
        ty = y if reg == "identity" else fd_normal(y)
        grad = op.adjoint(op.forward(y) - b) + lam * ty
        x_new = y - tau * grad
        if nonneg:
            x_new = np.maximum(x_new, 0.0)
        x_prev, x = x, x_new
    return x


def paper_tau(ata_norm, lam, reg, shape):
    """tau = 1 / (||A^*A||_2 + lam ||T^*T||_2) (after eq. iters)."""
    from .regularizer import fd_normal_norm
    tt = 1.0 if reg == "identity" else fd_normal_norm(shape)
    return 1.0 / (ata_norm + lam * tt)
