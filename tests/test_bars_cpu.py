"""The bars of the GPU tests, checked on the CPU against mistakes planted in
the oracle: each bar must pass a correct run and fail a wrong one.

* Per-band bars (tests/helpers.py): dropping a harmonic band, or scaling it
  by 1%, gives a per-band error of order 1 (or 1e-2), far above the mixed
  forward's 3e-2 only when the band is dropped or halved -- so the bar sees a
  lost or misscaled band, not rounding.
* Cluster bars of mid-run solves: fresh runs with operator noise anywhere in
  the FP32 range land within 4 radii of the path between the two clusters'
  means; runs of a CGLS with a planted mistake in its recurrences (the lambda
  term left out of delta, a wrong beta) land outside, with the same noise.
"""
import numpy as np

from oracle import operator as oop, solvers
from paper_2511_06627_amd import configs
from helpers import (config_geometry, band_errors, band_confined_data, BAND_TOL16_FWD, BAND_TOL16_ADJ,
                     BAND_TOL32, cgls_path, CLUSTER_BAR, PerturbedOperator, rel_l2, random_volume)


def _small():
    from oracle.geometry import Geometry
    g = Geometry(nx=16, ny=16, nz=6, n_angles=5, n_t=1024, drive_cycles=1024 / 256 + 1 / 3, psf_width=2.0,
                 harm_lo=1, harm_hi=6, half_band=1)
    return oop.normalised(g, iters_min=30, rtol=1e-9)


def test_band_bars_see_a_dropped_or_halved_band():
    g = _small()
    bw = 2 * g.half_band + 1
    want = oop.forward(g, random_volume(g, 1))
    assert np.all(band_errors(want, want, g) == 0.0)
    for h in (0, g.n_bins // bw - 1):
        for factor, least in ((0.0, 1.0), (0.5, 0.5)):
            got = want.copy()
            got[..., h * bw:(h + 1) * bw] *= factor
            e = band_errors(got, want, g)
            assert abs(e[h] - least) <= 1e-12 and e[h] > BAND_TOL16_FWD > BAND_TOL16_ADJ > BAND_TOL32
            assert np.all(np.delete(e, h) == 0.0)
    # band-confined data: each slice's adjoint depends on its own band only
    y, band = band_confined_data(g, 2)
    x = oop.adjoint(g, y)
    for k in range(g.nz):
        yk = np.zeros_like(y)
        yk[:, k] = y[:, k]
        assert rel_l2(oop.adjoint(g, yk)[k], x[k]) <= 1e-13
        h = band[k]
        assert np.all(y[:, k, :h * bw] == 0) and np.all(y[:, k, (h + 1) * bw:] == 0)


def _cgls_planted(op, b, lam, iters, mistake):
    """CGLS with one planted mistake in its recurrences."""
    sq = lambda v: float(np.sum(np.abs(v) ** 2))  # noqa: E731
    x = np.zeros((op.g.nz, op.g.ny, op.g.nx))
    r = b.copy()
    s = op.adjoint(r)
    p = s.copy()
    gamma = sq(s)
    for _ in range(iters):
        q = op.forward(p)
        delta = sq(q) + (0.0 if mistake == "no_lambda" else lam) * sq(p)
        alpha = gamma / delta
        x = x + alpha * p
        r = r - alpha * q
        s = op.adjoint(r) - lam * x
        gn = sq(s)
        beta = gn / gamma * (0.9 if mistake == "beta" else 1.0)
        p = s + beta * p
        gamma = gn
    return x


def test_cluster_bar_passes_noise_and_fails_planted_solver_mistakes():
    cfg = configs.PARITY_32
    g = config_geometry(cfg)
    b, _ = oop.make_data(g, configs.make_phantom(cfg), cfg.noise, cfg.noise_seed)
    b = b.astype(np.complex64).astype(np.complex128)
    op = oop.Operator(g, precomposed=True)
    run = lambda o: solvers.cgls(o, b, cfg.lam, cfg.iters)  # noqa: E731
    cl = cgls_path(run, op)
    bar = CLUSTER_BAR * cl.radius
    for eps, s in ((1e-7, 301), (3e-7, 302), (1e-6, 303)):
        assert cl.distance(run(PerturbedOperator(op, eps, s))) <= bar, eps
    for mistake in ("beta", "no_lambda"):
        d = cl.distance(_cgls_planted(PerturbedOperator(op, 1e-6, 304), b, cfg.lam, cfg.iters, mistake))
        assert d > bar, (mistake, d, bar)
