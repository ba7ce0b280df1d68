"""Shared test helpers: oracle geometries for the scan configs, seeded inputs."""
import numpy as np

from oracle import geometry, operator


def oracle_geometry(nx, ny, nz, n_angles, n_t, drive_cycles, psf_width, harm_lo, harm_hi, half_band,
                    op_scale=1.0, rx_filter=None):
    return geometry.Geometry(nx=nx, ny=ny, nz=nz, n_angles=n_angles, n_t=n_t, drive_cycles=drive_cycles,
                             psf_width=psf_width, harm_lo=harm_lo, harm_hi=harm_hi, half_band=half_band,
                             op_scale=op_scale, rx_filter=rx_filter)


def config_geometry(cfg, normalise=True):
    g = oracle_geometry(cfg.nx, cfg.ny, cfg.nz, cfg.n_angles, cfg.n_t, cfg.drive_cycles, cfg.psf_width,
                        cfg.harm_lo, cfg.harm_hi, cfg.half_band)
    if normalise:
        g = operator.normalised(g, iters_min=30, rtol=1e-9)
    return g


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        a = np.stack([np.real(a), np.imag(a)], -1)
        b = np.stack([np.real(b), np.imag(b)], -1)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def random_volume(g, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (g.nz, g.ny, g.nx))


def random_data(g, seed):
    rng = np.random.default_rng(seed)
    shape = (g.n_angles, g.nz, g.n_bins)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


class PerturbedOperator:
    """The oracle operator with every output multiplied by (1 + eps * N(0,1)),
    independently per element and per call: a model of an implementation that
    rounds each operator result at relative precision eps."""

    def __init__(self, op, eps, seed):
        self.op = op
        self.g = op.g
        self.eps = eps
        self.rng = np.random.default_rng(seed)

    def forward(self, x):
        y = self.op.forward(x)
        return y * (1.0 + self.eps * self.rng.standard_normal(y.shape))

    def adjoint(self, y):
        x = self.op.adjoint(y)
        return x * (1.0 + self.eps * self.rng.standard_normal(x.shape))


# Relative error level of an FP32 operator application: the FP32 operator
# parity tests hold A and A^T to it (measured 1e-7 to 3e-6 relative L2; long
# fp32 sums over T samples and bilinear weights from fp32 coordinates).
FP32_OP_EPS = 1e-6


def fp32_envelope(run, op, seeds=(11, 12, 13), eps=FP32_OP_EPS):
    """Largest relative deviation between run(op) and run(perturbed op) over a
    few seeds: how far an implementation whose operator is accurate to about
    eps can drift from the FP64 iterate on this schedule."""
    ref = run(op)
    dev = max(rel_l2(run(PerturbedOperator(op, eps, s)), ref) for s in seeds)
    return ref, dev
