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


# Relative error level of one mixed-operator application (fp16 tables, scaled
# fp16 operand lines and time tile, bf16 gathers): the mixed operator tests
# measure 7e-5 .. 3e-4 relative L2 on whole vectors.
MIXED_OP_EPS = 2e-4


class Cluster:
    """Iterates of one schedule run on the oracle operator under independent
    random relative errors of one operator error level, one run per seed.

    CGLS is chaotic mid-run: any rounding moves the iterate away from the
    exact-arithmetic run by much more than the rounding (the exact run is an
    outlier), while runs with different rounding land close to one another.
    So an implementation is compared with the runs' mean, and the bar is a
    multiple of the cluster's radius: the largest distance of one run to the
    mean, relative to the mean's norm (``pairwise`` is the largest distance
    between two runs).  ``select`` picks what is compared (a sample of
    voxels, say) from a full iterate."""

    def __init__(self, runs, select=None):
        sel = (lambda v: np.asarray(v).ravel()) if select is None else select
        xs = [np.asarray(sel(x), dtype=np.float64) for x in runs]
        self.mean = np.mean(xs, axis=0)
        nm = np.linalg.norm(self.mean)
        self.radius = max(float(np.linalg.norm(x - self.mean) / nm) for x in xs)
        self.pairwise = max(float(np.linalg.norm(a - b) / nm) for i, a in enumerate(xs) for b in xs[i + 1:])
        self.n = len(xs)

    def distance(self, x):
        return float(np.linalg.norm(np.asarray(x, dtype=np.float64).ravel() - self.mean.ravel())
                     / np.linalg.norm(self.mean))


def segment_distance(x, a, b):
    """Distance of x from the segment [a, b] (flattened arrays), relative to |b|."""
    x, a, b = (np.asarray(v, dtype=np.float64).ravel() for v in (x, a, b))
    d = b - a
    dd = float(d @ d)
    t = 0.0 if dd == 0.0 else min(1.0, max(0.0, float((x - a) @ d) / dd))
    return float(np.linalg.norm(x - (a + t * d)) / np.linalg.norm(b))


class ClusterPath:
    """Clusters of one schedule at the low and the high end of an operator's
    per-call error range.  Where the iterate of a perturbed run lands drifts
    with the error level (the cluster means at 1e-7 and 1e-6 differ by more
    than either cluster's radius), and a real implementation's rounding has a
    part that repeats from call to call (its rounded tables, a consistent
    linear perturbation) and a part that does not, so its effective level lies
    somewhere in the range: an implementation is compared with the segment
    between the two means, and the bar is CLUSTER_BAR times the larger
    radius."""

    def __init__(self, lo, hi):
        self.lo, self.hi = lo, hi
        self.radius = max(lo.radius, hi.radius)
        self.span = float(np.linalg.norm(hi.mean - lo.mean) / np.linalg.norm(hi.mean))
        self.n = lo.n + hi.n

    def distance(self, x):
        return segment_distance(x, self.lo.mean, self.hi.mean)


# Per-call error range of the FP32 operator on CGLS's own vectors, measured on
# the GPU against the FP64 oracle: A p 1.4e-7 .. 6.3e-7, A^T r 2.2e-7 .. 1.2e-6.
FP32_EPS_RANGE = (1e-7, 1e-6)
# Per-call error range of the mixed operator (forward 7e-5 .. 1.2e-4, adjoint
# with fp16 lines up to about 3e-4 relative L2).
MIXED_EPS_RANGE = (5e-5, 3e-4)


def cgls_cluster(run, op, eps=FP32_OP_EPS, seeds=tuple(range(101, 109)), select=None):
    """Cluster of run(perturbed op) over the seeds (see Cluster)."""
    return Cluster([run(PerturbedOperator(op, eps, s)) for s in seeds], select)


def mixed_cluster(run, op, seeds=tuple(range(201, 209)), select=None, eps_outer=FP32_OP_EPS,
                  eps_inner=MIXED_OP_EPS):
    """Cluster of refinement runs run(outer, inner): outer operator at the FP32
    error level (the sweeps' residuals), inner operator at the mixed level."""
    return Cluster([run(PerturbedOperator(op, eps_outer, s), PerturbedOperator(op, eps_inner, s + 5000))
                    for s in seeds], select)


# Bar of a same-schedule solve comparison, in cluster radii.
CLUSTER_BAR = 4.0


def cgls_path(run, op, seeds=tuple(range(101, 107)), select=None, eps_range=FP32_EPS_RANGE):
    """ClusterPath of run(perturbed op) at the two ends of eps_range."""
    lo, hi = (cgls_cluster(run, op, eps, seeds, select) for eps in eps_range)
    return ClusterPath(lo, hi)


def band_errors(got, want, g, axis=-1):
    """Relative L2 error of each kept harmonic band (the 2D + 1 bins around one
    harmonic), over all lines: got/want complex data [..., n_bins]."""
    bw = 2 * g.half_band + 1
    got = np.moveaxis(np.asarray(got), axis, -1)
    want = np.moveaxis(np.asarray(want), axis, -1)
    return np.array([rel_l2(got[..., h * bw:(h + 1) * bw], want[..., h * bw:(h + 1) * bw])
                     for h in range(g.n_bins // bw)])


def band_confined_data(g, seed):
    """Data whose slice k holds random values in harmonic band k mod n_bands
    only: A is block diagonal over z-slices, so one adjoint call yields, slice
    by slice, the adjoint of each band's data alone.  Returns (y, band of each
    slice)."""
    bw = 2 * g.half_band + 1
    nbands = g.n_bins // bw
    rng = np.random.default_rng(seed)
    y = np.zeros((g.n_angles, g.nz, g.n_bins), dtype=np.complex128)
    band = np.arange(g.nz) % nbands
    for k in range(g.nz):
        h = band[k]
        y[:, k, h * bw:(h + 1) * bw] = rng.standard_normal((g.n_angles, bw)) + 1j * rng.standard_normal((g.n_angles, bw))
    return y, band


# Per-band bars.  FP32: 1e-4 per band.  Mixed forward: the time tile and the
# band table are rounded to fp16 (unit roundoff 2^-11) relative to the whole
# line's signal, so a weak band's own relative error grows as its share of the
# signal shrinks: modelled (numpy fp16 rounding of the oracle's tables, lines
# and time tile) at 4.4e-3 for harmonic 31 of the 192x192x96 scan and 1.2e-2
# for harmonic 47 of the 256x256x128 scan; bar 3e-2.  Mixed adjoint: each
# band's data is scaled toward unit size before rounding (per-band scaling),
# so a band confined to its own data keeps the operator bar, 5e-3.  Dropping a
# band, or scaling it wrongly, gives errors of order 1.
BAND_TOL32 = 1e-4
BAND_TOL16_FWD = 3e-2
BAND_TOL16_ADJ = 5e-3


def band_table(name, rows, harm_lo=1):
    """Log lines of a per-harmonic error table: rows = {label: errors}."""
    labels = list(rows)
    n = len(next(iter(rows.values())))
    out = ["%s per-harmonic rel err: harmonic | %s" % (name, " | ".join(labels))]
    for h in range(n):
        out.append("  %3d | %s" % (h + harm_lo, " | ".join("%.2e" % rows[k][h] for k in labels)))
    return "\n".join(out)
