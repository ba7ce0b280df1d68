"""Scan workloads: geometry, phantom recipe, noise and solve schedule.

Plain data.  Every modelling choice the paper leaves open is an explicit
field here (drive periods per line, PSF width, kept bands, ...).

Drive periods per line P = T/256 + 1/3: non-integer, so the harmonics fall
between DFT bins and the side bins around each harmonic carry signal.
Drive amplitude a = Nu/2: the sweep spans the fast axis edge to edge.
"""
from dataclasses import dataclass, field


@dataclass(frozen=True)
class ScanConfig:
    name: str
    nx: int
    ny: int
    nz: int
    n_angles: int
    n_t: int
    psf_width: float
    harm_lo: int
    harm_hi: int
    half_band: int
    noise: float
    lam: float
    iters: int
    phantom: str                 # "blobs" | "blobs_organ" | "organ_satellites"
    phantom_seed: int
    noise_seed: int
    clamp_every: int = 0         # nonnegativity clamp + restart period (0 = none)
    refine_sweeps: int = 0       # mixed precision: outer sweeps x inner iterations
    inner_iters: int = 0

    @property
    def drive_cycles(self):
        return self.n_t / 256.0 + 1.0 / 3.0

    @property
    def n_u(self):
        return self.nx

    @property
    def drive_amp(self):
        return self.nx / 2.0

    @property
    def n_bins(self):
        return (self.harm_hi - self.harm_lo + 1) * (2 * self.half_band + 1)

    @property
    def n_lines(self):
        return self.n_angles * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


PARITY_32 = ScanConfig("parity_32cube", 32, 32, 32, 8, 2048, 2.0, 1, 15, 2, 0.01, 1e-3, 20,
                       "blobs", 0, 1)
REALISTIC_192 = ScanConfig("realistic_192x192x96", 192, 192, 96, 36, 8192, 3.0, 1, 31, 3, 0.005,
                           1e-3, 50, "blobs_organ", 10, 11)
MIXED_192 = ScanConfig("mixed_192x192x96", 192, 192, 96, 36, 8192, 3.0, 1, 31, 3, 0.005,
                       1e-3, 60, "blobs_organ", 10, 11, refine_sweeps=3, inner_iters=20)
HDR_256 = ScanConfig("hdr_256x256x128", 256, 256, 128, 60, 16384, 3.0, 1, 47, 3, 0.001,
                     1e-3, 100, "organ_satellites", 40, 41, clamp_every=10)

# Serving stream: request classes drawn uniformly from these sets.
SERVE_VOLUMES = ((64, 64, 64), (128, 128, 64), (192, 192, 96))   # (nx, ny, nz)
SERVE_ANGLES = (12, 24, 36)
SERVE_T = (4096, 6144, 8192)
SERVE_RATE_HZ = 2.0
SERVE_REQUESTS = 64
SERVE_ARRIVAL_SEED = 3000
SERVE_ITERS = 40              # 2 refinement sweeps x 20 inner iterations
SERVE_BUDGET_BYTES = 200 * 10 ** 9


def serve_config(nx, ny, nz, n_angles, n_t, idx):
    return ScanConfig("serve_%dx%dx%d_m%d_t%d" % (nx, ny, nz, n_angles, n_t), nx, ny, nz, n_angles,
                      n_t, 3.0, 1, 31, 3, 0.005, 1e-3, SERVE_ITERS, "blobs_organ", 1000 + idx,
                      2000 + idx, refine_sweeps=2, inner_iters=20)


ALL = {c.name: c for c in (PARITY_32, REALISTIC_192, MIXED_192, HDR_256)}


def make_phantom(cfg):
    """The seeded phantom volume (Nz, Ny, Nx) float64 for a config."""
    from . import phantoms
    if cfg.phantom == "blobs":
        return phantoms.gaussian_blobs(cfg.shape, 6, (1.5, 4.0), (-2.0, 0.0), cfg.phantom_seed)
    if cfg.phantom == "blobs_organ":
        return phantoms.blobs_and_organ(cfg.shape, 40, (1.0, 10.0), (-3.0, 0.0), cfg.phantom_seed)
    if cfg.phantom == "organ_satellites":
        vol, _ = phantoms.organ_with_satellites(cfg.shape, 30, (1.0, 2.0), (-4.0, -2.0), (2.0, 5.0),
                                                cfg.phantom_seed)
        return vol
    raise ValueError(cfg.phantom)
