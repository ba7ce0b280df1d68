"""The band DFT factored over drive cycles, checked on the CPU against the dense
definition (numpy only; no GPU code involved).

Appendix A's transform on the kept bins (eq. bcompress, eq. DCmodel),
b_j = sum_t s[t] D_j e^{+2 pi i (omega_j t mod T) / T} / sqrt(T), has integer bins,
so with t = n1 + P n2 (T = C P) the phase splits exactly:
omega_j t = omega_j n1 + (omega_j mod C) T n2 / C (mod T).  The FP32 kernels
evaluate b as a C-point sum at the residues r = omega_j mod C followed by a
P-point sum per bin, and the adjoint as the transpose of both steps.  These
tests pin that regrouping -- its twiddle signs, the residue bookkeeping and the
transpose -- on the scan configurations' own bin sets, with a receive filter,
for the C values the plan may take.
"""
import math

import numpy as np
import pytest

from paper_2511_06627_amd import configs


def _bins(T, cycles, klo, khi, half):
    out = []
    for k in range(klo, khi + 1):
        c = math.floor(k * cycles + 0.5)
        out += [c + d for d in range(-half, half + 1)]
    return np.asarray(out, dtype=np.int64)


def _dense(T, bins, D):
    t = np.arange(T)
    a = D[None, :] * np.exp(2j * np.pi * ((bins[None, :] * t[:, None]) % T) / T) / np.sqrt(T)
    F = np.zeros((T, 2 * len(bins)))
    F[:, 0::2], F[:, 1::2] = a.real, a.imag
    return F


def _factored(T, C, bins, D, s=None, y=None):
    """Forward b from the signal s, or adjoint g from the data y, in the
    factored order (residue DFT over n2, then phase sum over n1)."""
    P = T // C
    res = sorted(set(int(b) % C for b in bins))
    q_of = {r: i for i, r in enumerate(res)}
    n1, n2 = np.arange(P), np.arange(C)
    E = np.zeros((C, 2 * len(res)))
    for q, r in enumerate(res):
        ph = 2 * np.pi * ((r * n2) % C) / C
        E[:, 2 * q], E[:, 2 * q + 1] = np.cos(ph), np.sin(ph)
    G = np.stack([D[j] * np.exp(2j * np.pi * ((int(bins[j]) * n1) % T) / T) / np.sqrt(T)
                  for j in range(len(bins))])
    if s is not None:
        Y = s.reshape(C, P).T @ E                     # [n1][2R]: t = n1 + P n2
        out = np.zeros(2 * len(bins))
        for j in range(len(bins)):
            q = q_of[int(bins[j]) % C]
            yr, yi = Y[:, 2 * q], Y[:, 2 * q + 1]
            out[2 * j] = np.sum(yr * G[j].real - yi * G[j].imag)
            out[2 * j + 1] = np.sum(yr * G[j].imag + yi * G[j].real)
        return out
    Z = np.zeros((P, 2 * len(res)))
    for j in range(len(bins)):
        q = q_of[int(bins[j]) % C]
        y0, y1 = y[2 * j], y[2 * j + 1]
        Z[:, 2 * q] += G[j].real * y0 + G[j].imag * y1
        Z[:, 2 * q + 1] += -G[j].imag * y0 + G[j].real * y1
    return (Z @ E.T).T.reshape(T)                     # [n2][n1] -> t = n1 + P n2


@pytest.mark.parametrize("cfg,C", [(configs.HDR_256, 64), (configs.REALISTIC_192, 32), (configs.PARITY_32, 32)])
def test_factored_band_dft_is_the_dense_one(cfg, C):
    T = cfg.n_t
    bins = _bins(T, cfg.drive_cycles, cfg.harm_lo, cfg.harm_hi, cfg.half_band)
    rng = np.random.default_rng(7)
    D = rng.standard_normal(len(bins)) + 1j * rng.standard_normal(len(bins))   # a receive filter
    F = _dense(T, bins, D)
    s = rng.standard_normal(T)
    y = rng.standard_normal(2 * len(bins))
    fwd = _factored(T, C, bins, D, s=s)
    adj = _factored(T, C, bins, D, y=y)
    assert np.linalg.norm(fwd - s @ F) <= 1e-12 * np.linalg.norm(s @ F)
    assert np.linalg.norm(adj - F @ y) <= 1e-12 * np.linalg.norm(F @ y)
    # the adjoint is the transpose: <F^T s, y> = <s, F y> through the factored forms
    assert abs(fwd @ y - s @ adj) <= 1e-12 * np.linalg.norm(fwd) * np.linalg.norm(y)
