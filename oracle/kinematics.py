"""Stellar velocity dispersion sigma_gal as a free parameter: the Fourier stage of the
continuum projection (Sec. 2.5 "kinematics", App. F "projected in two stages").  Test
infrastructure only (used by tests/, the smoke check and the bench's CPU baseline).

The continuum on the model grid, which must be uniform in ln(lambda) (the stage's uniform
grid is then the model grid itself), is cut to a window of nodes that covers everything
the projection reads, copied into a transform buffer padded with the window's edge
values, multiplied in Fourier space by exp(-2 pi^2 sigma_gal^2 nu^2) with nu conjugate
to c ln(lambda), and transformed back.  sigma_gal = 0 leaves the continuum as it is.

Readings (the paper fixes the operation, not these sizes):
  - window of a spectrum: the nodes within M of the pixels' rest-frame range at the
    point's redshift, M = ceil(5 max_i sigma_i / (c dlnl)) + ceil(5 sigma_max / (c dlnl)) + 2
    with sigma_i the banded kernel's width at pixel i and sigma_max the largest dispersion
    the library admits (what five-dispersion rows reach, what reaches them through the
    Fourier stage, and the interpolation brackets); of photometry: the filter nodes'
    rest-frame range with M = ceil(5 sigma_max / (c dlnl)) + 2;
  - transform length: the smallest power of two that holds the longest window of the
    observation plus ceil(5 sigma_max / (c dlnl)) edge values on each side, sigma_max
    the largest dispersion the library admits, so that the wrap-around of the cyclic
    transform lies five dispersions away from the window;
  - the padding after the window holds its last value for half the free length (the
    larger half), then its first value up to the end of the buffer;
  - values of sigma_gal outside [0, sigma_max] make the point's model NaN.
"""
from __future__ import annotations

import math

import numpy as np

from .constants import C_KMS


def log_step(wave):
    """dlnl of a grid uniform in ln(lambda); ValueError otherwise."""
    ln = np.log(np.asarray(wave, dtype=np.float64))
    d = np.diff(ln)
    step = (ln[-1] - ln[0]) / (len(ln) - 1)
    if np.max(np.abs(d - step)) > 1e-6 * step:
        raise ValueError("the Fourier stage needs a model grid uniform in ln(lambda)")
    return step


def margin_nodes(sigma_kms, dlnl, n_sigma=5.0):
    """Nodes within n_sigma dispersions: ceil(n_sigma sigma / (c dlnl))."""
    return int(math.ceil(n_sigma * float(sigma_kms) / (C_KMS * dlnl)))


def window(wave, lam_lo_obs, lam_hi_obs, z, M):
    """[j0, j1): the model nodes from floor(u(lam_lo)) - M to floor(u(lam_hi)) + 1 + M,
    clipped to the grid, with u(lam) = (ln(lam / (1 + z)) - ln(wave[0])) / dlnl."""
    dlnl = log_step(wave)
    ln0 = math.log(wave[0])
    u0 = (math.log(lam_lo_obs) - math.log1p(z) - ln0) / dlnl
    u1 = (math.log(lam_hi_obs) - math.log1p(z) - ln0) / dlnl
    j0 = max(int(math.floor(u0)) - M, 0)
    j1 = min(int(math.floor(u1)) + 2 + M, len(wave))
    return j0, max(j1, j0)


def fft_length(lam_lo_obs, lam_hi_obs, dlnl, M, sigma_max_kms):
    """Smallest power of two >= ceil(ln(lam_hi / lam_lo) / dlnl) + 2 M + 2 + 2 m_gal."""
    need = int(math.ceil(math.log(lam_hi_obs / lam_lo_obs) / dlnl)) + 2 * M + 2 \
        + 2 * margin_nodes(sigma_max_kms, dlnl)
    n = 1
    while n < need:
        n *= 2
    return n


def fourier_broaden(x, n_fft, sigma_kms, dlnl):
    """The window x convolved with a Gaussian of dispersion sigma_kms in c ln(lambda):
    edge-padded buffer of n_fft values, times exp(-2 pi^2 sigma^2 nu^2) in Fourier space."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if sigma_kms == 0.0 or n == 0:
        return x.copy()
    if n > n_fft:
        raise ValueError("window longer than the transform")
    buf = np.empty(n_fft)
    buf[:n] = x
    h = (n_fft - n + 1) // 2
    buf[n:n + h] = x[-1]
    buf[n + h:] = x[0]
    nu = np.fft.fftfreq(n_fft, d=C_KMS * dlnl)
    H = np.exp(-2.0 * math.pi ** 2 * sigma_kms ** 2 * nu ** 2)
    return np.fft.ifft(np.fft.fft(buf) * H).real[:n]
