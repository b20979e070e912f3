"""Pins for the oracle's Fourier stage: the free stellar velocity dispersion sigma_gal on
the continuum (Sec. 2.5, App. F "projected in two stages").

The stage is checked against closed forms and brute force, not against its own formula:
  - a sampled Gaussian of dispersion s comes out as the sampled Gaussian of dispersion
    sqrt(s^2 + sigma^2) with the same area (Gaussians compose in quadrature);
  - an exponential in ln(lambda) (a power law lambda^k) is an eigenfunction of the
    convolution: it comes out multiplied by exp(k^2 (sigma / c)^2 / 2) away from the edges;
  - away from the edges the result is the direct convolution, by explicit loops, with the
    normalised sampled Gaussian;
  - a window that is constant near each edge keeps those values there (the edge padding:
    the window edges are not darkened), and sigma = 0 is the identity;
  - on the whole model, the two stages (Fourier sigma_gal, then the banded kernel of the
    fixed width) agree with the single banded kernel of the total width (eq. one_kernel),
    sigma_gal = 0 leaves the model unchanged, and out-of-range values give NaN.
"""
import math

import numpy as np
import pytest

from oracle import kinematics as kin
from oracle import model as om
from oracle.constants import C_KMS
from synth import workloads as wl

DLNL = 1.0e-3                      # grid step in ln(lambda): c dlnl = 299.8 km/s


def test_gaussian_composes_in_quadrature():
    n, nfft = 600, 1024
    j = np.arange(n)
    px = C_KMS * DLNL
    for s_px, sig_kms in ((4.0, 900.0), (6.5, 300.0), (3.0, 1500.0)):
        x = np.exp(-0.5 * ((j - 301.3) / s_px) ** 2) / (math.sqrt(2 * math.pi) * s_px)
        y = kin.fourier_broaden(x, nfft, sig_kms, DLNL)
        st = math.hypot(s_px, sig_kms / px)
        ref = np.exp(-0.5 * ((j - 301.3) / st) ** 2) / (math.sqrt(2 * math.pi) * st)
        assert np.max(np.abs(y - ref)) < 1e-13 * ref.max()


def test_power_law_is_an_eigenfunction():
    n, nfft, k = 700, 2048, 10.0
    x = np.exp(k * DLNL * np.arange(n))
    # dispersions of two nodes and more: below that the multiplier is still far from zero at
    # the Nyquist frequency and the step between the padding's two edge values rings into
    # the window (3.7e-5 at 0.83 nodes, 4.5e-9 at 1.7; the paper's sampling is 2 nodes)
    for sig in (800.0, 1200.0, 2500.0):
        y = kin.fourier_broaden(x, nfft, sig, DLNL)
        m = kin.margin_nodes(sig, DLNL, 8.0)
        inner = slice(m, n - m)
        gain = math.exp(0.5 * (k * sig / C_KMS) ** 2)
        np.testing.assert_allclose(y[inner] / x[inner], gain, rtol=1e-12, atol=0.0)


def test_interior_equals_direct_convolution():
    rng = np.random.default_rng(5)
    n, nfft = 400, 1024
    x = np.exp(rng.normal(0.0, 0.5, n))
    sig = 1100.0                   # 3.67 nodes: the sampled kernel's aliasing is ~e^-66
    y = kin.fourier_broaden(x, nfft, sig, DLNL)
    s = sig / (C_KMS * DLNL)
    r = int(math.ceil(12 * s))
    g = np.array([math.exp(-0.5 * (d / s) ** 2) for d in range(-r, r + 1)])
    g /= g.sum()
    for i in range(r, n - r):
        acc = 0.0
        for d in range(-r, r + 1):
            acc += g[d + r] * x[i - d]
        assert y[i] == pytest.approx(acc, rel=1e-12, abs=0.0)


def test_edges_keep_their_values_and_zero_width_is_the_identity():
    n, nfft = 300, 512
    x = np.where(np.arange(n) < 150, 2.0, 5.0)
    y = kin.fourier_broaden(x, nfft, 900.0, DLNL)      # 3 nodes
    np.testing.assert_allclose(y[:100], 2.0, rtol=1e-12, atol=0.0)
    np.testing.assert_allclose(y[200:], 5.0, rtol=1e-12, atol=0.0)
    assert np.array_equal(kin.fourier_broaden(x, nfft, 0.0, DLNL), x)
    c = np.full(n, 3.7)
    np.testing.assert_allclose(kin.fourier_broaden(c, nfft, 2500.0, DLNL), c, rtol=1e-14, atol=0.0)


def test_window_and_length_rules():
    wave = np.exp(np.log(1000.0) + DLNL * np.arange(3000))
    j0, j1 = kin.window(wave, 6000.0, 9000.0, 1.0, 5)
    u0 = (math.log(3000.0) - math.log(1000.0)) / DLNL
    u1 = (math.log(4500.0) - math.log(1000.0)) / DLNL
    assert (j0, j1) == (math.floor(u0) - 5, math.floor(u1) + 7)
    assert wave[j0 + 5] <= 3000.0 < wave[j0 + 6] and wave[j1 - 7] <= 4500.0 < wave[j1 - 6]
    assert kin.window(wave, 6000.0, 9000.0, 500.0, 5) == (0, 0)      # below the grid
    n = kin.fft_length(6000.0, 9000.0, DLNL, 5, 1000.0)
    assert n == 512 and n >= (j1 - j0) + 2 * kin.margin_nodes(1000.0, DLNL)
    with pytest.raises(ValueError):
        kin.log_step(np.linspace(1000.0, 2000.0, 50))


# the full-size wavelength grid (c dlnl = 311 km/s), so that the widths are resolved
CFG = wl.reduced(wl.CONFIGS["c3"], n_age=30, logz=tuple(np.linspace(-2.5, 0.5, 4)), n_wave=5994, n_sfh=12, n_zh=4,
                 n_lines=0, n_pix=300)


@pytest.fixture(scope="module")
def spec_parts():
    lib = wl.make_library(CFG, 0)
    dust = wl.make_dust_tables(CFG, lib["wave"])
    L0 = om.build_library(CFG, lib, None, dust)
    L1 = om.build_library(CFG, lib, None, dust, sigma_gal_max=3000.0)
    grid = wl.make_spectrum_grid(CFG.n_pix)
    return L0, L1, grid


def _spectrum(grid, sigma_gal_fixed=0.0):
    return om.Spectrum(grid["pix_wave"], grid["lsf_mode"], grid["lsf_value"], 0.0, sigma_gal_fixed, z_ref=3.0)


def test_two_stages_equal_the_single_kernel_of_the_total_width(spec_parts):
    # eq. one_kernel: sigma_gal in the Fourier stage, then the banded kernel of sigma_fix
    # (1245 km/s), is the banded kernel of sqrt(sigma_fix^2 + sigma_gal^2); both truncate at
    # five dispersions (a tail of 6e-7 of the mass), so they agree to a few 1e-8 of the row
    L0, L1, grid = spec_parts
    th0 = wl.make_theta(CFG, 6, seed=3)
    for sg in (600.0, 1500.0, 3000.0):
        th1 = np.concatenate([th0, np.full((6, 1), sg)], axis=1)
        two = om.predict(L1, _spectrum(grid), th1)
        one = om.predict(L0, _spectrum(grid, sg), th0)
        err = np.abs(two - one) / np.abs(one).max(axis=1, keepdims=True)
        assert err.max() < 2e-7
        assert np.max(np.abs(two - om.predict(L0, _spectrum(grid), th0)) / np.abs(one).max()) > 1e-4


def test_zero_dispersion_is_the_model_without_the_stage_and_out_of_range_is_nan(spec_parts):
    L0, L1, grid = spec_parts
    th0 = wl.make_theta(CFG, 4, seed=9)
    th1 = np.concatenate([th0, np.zeros((4, 1))], axis=1)
    obs = _spectrum(grid)
    assert np.array_equal(om.predict(L1, obs, th1), om.predict(L0, obs, th0))
    th1[1, -1] = -1.0
    th1[2, -1] = 3000.5
    m = om.predict(L1, obs, th1)
    assert np.all(np.isnan(m[1])) and np.all(np.isnan(m[2])) and np.all(np.isfinite(m[[0, 3]]))
    phot = om.Photometry(filters=wl.make_filters("gauss20"))
    cfgp = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 6)), n_wave=1500, n_sfh=12,
                      n_zh=4, n_lines=0)
    lib = wl.make_library(cfgp, 0)
    dust = wl.make_dust_tables(cfgp, lib["wave"])
    P0 = om.build_library(cfgp, lib, None, dust)
    P1 = om.build_library(cfgp, lib, None, dust, sigma_gal_max=1000.0)
    tp = wl.make_theta(cfgp, 4, seed=2)
    tq = np.concatenate([tp, np.zeros((4, 1))], axis=1)
    assert np.array_equal(om.predict(P1, phot, tq), om.predict(P0, phot, tp))
    tq[:, -1] = 1000.0
    d = np.abs(om.predict(P1, phot, tq) / om.predict(P0, phot, tp) - 1.0)
    # broad bands (4-13 per cent in width) see 1000 km/s only where a break falls inside one
    assert 1e-9 < d.max() < 1e-2 and np.median(d) < 1e-4
