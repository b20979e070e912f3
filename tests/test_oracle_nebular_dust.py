"""Pins for the oracle's nebular and dust steps (Sec. 2.3, 2.4, App. C, App. D.1)."""
import math

import numpy as np
import pytest

from oracle import dust, nebular
from oracle.constants import C_CMS, H_PLANCK, LSUN

ANG = 1e-8


def test_ionising_rate_matches_fnu_form_of_eq_C1():
    # eq. C1 as printed: Q = (Lsun/h) int f_nu / lambda dlambda (f_nu per Hz), here with
    # every quantity converted to cm; the oracle integrates f_lambda lambda / (h c).
    wave = np.geomspace(100.0, 5e4, 3000)
    flux = np.exp(-((np.log(wave) - np.log(600.0)) / 0.8) ** 2)[None, None, None, :] * 3.0
    Q = nebular.ionising_rate(wave, flux)[0, 0, 0]
    sel = wave <= 912.0
    lam_cm = wave[sel] * ANG
    f_lam_cm = flux[0, 0, 0, sel] / ANG              # Lsun per cm
    f_nu = f_lam_cm * lam_cm ** 2 / C_CMS            # Lsun per Hz
    integrand = f_nu / lam_cm
    q_ref = LSUN / H_PLANCK * np.sum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(lam_cm))
    assert Q == pytest.approx(q_ref, rel=1e-12, abs=0.0)


def test_ionising_rate_flat_spectrum_closed_form():
    wave = np.linspace(100.0, 1500.0, 1401)        # 1 A nodes, 912 is a node
    flux = np.full((1, 1, 1, len(wave)), 2.0)
    Q = nebular.ionising_rate(wave, flux)[0, 0, 0]
    # int_100^912 2 lambda dlambda = 912^2 - 100^2  [Lsun A per Msun]
    assert Q == pytest.approx(LSUN * ANG * (912.0 ** 2 - 100.0 ** 2) / (H_PLANCK * C_CMS), rel=1e-13, abs=0.0)


def test_line_profiles_conserve_flux_and_have_two_pixel_sigma():
    wave = np.geomspace(100.0, 5e4, 5994)
    lines = np.array([1215.67, 4862.7, 6564.6, 18756.0])
    G = nebular.line_profiles_grid(wave, lines)
    for l, lam in enumerate(lines):
        g = G[l]
        # integral over the grid, by an independent trapezoid, is 1
        assert np.trapezoid(g, wave) == pytest.approx(1.0, rel=1e-12, abs=0.0)
        mean = np.trapezoid(g * wave, wave)
        var = np.trapezoid(g * (wave - mean) ** 2, wave)
        k = np.searchsorted(wave, lam) - 1
        pix = wave[k + 1] - wave[k]
        assert abs(mean - lam) < 0.05 * pix
        assert math.sqrt(var) == pytest.approx(2.0 * pix, rel=0.03, abs=0.0)
        assert np.count_nonzero(g) <= 21


def test_bilinear_table_interpolation():
    zg = np.linspace(-1.3, 0.3, 7)
    lu = np.linspace(-4.0, -1.0, 7)
    # a bilinear function of (zg, lu) is reproduced exactly, and clamped outside
    f = lambda a, b: -12.0 + 0.3 * a - 0.2 * b + 0.05 * a * b
    table = f(zg[:, None], lu[None, :])[None, None, :, :] * np.ones((3, 2, 1, 1))
    for a, b in ((-0.77, -2.2), (0.3, -1.0), (-1.3, -4.0), (0.1, -3.999)):
        out = nebular.line_table_interp(table, zg, lu, a, b)
        assert np.allclose(out, f(a, b), atol=1e-13)
    out = nebular.line_table_interp(table, zg, lu, 2.0, -9.0)
    assert np.allclose(out, f(0.3, -4.0), atol=1e-13)


def test_line_luminosity_sum():
    rng = np.random.default_rng(1)
    W = rng.uniform(size=(1, 3, 6))
    Q = rng.uniform(1e45, 1e47, size=(1, 3, 6))
    lhat = np.full((5, 4), -12.5)
    Ll = nebular.line_luminosity(W, Q, lhat, 4)
    assert np.allclose(Ll, 10 ** -12.5 * np.sum(W[:, :, :4] * Q[:, :, :4]), rtol=1e-14)


def test_dust_zero_optical_depth_is_identity():
    wave = np.geomspace(100, 5e4, 50)
    Y, O = np.arange(50.0), np.arange(50.0)[::-1] + 1
    a, d = (wave / 5500) ** -0.7, np.ones(50)
    F = dust.attenuate(Y, O, wave, 0.0, -0.7, 0.0, 0.3, a, d)
    assert np.array_equal(F, Y + O)
    # old-only light does not see the birth cloud
    F1 = dust.attenuate(0 * Y, O, wave, 0.0, -0.7, 0.5, 0.1, a, d)
    F2 = dust.attenuate(0 * Y, O, wave, 3.0, -1.3, 0.5, 0.1, a, d)
    assert np.array_equal(F1, F2)


def test_dust_optical_depth_at_v_band():
    # at 5500 A with a(V)=1, d(V)=0 the optical depth is the parameter itself
    t = dust.diffuse_tau(np.array([5500.0]), 0.8, -0.4, np.array([1.0]), np.array([0.0]))
    assert t[0] == pytest.approx(0.8, rel=1e-15, abs=0.0)
    t = dust.birth_cloud_tau(np.array([5500.0, 11000.0]), 1.2, -0.7)
    assert t[0] == pytest.approx(1.2) and t[1] == pytest.approx(1.2 * 2 ** -0.7)
    # the bump strength falls with delta: E_b(0) = 0.85, E_b(0.2) = 0.47
    t0 = dust.diffuse_tau(np.array([5500.0]), 1.0, 0.0, np.array([0.0]), np.array([1.0]))
    t2 = dust.diffuse_tau(np.array([5500.0]), 1.0, 0.2, np.array([0.0]), np.array([1.0]))
    assert t0[0] == pytest.approx(0.85) and t2[0] == pytest.approx(0.47)
