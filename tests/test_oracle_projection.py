"""Pins for the oracle's photometric (App. E) and spectral (App. F) projections and logL."""
import math

import numpy as np
import pytest
from scipy import optimize, stats

from oracle import likelihood, projection
from oracle.constants import ANG_CM, C_CMS, C_KMS, FNU_AB
from synth import workloads as wl


# ---------------------------------------------------------------------------- photometry
def test_flat_fnu_gives_equal_ab_magnitudes_exact_on_shared_nodes():
    # observer-frame grid = rest grid * (1+z); filters whose nodes are model nodes (H = I)
    rest = np.geomspace(100.0, 5e4, 4000)
    z = 2.0
    obs = rest * (1 + z)
    filters = []
    for lo in (900, 1500, 2200, 3100):
        idx = np.nonzero((obs >= lo * 10) & (obs <= lo * 13))[0]
        R = np.exp(-0.5 * ((obs[idx] - obs[idx].mean()) / (0.1 * obs[idx].mean())) ** 2)
        R[0] = R[-1] = 0.0
        filters.append((obs[idx], R))
    mag = 21.3
    fnu = np.full_like(rest, FNU_AB * 10 ** (-0.4 * mag))
    m = projection.band_maggies(rest, fnu, z, filters)
    assert np.allclose(m, 10 ** (-0.4 * mag), rtol=1e-13)


def test_flat_fnu_generic_filters_within_interpolation_bound():
    rest = np.geomspace(100.0, 5e4, 5994)
    fnu = np.full_like(rest, FNU_AB)
    for z in (0.5, 3.3, 11.9):
        m = projection.band_maggies(rest, fnu, z, wl.make_filters("gauss20"))
        # linear interpolation of lambda^-2 between nodes spaced by dlnlambda=1.04e-3:
        # relative error <= (dlnlambda)^2 * 6/8 ~ 1e-6
        assert np.allclose(m, 1.0, rtol=2e-6)
        m = projection.band_maggies(rest, fnu, z, wl.make_filters("tophat8"))
        assert np.allclose(m, 1.0, rtol=2e-6)


def test_riemann_and_trapezoid_sums_agree_with_zero_end_nodes():
    lam, R = wl.make_filters("gauss20")[3]
    num_w = R * lam * projection.local_spacing(lam)
    from oracle.nebular import trapezoid_weights
    trap_w = R * lam * trapezoid_weights(lam)
    assert np.allclose(num_w, trap_w, rtol=1e-13)


def test_filter_interpolation_linear_is_exact():
    # an f_lambda that is linear in lambda_obs is interpolated exactly onto the filter nodes
    rest = np.geomspace(1000.0, 3e4, 700)
    z = 1.7
    lo = rest * (1 + z)
    f_lam = 1e-18 * (1.0 + 1e-5 * lo)
    fnu = f_lam * (lo * ANG_CM) ** 2 / C_CMS
    lam = np.linspace(20000.0, 30000.0, 77)
    R = np.ones(77)
    R[0] = R[-1] = 0.0
    m = projection.band_maggies(rest, fnu, z, [(lam, R)])[0]
    f_ab = FNU_AB * C_CMS / (lam * ANG_CM) ** 2
    dl = projection.local_spacing(lam)
    ref = np.sum(R * lam * dl * 1e-18 * (1 + 1e-5 * lam)) / np.sum(R * lam * dl * f_ab)
    assert m == pytest.approx(ref, rel=1e-13, abs=0.0)


# ---------------------------------------------------------------------------- spectra
def test_lsf_modes_are_consistent():
    lam = np.geomspace(6000, 53000, 50)
    R = 100.0
    r_fwhm = projection.sigma_inst_kms(lam, "R_fwhm", R)
    assert np.allclose(projection.sigma_inst_kms(lam, "fwhm_aa", lam / R), r_fwhm, rtol=1e-14)
    assert np.allclose(projection.sigma_inst_kms(lam, "sigma_aa", lam / R),
                       projection.sigma_inst_kms(lam, "R_sigma", R), rtol=1e-14)
    assert np.allclose(projection.sigma_inst_kms(lam, "fwhm_kms", 2.3548200450309493 * 300.0),
                       300.0, rtol=1e-14)
    assert r_fwhm[0] == pytest.approx(1273.1, abs=0.1)      # c / (2.3548 * 100)
    with pytest.raises(ValueError):
        projection.sigma_inst_kms(lam, "R", R)


def test_library_resolution_of_log_grid():
    rest = np.geomspace(100.0, 5e4, 5994)
    s = projection.sigma_lib_kms(rest)
    dln = math.log(500.0) / 5993
    # (c/2.3548) * 2 dlambda/lambda with dlambda/lambda = sinh(dln) on the interior
    assert np.allclose(s[1:-1], C_KMS / 2.3548200450309493 * 2 * math.sinh(dln), rtol=1e-9)
    assert s[1000] == pytest.approx(264.0, abs=0.5)


def _spec_setup():
    rest = np.geomspace(100.0, 5e4, 5994)
    pix = np.geomspace(6000.0, 53000.0, 3000)
    sig = projection.kernel_sigma_kms(pix, "R_fwhm", 100.0, rest, 2.0, 0.0)
    return rest, pix, sig


def test_lsf_rows_sum_to_one_flat_spectrum_preserved():
    rest, pix, sig = _spec_setup()
    assert np.allclose(sig, math.sqrt(1273.1 ** 2 - 264.0 ** 2), rtol=2e-3)
    out = projection.spectrum_continuum(pix, sig, rest, np.full_like(rest, 7.0), 2.0)
    assert np.allclose(out, 7.0, rtol=1e-14)


def test_lsf_gaussian_widths_compose_in_quadrature():
    rest, pix, sig = _spec_setup()
    z = 2.0
    s_in = 2e-3                       # input Gaussian dispersion in ln lambda
    x0 = math.log(20000.0 / (1 + z))
    fnu = np.exp(-0.5 * ((np.log(rest) - x0) / s_in) ** 2)
    out = projection.spectrum_continuum(pix, sig, rest, fnu, z)
    lnp = np.log(pix)
    w = out / out.sum()
    mu = np.sum(w * lnp)
    var = np.sum(w * (lnp - mu) ** 2)
    expect = s_in ** 2 + (sig[1500] / C_KMS) ** 2
    assert mu == pytest.approx(math.log(20000.0), abs=1e-4)
    assert var == pytest.approx(expect, rel=0.02, abs=0.0)


def test_narrow_lsf_reduces_to_linear_interpolation():
    rest = np.geomspace(100.0, 5e4, 5994)
    pix = np.geomspace(6000.0, 53000.0, 200)
    fnu = np.log(rest) ** 2
    out = projection.spectrum_continuum(pix, np.full(200, 1.0), rest, fnu, 0.7)
    x = np.log(pix) - math.log(1.7)
    assert np.allclose(out, np.interp(x, np.log(rest), fnu), rtol=1e-14)


def test_line_profiles_on_pixels_integrate_to_line_flux():
    pix = np.geomspace(6000.0, 53000.0, 3000)
    lobs = np.array([9000.0, 21000.0, 40000.0])
    Fl = np.array([1e-17, 3e-18, 5e-19])
    s = np.sqrt(100.0 ** 2 + 1273.1 ** 2) / C_KMS * np.ones(3)
    f = projection.line_profile_pixels(pix, Fl, lobs, s)
    nu = C_CMS / (pix * ANG_CM)
    total = -np.trapezoid(f, nu)
    assert total == pytest.approx(Fl.sum(), rel=1e-6, abs=0.0)


# ---------------------------------------------------------------------------- likelihood
def test_logl_matches_normal_logpdf_and_perfect_model():
    rng = np.random.default_rng(2)
    d = rng.normal(size=30)
    m = d + rng.normal(size=30) * 0.1
    s = rng.uniform(0.05, 0.3, 30)
    mask = likelihood.inclusion_mask(d, s)
    assert likelihood.lnlike(d, m, s, mask) == pytest.approx(stats.norm.logpdf(d, m, s).sum(), rel=1e-13, abs=0.0)
    assert likelihood.lnlike(d, d, s, mask) == pytest.approx(-0.5 * np.sum(np.log(2 * np.pi * s ** 2)),
                                                             rel=1e-14, abs=0.0)


def test_mask_excludes_bad_data():
    d = np.array([1.0, np.nan, 2.0, 3.0, 4.0])
    s = np.array([0.1, 0.1, -1.0, np.inf, 0.2])
    mask = likelihood.inclusion_mask(d, s, np.array([1, 1, 1, 1, 0]))
    assert mask.tolist() == [True, False, False, False, False]
    assert likelihood.lnlike(d, np.ones(5), s, mask) == pytest.approx(stats.norm.logpdf(1.0, 1.0, 0.1))


def test_noise_scale_maximum_at_chi2_over_n():
    rng = np.random.default_rng(3)
    d = rng.normal(size=40)
    m = np.zeros(40)
    s = np.full(40, 0.5)
    mask = likelihood.inclusion_mask(d, s)
    res = optimize.minimize_scalar(lambda sc: -likelihood.lnlike(d, m, s, mask, s=sc),
                                   bounds=(0.1, 10), method="bounded", options=dict(xatol=1e-10))
    chi2 = np.sum((d / s) ** 2)
    assert res.x == pytest.approx(math.sqrt(chi2 / 40), rel=1e-6, abs=0.0)


def test_noise_floor_terms_add_in_quadrature():
    v = likelihood.effective_variance(np.array([2.0]), np.array([-10.0]), np.array([5.0]),
                                      s=1.5, f_calib=0.1, f_data=0.2, jitter=0.3)
    assert v[0] == pytest.approx(9.0 + 1.0 + 1.0 + 0.09)
