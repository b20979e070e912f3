"""Pins for the oracle's whole forward model: invariants stated in the paper and brute force."""
import math

import numpy as np
import pytest

from oracle import model as om
from oracle import sfh
from oracle.constants import ANG_CM, C_CMS, FNU_AB, LSUN
from synth import workloads as wl


@pytest.fixture(scope="module")
def c0():
    cfg = wl.CONFIGS["c0"]
    lib = wl.make_library(cfg, 0)
    L = om.build_library(cfg, lib, None, wl.make_dust_tables(cfg, lib["wave"]))
    return cfg, L


@pytest.fixture(scope="module")
def small_c1():
    # c1 physics on a reduced grid: 40 ages, 6 metallicities, 1500 wavelengths, 24 bins
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.5, -1.9, -1.3, -0.7, -0.1, 0.5),
                     n_wave=1500, n_sfh=24, n_zh=6, n_lines=16)
    lib = wl.make_library(cfg, 0)
    lines = wl.make_lines(cfg, lib, 1)
    L = om.build_library(cfg, lib, lines, wl.make_dust_tables(cfg, lib["wave"]))
    return cfg, L


def test_contraction_brute_force_triple_loop(small_c1):
    cfg, L = small_c1
    th = wl.make_theta(cfg, 3, seed=4)
    rf = om.rest_frame(L, th, lines_on_grid=False)
    n_af, n_z, n_age, n_w = L.flux.shape
    for b in range(3):
        W = rf["per"][b]["W"]
        Y = np.zeros(n_w)
        O = np.zeros(n_w)
        for ia in range(n_af):
            for m in range(n_z):
                for a in range(n_age):
                    if L.ages[a] < L.t_young:
                        Y += W[ia, m, a] * L.flux[ia, m, a]
                    else:
                        O += W[ia, m, a] * L.flux[ia, m, a]
        assert np.allclose(rf["Y"][b], Y, rtol=1e-12, atol=0)
        assert np.allclose(rf["O"][b], O, rtol=1e-12, atol=0)


def test_zero_optical_depth_is_identity(small_c1):
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 4, seed=5)
    th[:, cols["tau_bc"]] = 0.0
    th[:, cols["tau_diff"]] = 0.0
    rf = om.rest_frame(L, th)
    assert np.array_equal(rf["F"], rf["Y"] + rf["O"])


def test_old_only_population_ignores_birth_cloud(small_c1):
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 2, seed=6)
    m = np.zeros(cfg.n_sfh)
    m[-3:] = 1.0 / 3
    th[:, cols["sfh"]:cols["sfh"] + cfg.n_sfh] = m
    a = om.rest_frame(L, th)["F"]
    th[:, cols["tau_bc"]] = 3.7
    th[:, cols["alpha_bc"]] = -1.4
    b = om.rest_frame(L, th)["F"]
    assert np.array_equal(a, b)


def test_linear_in_mass(small_c1):
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 3, seed=7)
    obs = om.Photometry(filters=wl.make_filters("gauss20"))
    m1 = om.predict(L, obs, th)
    th2 = th.copy()
    th2[:, cols["logmass"]] += 0.37
    m2 = om.predict(L, obs, th2)
    assert np.allclose(m2, 10 ** 0.37 * m1, rtol=1e-13)


def test_single_age_bin_returns_mass_scaled_ssp(c0):
    cfg, L = c0
    for a, m in ((3, 0), (11, 2), (19, 1)):
        top = L.hi[a] if np.isfinite(L.hi[a]) else 2 * L.ages[-1]
        w = sfh.step_weights(np.array([L.lo[a], top]), np.array([2.5]), L.lo, L.hi)
        W = sfh.ssp_weights(w, np.array([L.logz[m]]), L.logz)
        spec = np.einsum("zma,zmaw->w", W, L.flux)
        assert np.array_equal(spec, 2.5 * L.flux[0, m, a])


def test_observer_frame_conserves_bolometric_flux(c0):
    """Sec. 2.6: the observer-frame F_nu, converted per node to a density per observed
    wavelength with the exact Jacobian c / lambda_obs^2, integrates to L_bol 10^logmass /
    (4 pi D_L^2).  Both sides are trapezoid sums on the same nodes (lambda_obs = (1+z)
    lambda), so they agree to rounding."""
    cfg, L = c0
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 3, seed=8)
    rf = om.rest_frame(L, th)
    for b in range(3):
        scale, dl = om.observer_scale(L, th[b], cols)
        fnu = om.fnu_observed(L, rf["F"][b], scale)
        z = th[b, cols["zred"]]
        lam_obs_cm = (1 + z) * L.wave * ANG_CM
        f_obs = np.trapezoid(fnu * C_CMS / lam_obs_cm ** 2, lam_obs_cm)   # erg/s/cm^2
        lbol = LSUN * np.trapezoid(rf["F"][b], L.wave)                    # erg/s per Msun
        expect = 10 ** th[b, cols["logmass"]] * lbol / (4 * math.pi * dl ** 2)
        assert f_obs / expect == pytest.approx(1.0, rel=1e-12, abs=0.0)


def test_lines_on_grid_carry_their_luminosity(small_c1):
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 2, seed=9)
    th[:, cols["tau_bc"]] = 0.0
    th[:, cols["tau_diff"]] = 0.0
    with_l = om.rest_frame(L, th, lines_on_grid=True)
    no_l = om.rest_frame(L, th, lines_on_grid=False)
    added = np.trapezoid(with_l["F"] - no_l["F"], L.wave, axis=1)
    assert np.allclose(added, with_l["Lline"].sum(axis=1) / LSUN, rtol=1e-12)


def test_ionising_continuum_of_nebular_ages_removed(small_c1):
    cfg, L = small_c1
    sel = L.wave < 912.0
    assert np.all(L.flux[:, :, :L.n_neb][..., sel] == 0.0)
    assert np.all(L.flux[:, :, L.n_neb:][..., sel] > 0.0)
    assert np.array_equal(L.Q, __import__("oracle.nebular", fromlist=["x"]).ionising_rate(L.wave, L.flux_raw))


def test_spectrum_mass_linearity_and_flat_parts(small_c1):
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    g = wl.make_spectrum_grid(300)
    th = wl.make_theta(cfg, 2, seed=10)
    obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"],
                      g["sigma_gal_kms"], z_ref=3.0)
    m1 = om.predict(L, obs, th)
    th[:, cols["logmass"]] -= 0.5
    m2 = om.predict(L, obs, th)
    assert np.allclose(m2, 10 ** -0.5 * m1, rtol=1e-13)
    assert np.all(np.isfinite(m1)) and np.all(m1 > 0)


def _line_free_copy(L):
    """The same library with every line table entry at 10^-300 (lines vanish, continuum unchanged)."""
    import copy
    L0 = copy.copy(L)
    L0.lines = dict(L.lines)
    L0.lines["line_table"] = np.full_like(L.lines["line_table"], -300.0)
    return L0


def test_spectral_line_flux_is_luminosity_over_4pi_dl2(small_c1):
    """App. I.1 and eq. F6: at zero optical depth a line's flux integrated over frequency
    is L 10^logmass / (4 pi D_L^2), the definition of the luminosity distance (no (1+z):
    an integrated flux carries no bandwidth factor).  The same lines placed on the model
    grid (Sec. 2.3.1) and carried to the observer frame by the photometric path's
    conversion must give the same integrated flux."""
    from oracle import cosmology
    cfg, L = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 3, seed=11)
    th[:, cols["tau_bc"]] = 0.0
    th[:, cols["tau_diff"]] = 0.0
    th[:, cols["zred"]] = (0.7, 1.3, 2.2)
    lw = L.lines["line_wave"]
    L0 = _line_free_copy(L)
    for b in range(3):
        z = th[b, cols["zred"]]
        lo, hi = 0.8 * lw.min() * (1 + z), 1.2 * lw.max() * (1 + z)
        pix = np.exp(np.arange(math.log(lo), math.log(hi), 4e-4))
        spec = om.Spectrum(pix, "R_fwhm", 100.0, 100.0, 0.0, z_ref=float(z))
        only = (om.predict(L, spec, th[b:b + 1]) - om.predict(L0, spec, th[b:b + 1]))[0] * FNU_AB
        # dnu = (c / lambda) dln(lambda); the profiles are Gaussians in ln(lambda), whose
        # trapezoid sum on this uniform ln(lambda) grid is exact to rounding
        f_spec = np.trapezoid(only * C_CMS / (pix * ANG_CM), np.log(pix))   # erg/s/cm^2
        dl = float(cosmology.luminosity_distance_cm(z, L.H0, L.Om))
        lline = om.rest_frame(L, th[b:b + 1], lines_on_grid=False)["Lline"][0]
        expect = lline.sum() * 10 ** th[b, cols["logmass"]] / (4 * math.pi * dl ** 2)
        assert f_spec / expect == pytest.approx(1.0, rel=1e-10, abs=0.0)
        # photometric path: lines on the rest grid, observer-frame F_nu, integrated over nu_obs
        rf1 = om.rest_frame(L, th[b:b + 1], lines_on_grid=True)
        rf0 = om.rest_frame(L, th[b:b + 1], lines_on_grid=False)
        scale, _ = om.observer_scale(L, th[b], cols)
        fnu = om.fnu_observed(L, rf1["F"][0] - rf0["F"][0], scale)
        lam_obs_cm = (1 + z) * L.wave * ANG_CM
        f_phot = np.trapezoid(fnu * C_CMS / lam_obs_cm ** 2, lam_obs_cm)
        assert f_phot / expect == pytest.approx(1.0, rel=1e-12, abs=0.0)


def test_flat_fnu_spectrum_returns_its_ab_maggies(small_c1):
    """Sec. 3.1/3.2: model spectra are in maggies, F_nu / 3631 Jy.  An SSP grid with
    f_lambda proportional to lambda^-2 has a flat observer-frame F_nu (Sec. 2.6); with its
    normalisation chosen from the luminosity distance so that F_nu = 3631 Jy 10^(-0.4 m),
    every pixel whose LSF row lies on the grid must return 10^(-0.4 m)."""
    import copy

    from oracle import cosmology
    cfg, Lc = small_c1
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = wl.make_theta(cfg, 2, seed=12)
    th[:, cols["tau_bc"]] = 0.0
    th[:, cols["tau_diff"]] = 0.0
    th[:, cols["zred"]] = (1.1, 3.4)
    th[:, cols["sfh"]:cols["sfh"] + cfg.n_sfh] /= th[:, cols["sfh"]:cols["sfh"] + cfg.n_sfh].sum(1, keepdims=True)
    mag = 25.0
    for b in range(2):
        z = th[b, cols["zred"]]
        dl = float(cosmology.luminosity_distance_cm(z, Lc.H0, Lc.Om))
        scale = 10 ** th[b, cols["logmass"]] * (1 + z) / (4 * math.pi * dl ** 2)
        A = FNU_AB * 10 ** (-0.4 * mag) * C_CMS / (scale * LSUN * ANG_CM)
        L = copy.copy(Lc)
        L.lines = None
        L.flux = np.broadcast_to(A / Lc.wave ** 2, Lc.flux.shape).copy()
        pix = np.geomspace(Lc.wave[40] * (1 + z), Lc.wave[-40] * (1 + z), 400)
        spec = om.Spectrum(pix, "R_fwhm", 100.0, 100.0, 0.0, z_ref=float(z))
        m = om.predict(L, spec, th[b:b + 1])[0]
        assert np.allclose(m, 10 ** (-0.4 * mag), rtol=1e-12, atol=0)
