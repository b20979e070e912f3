"""Pins for the oracle's analytic marginalisation of line fluxes (Sec. 4.1, App. I.3,
eq. app_line_marg).

The closed form is checked against direct numerical integration of its definition, the
Gaussian likelihood of the model with the line fluxes as free amplitudes times their prior
(Gaussian around the grid flux, or flat), over one and two amplitudes; the narrow-prior limit
is the likelihood at the grid fluxes; the posterior mean of flat lines is the least-squares
flux (it recovers known fluxes from noise-free data); and on the whole model, lines outside
the pixel range do not enter, and the posterior mean recovers the fluxes a spectrum was made
with.

The joint marginalisation over a spectrum and a line catalogue of one object is checked
against the closed-form Gaussian convolution of a catalogue-only line, against direct
numerical integration over two amplitudes seen by both observations (a blend and an
upper limit among the entries), and reduces to the spectrum's own marginal when the
catalogue has no detection.  With photometry as well: the band responses of all the
library's lines times their grid fluxes are exactly the model's line contribution to each
band (the model with and without its lines on the grid), and the three-observation closed
form matches direct integration.
"""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import likelihood as lk
from oracle import model as om
from synth import workloads as wl


def _toy(n=120, seed=0):
    rng = np.random.default_rng(seed)
    x = np.linspace(-1.0, 1.0, n)
    mu = 1.0 + 0.2 * x
    prof = np.stack([np.exp(-0.5 * ((x - c) / 0.06) ** 2) for c in (-0.3, -0.18)], axis=1)
    sigma = 0.05 + 0.01 * rng.random(n)
    mask = np.ones(n, dtype=bool)
    mask[[5, 40]] = False
    return x, mu, prof, sigma, mask, rng


def _direct(d, mu, A, sigma, mask, alpha_bar, sd, flat, grids):
    """ln of the integral over alpha of N(d; mu + A alpha, sigma^2) p(alpha) on a grid."""
    mesh = np.meshgrid(*grids, indexing="ij")
    al = np.stack([m.ravel() for m in mesh], axis=1)
    dv = np.prod([g[1] - g[0] for g in grids])
    v = np.where(mask, sigma, 1.0) ** 2
    vals = []
    for a in al:
        r = np.where(mask, d - mu - A @ a, 0.0)
        ll = np.sum(np.where(mask, -0.5 * r * r / v - 0.5 * np.log(2 * np.pi * v), 0.0))
        lp = sum(0.0 if flat[j] else -0.5 * ((a[j] - alpha_bar[j]) / sd[j]) ** 2 - 0.5 * math.log(2 * math.pi * sd[j] ** 2)
                 for j in range(len(a)))
        vals.append(ll + lp)
    return logsumexp(vals) + math.log(dv)


@pytest.mark.parametrize("flat", [(False,), (True,)])
def test_one_line_matches_direct_integration(flat):
    x, mu, prof, sigma, mask, rng = _toy()
    A = prof[:, :1]
    a_true, a_bar = 0.8, 0.7
    d = mu + A[:, 0] * a_true + sigma * rng.normal(size=x.size)
    sd = np.array([0.2])
    model = mu + A[:, 0] * a_bar
    closed = lk.line_marginal_lnlike(d, model, sigma, mask, A, np.array([a_bar]), sd, np.array(flat))
    g = np.linspace(0.3, 1.3, 8001)
    assert closed == pytest.approx(_direct(d, mu, A, sigma, mask, [a_bar], sd, flat, [g]), rel=0.0, abs=1e-8)


def test_two_overlapping_lines_match_direct_integration():
    x, mu, prof, sigma, mask, rng = _toy(seed=1)
    a_true, a_bar = np.array([0.5, 0.9]), np.array([0.6, 0.8])
    d = mu + prof @ a_true + sigma * rng.normal(size=x.size)
    sd = np.array([0.15, 0.3])
    flat = np.array([False, True])
    model = mu + prof @ a_bar
    closed = lk.line_marginal_lnlike(d, model, sigma, mask, prof, a_bar, sd, flat)
    g0 = np.linspace(0.2, 0.85, 601)
    g1 = np.linspace(0.45, 1.4, 601)
    assert closed == pytest.approx(_direct(d, mu, prof, sigma, mask, a_bar, sd, flat, [g0, g1]), rel=0.0, abs=1e-5)


def test_narrow_prior_is_the_likelihood_at_the_grid_fluxes():
    x, mu, prof, sigma, mask, rng = _toy(seed=2)
    a_bar = np.array([0.6, 0.8])
    d = mu + prof @ np.array([0.5, 0.9]) + sigma * rng.normal(size=x.size)
    model = mu + prof @ a_bar
    got = lk.line_marginal_lnlike(d, model, sigma, mask, prof, a_bar, 1e-9 * a_bar, np.zeros(2, dtype=bool))
    assert got == pytest.approx(lk.lnlike(d, model, sigma, mask), rel=0.0, abs=1e-9)


def test_flat_posterior_mean_recovers_the_fluxes():
    x, mu, prof, sigma, mask, _ = _toy(seed=3)
    a_true = np.array([0.37, 1.21])
    d = mu + prof @ a_true
    model = mu + prof @ np.array([0.1, 0.1])
    _, mean = lk.line_marginal_lnlike(d, model, sigma, mask, prof, np.array([0.1, 0.1]), np.ones(2),
                                      np.ones(2, dtype=bool), return_mean=True)
    np.testing.assert_allclose(mean, a_true, rtol=1e-12, atol=0.0)


CFG = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 6)), n_wave=1500, n_sfh=12, n_zh=4,
                 n_lines=24, n_pix=300)


@pytest.fixture(scope="module")
def spec_case():
    lib = wl.make_library(CFG, 0)
    lines = wl.make_lines(CFG, lib, 1)
    dust = wl.make_dust_tables(CFG, lib["wave"])
    L = om.build_library(CFG, lib, lines, dust)
    g = wl.make_spectrum_grid(CFG.n_pix)
    th = wl.make_theta(CFG, 4, seed=5)
    th[:, 1] = [1.0, 2.5, 4.0, 6.0]
    obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"], 0.0, z_ref=2.5)
    return L, obs, th


def test_model_lines_outside_the_pixels_do_not_enter(spec_case):
    L, obs, th = spec_case
    cols = om.lib_columns(L)
    rf = om.rest_frame(L, th, lines_on_grid=False)
    lw = L.lines["line_wave"]
    for b in range(th.shape[0]):
        obs.line_marg, obs.line_prior_frac = "gauss", 0.3
        t = om.line_marg_terms(L, obs, th[b], cols, rf["Lline"][b])
        lobs = (1.0 + th[b, 1]) * lw[t["idx"]]
        assert np.all((lobs >= obs.pix_wave[0]) & (lobs <= obs.pix_wave[-1]))
        out = np.setdiff1d(np.arange(len(lw)), t["idx"])
        lo = (1.0 + th[b, 1]) * lw[out]
        assert np.all((lo < obs.pix_wave[0]) | (lo > obs.pix_wave[-1]) | (rf["Lline"][b][out] <= 0.0))


def test_model_marginal_likelihood_limits_and_recovery(spec_case):
    L, obs, th = spec_case
    cols = om.lib_columns(L)
    obs.line_marg, obs.line_prior_frac, obs.line_flat = None, 0.0, None
    m = om.predict(L, obs, th)
    sigma = 0.02 * np.abs(m[1]) + 0.01 * np.median(np.abs(m[1]))
    # data: the model of point 1 with its window's line fluxes scaled by 1.5
    rf = om.rest_frame(L, th, lines_on_grid=False)
    obs.line_marg, obs.line_prior_frac = "flat", 0.0
    t = om.line_marg_terms(L, obs, th[1], cols, rf["Lline"][1])
    assert len(t["idx"]) >= 3
    d = m[1] + t["A"] @ (0.5 * t["alpha_bar"])
    obs.data, obs.sigma = d, sigma
    mask = np.ones(d.size, dtype=bool)
    _, mean = lk.line_marginal_lnlike(d, m[1], sigma, mask, t["A"], t["alpha_bar"], t["prior_sd"], t["flat"],
                                      return_mean=True)
    np.testing.assert_allclose(mean, 1.5 * t["alpha_bar"], rtol=1e-8, atol=1e-10 * t["alpha_bar"].max())
    # a narrow Gaussian prior gives the likelihood at the grid fluxes
    obs.line_marg, obs.line_prior_frac = "gauss", 1e-10
    obs.noise = {}
    narrow = om.logl(L, obs, th, model=m)
    obs.line_marg = None
    plain = om.logl(L, obs, th, model=m)
    np.testing.assert_allclose(narrow, plain, rtol=1e-9, atol=1e-6)


def _spec(d, mu_model, sigma, mask, A):
    return dict(data=d, model=mu_model, sigma=sigma, mask=mask, A=A)


def test_joint_catalogue_only_line_is_the_gaussian_convolution():
    x, mu, prof, sigma, mask, rng = _toy(seed=4)
    d = mu + sigma * rng.normal(size=x.size)
    F, sd, dc, sc = 0.8, 0.25, 1.1, 0.3
    spec = _spec(d, mu, sigma, mask, np.zeros((x.size, 1)))      # the line misses the spectrum
    cat = dict(data=np.array([dc]), model=np.array([F]), sigma=np.array([sc]), mask=np.array([True]),
               upper=np.array([False]), A=np.ones((1, 1)))
    got = lk.joint_line_marginal_lnlike(spec, cat, np.array([F]), np.array([sd]), np.array([False]))
    # integral of exp(-(d - a)^2 / 2 sc^2) N(a; F, sd^2) da
    want = lk.lnlike(d, mu, sigma, mask) + math.log(sc / math.sqrt(sc ** 2 + sd ** 2)) \
        - 0.5 * (dc - F) ** 2 / (sc ** 2 + sd ** 2)
    assert got == pytest.approx(want, rel=0.0, abs=1e-10)


def test_joint_matches_direct_integration_over_two_lines():
    x, mu, prof, sigma, mask, rng = _toy(seed=5)
    a_true, a_bar = np.array([0.5, 0.9]), np.array([0.6, 0.8])
    sd = np.array([0.15, 0.3])
    flat = np.array([False, True])
    d = mu + prof @ a_true + sigma * rng.normal(size=x.size)
    model = mu + prof @ a_bar
    # catalogue: line 0, the blend of both, and an upper limit on line 1 the grid model exceeds
    Ac = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    dc = np.array([0.55, 1.35, 0.6])
    sc = np.array([0.05, 0.1, 0.2])
    up = np.array([False, False, True])
    mc = Ac @ a_bar
    spec = _spec(d, model, sigma, mask, prof)
    cat = dict(data=dc, model=mc, sigma=sc, mask=np.ones(3, dtype=bool), upper=up, A=Ac)
    closed = lk.joint_line_marginal_lnlike(spec, cat, a_bar, sd, flat)
    g0 = np.linspace(0.25, 0.85, 601)
    g1 = np.linspace(0.5, 1.25, 601)
    A0, A1 = np.meshgrid(g0, g1, indexing="ij")
    v = np.where(mask, sigma, 1.0) ** 2
    ul = -0.5 * ((dc[2] - mc[2]) / sc[2]) ** 2 if mc[2] > dc[2] else 0.0
    vals = np.empty(A0.shape)
    for i in range(A0.shape[0]):
        for j in range(A0.shape[1]):
            a = np.array([A0[i, j], A1[i, j]])
            r = np.where(mask, d - mu - prof @ a, 0.0)
            ll = np.sum(np.where(mask, -0.5 * r * r / v - 0.5 * np.log(2 * np.pi * v), 0.0))
            rc = dc[:2] - Ac[:2] @ a
            ll += -0.5 * np.sum((rc / sc[:2]) ** 2) + ul
            ll += -0.5 * ((a[0] - a_bar[0]) / sd[0]) ** 2 - 0.5 * math.log(2 * math.pi * sd[0] ** 2)
            vals[i, j] = ll
    direct = logsumexp(vals) + math.log((g0[1] - g0[0]) * (g1[1] - g1[0]))
    assert closed == pytest.approx(direct, rel=0.0, abs=1e-5)


def test_joint_without_catalogue_detections_is_the_spectrum_marginal():
    x, mu, prof, sigma, mask, rng = _toy(seed=6)
    a_bar = np.array([0.6, 0.8])
    d = mu + prof @ np.array([0.5, 0.9]) + sigma * rng.normal(size=x.size)
    model = mu + prof @ a_bar
    sd = np.array([0.2, 0.1])
    flat = np.array([True, False])
    spec = _spec(d, model, sigma, mask, prof)
    # one masked detection and an upper limit above the grid model: neither contributes
    cat = dict(data=np.array([np.nan, 5.0]), model=np.array([0.6, 1.4]), sigma=np.array([0.1, 0.1]),
               mask=np.array([False, True]), upper=np.array([False, True]), A=np.array([[1.0, 0.0], [1.0, 1.0]]))
    got = lk.joint_line_marginal_lnlike(spec, cat, a_bar, sd, flat)
    want = lk.line_marginal_lnlike(d, model, sigma, mask, prof, a_bar, sd, flat)
    assert got == pytest.approx(want, rel=1e-14, abs=1e-10)


def test_band_responses_times_fluxes_are_the_models_line_contribution():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 6)), n_wave=1500, n_sfh=12,
                     n_zh=4, n_lines=24)
    lib = wl.make_library(cfg, 0)
    lines = wl.make_lines(cfg, lib, 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    for kw in (dict(), dict(escape="runaway_bc", igm=True)):
        L = om.build_library(cfg, lib, lines, dust, **kw)
        cols = om.lib_columns(L)
        phot = om.Photometry(filters=wl.make_filters("gauss20"))
        th = wl.make_theta(cfg, 3, seed=9, escape=bool(kw), igm=bool(kw))
        th[:, 1] = [0.7, 2.5, 6.0]
        with_lines = om.predict(L, phot, th)
        no_lines = om.predict(L, phot, th, rf=om.rest_frame(L, th, lines_on_grid=False))
        rf = om.rest_frame(L, th, lines_on_grid=False)
        idx = np.arange(cfg.n_lines)
        for b in range(th.shape[0]):
            A = om.line_band_response(L, phot, th[b], cols, rf["Lline"][b], idx)
            _, dl = om.observer_scale(L, th[b], cols)
            Fl = om.line_fluxes(L, th[b], cols, rf["Lline"][b], dl)
            np.testing.assert_allclose(A @ Fl, with_lines[b] - no_lines[b], rtol=1e-10,
                                       atol=1e-12 * np.max(np.abs(with_lines[b])))


def test_joint_with_photometry_matches_direct_integration():
    x, mu, prof, sigma, mask, rng = _toy(seed=7)
    a_true, a_bar = np.array([0.5, 0.9]), np.array([0.6, 0.8])
    sd = np.array([0.15, 0.3])
    flat = np.array([False, True])
    d = mu + prof @ a_true + sigma * rng.normal(size=x.size)
    model = mu + prof @ a_bar
    # three bands that see the lines with different responses, one masked
    Ap = np.array([[0.8, 0.1], [0.3, 0.6], [0.5, 0.5]])
    mp0 = np.array([2.0, 1.5, 1.0])
    dp = mp0 + Ap @ a_true + np.array([0.02, -0.03, 0.0])
    sp = np.array([0.05, 0.04, 0.05])
    mkp = np.array([True, True, False])
    spec = _spec(d, model, sigma, mask, prof)
    phot = dict(data=dp, model=mp0 + Ap @ a_bar, sigma=sp, mask=mkp, A=Ap)
    closed = lk.joint_line_marginal_lnlike(spec, None, a_bar, sd, flat, phot=phot)
    g0 = np.linspace(0.3, 0.75, 451)
    g1 = np.linspace(0.6, 1.2, 451)
    v = np.where(mask, sigma, 1.0) ** 2
    vals = np.empty((g0.size, g1.size))
    for i, a0 in enumerate(g0):
        for j, a1 in enumerate(g1):
            a = np.array([a0, a1])
            r = np.where(mask, d - mu - prof @ a, 0.0)
            ll = np.sum(np.where(mask, -0.5 * r * r / v - 0.5 * np.log(2 * np.pi * v), 0.0))
            rp = (dp - mp0 - Ap @ a)[mkp]
            ll += np.sum(-0.5 * (rp / sp[mkp]) ** 2 - 0.5 * np.log(2 * np.pi * sp[mkp] ** 2))
            ll += -0.5 * ((a0 - a_bar[0]) / sd[0]) ** 2 - 0.5 * math.log(2 * math.pi * sd[0] ** 2)
            vals[i, j] = ll
    direct = logsumexp(vals) + math.log((g0[1] - g0[0]) * (g1[1] - g1[0]))
    assert closed == pytest.approx(direct, rel=0.0, abs=1e-5)
