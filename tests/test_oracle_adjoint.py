"""Pins for the oracle's hand-written adjoint: central finite differences (h = 1e-6)
of the oracle forward model, plus the closed form of d logL / d logmass.

Smooth synthetic libraries (no per-pixel noise) keep the finite differences away
from the kinks of the piecewise-linear redshift interpolation; spectral tests
widen the LSF truncation so that no tap enters or leaves a window under a step.
"""
import math

import numpy as np
import pytest

from oracle import adjoint
from oracle import model as om
from synth import workloads as wl


def _case(cfg, kind, B=3, seed=0, noise=(), n_pix=None):
    lib = wl.make_library(cfg, seed, noise=0.0)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = om.build_library(cfg, lib, lines, dust)
    th_true = wl.make_theta(cfg, 1, seed=11)
    nz = {k: True for k in noise}
    if kind == "phot":
        obs = om.Photometry(filters=wl.make_filters(cfg.filters if cfg.filters != "none" else "gauss20"), noise=nz)
        m = om.predict(L, obs, th_true)[0]
        obs.data, obs.sigma = wl.noisy_photometry(m, 3)
    else:
        g = wl.make_spectrum_grid(n_pix)
        obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"], g["sigma_gal_kms"],
                          z_ref=float(th_true[0, 1]), noise=nz)
        m = om.predict(L, obs, th_true)[0]
        obs.data, obs.sigma = wl.noisy_spectrum(m, 3)
    theta = wl.perturb_theta(cfg, np.repeat(th_true, B, axis=0), 0.05, seed=21)
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    for name in noise:
        theta[:, cols["log_" + name if name != "err_scale" else "log_err_scale"]] = np.log(0.05)
    return L, obs, theta


def _fd(L, obs, th, cols_to_check, h=1e-6, trunc=5.0):
    out = {}
    for c in cols_to_check:
        tp, tm = th.copy(), th.copy()
        tp[c] += h
        tm[c] -= h
        out[c] = (om.logl(L, obs, tp, trunc=trunc)[0] - om.logl(L, obs, tm, trunc=trunc)[0]) / (2 * h)
    return out


def _check(L, obs, theta, cols, trunc=5.0, tol=2e-5):
    for b in range(theta.shape[0]):
        ll, g = adjoint.grad_point(L, obs, theta[b], trunc)
        assert ll == pytest.approx(om.logl(L, obs, theta[b], trunc=trunc)[0], rel=1e-12, abs=0.0)
        fd = _fd(L, obs, theta[b], cols, trunc=trunc)
        gmax = max(abs(v) for v in fd.values())
        for c, v in fd.items():
            assert abs(g[c] - v) <= tol * (abs(v) + 1e-3 * gmax), (b, c, g[c], v)


def test_adjoint_photometry_constant_metallicity():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=30, logz=(-2.0, -1.0, 0.0, 0.4), n_wave=1200, n_sfh=12, n_zh=0,
                     n_lines=0)
    L, obs, theta = _case(cfg, "phot")
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    check = [cols[n] for n in ("logmass", "zred", "tau_bc", "alpha_bc", "tau_diff", "delta", "logzsol")]
    check += list(range(cols["sfh"], cols["sfh"] + cfg.n_sfh))
    _check(L, obs, theta, check)


def test_adjoint_photometry_enrichment_history_and_lines():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 7)), n_wave=1500, n_sfh=16,
                     n_zh=5, n_lines=20)
    L, obs, theta = _case(cfg, "phot")
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    check = [cols[n] for n in ("logmass", "zred", "tau_bc", "alpha_bc", "tau_diff", "delta", "gas_logz",
                               "gas_logu")]
    check += list(range(cols["sfh"], cols["P"]))
    _check(L, obs, theta, check)


def test_adjoint_spectrum_with_lines():
    cfg = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 7)), n_wave=1500, n_sfh=12,
                     n_zh=4, n_lines=20)
    L, obs, theta = _case(cfg, "spec", B=2, n_pix=300)
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    check = [cols[n] for n in ("logmass", "zred", "tau_bc", "alpha_bc", "tau_diff", "delta", "gas_logz",
                               "gas_logu")]
    check += list(range(cols["sfh"], cols["P"]))
    _check(L, obs, theta, check, trunc=12.0)


def test_adjoint_alpha_axis_and_noise_floor():
    cfg = wl.reduced(wl.CONFIGS["c4"], n_age=30, logz=(-2.0, -1.0, 0.0), afe=(0.0, 0.2, 0.4), n_wave=1000,
                     n_sfh=10)
    L, obs, theta = _case(cfg, "phot", noise=("err_scale", "f_calib", "f_data", "jitter"))
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    theta[:, cols["log_jitter"]] = np.log(1e-9)
    check = [cols[n] for n in ("logmass", "zred", "afe", "logzsol", "log_err_scale", "log_f_calib",
                               "log_f_data", "log_jitter")]
    _check(L, obs, theta, check)


def test_logmass_gradient_closed_form():
    cfg = wl.CONFIGS["c0"]
    L, obs, theta = _case(cfg, "phot")
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    for b in range(3):
        m = om.predict(L, obs, theta[b])[0]
        expect = math.log(10) * np.sum(m * (obs.data - m) / obs.sigma ** 2)
        _, g = adjoint.grad_point(L, obs, theta[b])
        assert g[cols["logmass"]] == pytest.approx(expect, rel=1e-12, abs=0.0)
