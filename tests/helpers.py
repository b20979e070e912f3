"""Test-side setup: the same seeded synthetic inputs for the oracle and the GPU library.

Observation data are made by the oracle at a reference parameter vector
(model + 5 % Gaussian noise), then handed to both sides.
"""
from __future__ import annotations

import numpy as np

from oracle import model as om
from synth import workloads as wl


def make_case(cfg, B=None, seed=0, theta_seed=2, kind=None, n_pix=None, noise=(), wave_jitter=0.0):
    """wave_jitter > 0 moves each model wavelength by that fraction of the log step
    (sinusoidally), so that the grid is no longer log-uniform and the general
    interpolation paths are taken."""
    B = cfg.batch if B is None else B
    lib = wl.make_library(cfg, seed)
    if wave_jitter > 0.0:
        lw = np.log(lib["wave"])
        step = lw[1] - lw[0]
        lw = lw + wave_jitter * step * np.sin(0.7 * np.arange(lw.size))
        lib["wave"] = np.exp(lw)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    olib = om.build_library(cfg, lib, lines, dust)
    theta = wl.make_theta(cfg, B, seed=theta_seed)
    theta_true = wl.make_theta(cfg, 1, seed=theta_seed + 1000)
    kind = kind or ("spec" if cfg.spectrum else "phot")
    nz = {n: True for n in noise}
    if kind == "phot":
        filters = wl.make_filters(cfg.filters if cfg.filters != "none" else "gauss20")
        obs = om.Photometry(filters=filters, noise=nz)
        m_true = om.predict(olib, obs, theta_true)[0]
        obs.data, obs.sigma = wl.noisy_photometry(m_true, seed + 5)
    else:
        g = wl.make_spectrum_grid(n_pix or cfg.n_pix or 3000)
        z_true = float(theta_true[0, 1])
        obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"], g["sigma_gal_kms"],
                          z_ref=z_true, noise=nz)
        m_true = om.predict(olib, obs, theta_true)[0]
        obs.data, obs.sigma = wl.noisy_spectrum(m_true, seed + 5)
    return dict(cfg=cfg, lib=lib, lines=lines, dust=dust, olib=olib, theta=theta, theta_true=theta_true,
                obs=obs, kind=kind)


def gpu_objects(case, precisions=("fp64", "fp32"), max_batch=None):
    """Library and observation on the GPU for a case (imports the binding lazily)."""
    import paper_2609_30145_amd as sps
    cfg = case["cfg"]
    L = sps.Library(case["lib"], n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=case["dust"],
                    lines=case["lines"], precisions=precisions)
    obs = case["obs"]
    mb = max_batch or case["theta"].shape[0]
    noise = tuple(k for k, v in (obs.noise or {}).items() if v)
    if case["kind"] == "phot":
        O = sps.Observation(L, "phot", mb, filters=obs.filters, data=obs.data, sigma=obs.sigma, noise=noise)
    else:
        O = sps.Observation(L, "spec", mb, pix_wave=obs.pix_wave, lsf_mode=obs.lsf_mode, lsf_value=obs.lsf_value,
                            z_ref=obs.z_ref, sigma_gal_kms=obs.sigma_gal_kms, sigma_gas_kms=obs.sigma_gas_kms,
                            data=obs.data, sigma=obs.sigma, noise=noise)
    return L, O


def near_truth(cfg, theta_true, n, seed):
    """Perturbations of the data-generating vector: 1 % in the dust optical depths and
    the SFH bin masses, 0.004 dex in mass, 0.01 in the dust slope and the gas parameters.
    They put the logL bound to the test where a fit is within reach of the data."""
    rng = np.random.default_rng(seed)
    cols = wl.theta_columns(cfg.n_sfh, cfg.n_zh)
    th = np.repeat(theta_true, n, axis=0)
    th[:, cols["logmass"]] += 0.004 * rng.normal(size=n)
    for c in ("tau_bc", "tau_diff"):
        th[:, cols[c]] = np.clip(th[:, cols[c]] * (1.0 + 0.01 * rng.normal(size=n)), 0.0, 4.0)
    for c in ("delta", "gas_logz", "gas_logu"):
        th[:, cols[c]] += 0.01 * rng.normal(size=n)
    s0 = cols["sfh"]
    th[:, s0:s0 + cfg.n_sfh] *= 1.0 + 0.01 * rng.normal(size=(n, cfg.n_sfh))
    return th


def rel_err(got, ref, floor_frac=1e-3):
    """Per-output error relative to |ref| + floor_frac * max|ref| of the row."""
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    scale = np.abs(ref) + floor_frac * np.max(np.abs(ref), axis=1, keepdims=True)
    return np.abs(got - ref) / scale
