"""The whole forward model and logL for a batch of parameter vectors (FP64).

Order of operations (Fig. A1, Tiers A-D):
  1. per point: z -> t_univ(z), D_L(z) (Sec. 2.6); SFH edges rescaled to t_univ.
  2. SFH (step scheme) and ZH -> SSP weights W[alpha, m, a] (App. B).
  3. nebular line luminosities from the young weights and Q_ma (App. C).
  4. contraction with the SSP grid, young and old parts kept apart (eq. 1, D2);
     on the photometric path the lines are added to the young part on the model
     grid (Sec. 2.3.1); the ionising continuum of nebular-covered ages is
     removed (f_ob = 0, Fig. A1 "combine" step).
  5. attenuation F = e^{-tau_d}(Y e^{-tau_BC} + O) (App. D.1).
  6. observer frame: F_nu^obs = 10^logmass (1+z) Lsun F_lambda lambda^2 / (c 4 pi D_L^2) (Sec. 2.6).
  7. projection onto the observation (App. E or App. F) and logL (eq. 6, G1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import cosmology, dust, likelihood, nebular, projection, sfh
from .constants import ANG_CM, C_CMS, C_KMS, FNU_AB, LAM_LYMAN, LSUN

SCALARS = ("logmass", "zred", "tau_bc", "alpha_bc", "tau_diff", "delta", "logzsol",
           "gas_logz", "gas_logu", "afe", "log_err_scale", "log_f_calib", "log_f_data",
           "log_jitter")


def columns(n_sfh, n_zh):
    c = {n: i for i, n in enumerate(SCALARS)}
    c["sfh"] = len(SCALARS)
    c["zh"] = len(SCALARS) + n_sfh
    c["P"] = len(SCALARS) + n_sfh + n_zh
    return c


@dataclass
class Library:
    ages: np.ndarray
    logz: np.ndarray
    afe: np.ndarray
    wave: np.ndarray
    flux: np.ndarray          # stellar part f'_ma with the ionising mask applied
    flux_raw: np.ndarray
    t_young: float
    n_sfh: int
    T1: float
    n_zh: int
    H0: float
    Om: float
    dust_a: np.ndarray
    dust_d: np.ndarray
    young: np.ndarray = None
    lo: np.ndarray = None
    hi: np.ndarray = None
    Q: np.ndarray = None
    lines: dict | None = None
    G: np.ndarray | None = None
    n_neb: int = 0


def build_library(cfg, lib, lines=None, dust_tab=None) -> Library:
    """Static, parameter-independent preparation of the SSP grid (done once)."""
    ages, wave = lib["ages"], lib["wave"]
    flux_raw = np.asarray(lib["flux"], dtype=np.float64)
    H0, Om = cfg.cosmo
    if dust_tab is None:
        dust_tab = dict(dust_a=np.zeros_like(wave), dust_d=np.zeros_like(wave))
    L = Library(ages=ages, logz=np.asarray(lib["logz"]), afe=np.asarray(lib["afe"]), wave=wave,
                flux=flux_raw.copy(), flux_raw=flux_raw, t_young=lib["t_young"],
                n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, H0=H0, Om=Om,
                dust_a=dust_tab["dust_a"], dust_d=dust_tab["dust_d"])
    L.young = ages < L.t_young
    L.lo, L.hi = sfh.age_cells(ages)
    L.Q = nebular.ionising_rate(wave, flux_raw)
    if lines is not None:
        L.lines = lines
        L.n_neb = lines["line_table"].shape[1]
        if not np.all(L.young[:L.n_neb]) or L.n_neb != int(L.young.sum()):
            raise ValueError("line table ages must be exactly the birth-cloud ages")
        # f_ob = 0: the ionising continuum of nebular-covered ages is reprocessed
        L.flux[:, :, :L.n_neb, wave < LAM_LYMAN] = 0.0
        L.G = nebular.line_profiles_grid(wave, lines["line_wave"])
    return L


@dataclass
class Photometry:
    filters: list
    data: np.ndarray | None = None
    sigma: np.ndarray | None = None
    mask: np.ndarray | None = None
    noise: dict = field(default_factory=dict)   # {"err_scale","f_calib","f_data","jitter"}: bool
    kind: str = "phot"


@dataclass
class Spectrum:
    pix_wave: np.ndarray
    lsf_mode: str
    lsf_value: object
    sigma_gas_kms: float
    sigma_gal_kms: float
    z_ref: float
    data: np.ndarray | None = None
    sigma: np.ndarray | None = None
    mask: np.ndarray | None = None
    noise: dict = field(default_factory=dict)
    kind: str = "spec"


def point_weights(L: Library, th, cols):
    """Steps 1-2 for one parameter vector: t_univ, edges, W[alpha, m, a]."""
    z = th[cols["zred"]]
    t_univ = float(cosmology.age_of_universe_yr(z, L.H0, L.Om))
    edges = sfh.sfh_edges(t_univ, L.n_sfh, L.T1)
    masses = th[cols["sfh"]:cols["sfh"] + L.n_sfh]
    w = sfh.step_weights(edges, masses, L.lo, L.hi)
    if L.n_zh:
        zeta = sfh.bin_metallicity_hist(th[cols["zh"]:cols["zh"] + L.n_zh], edges, L.T1, t_univ)
    else:
        zeta = np.full(L.n_sfh, th[cols["logzsol"]])
    W = sfh.ssp_weights(w, zeta, L.logz, th[cols["afe"]], L.afe)
    return dict(t_univ=t_univ, edges=edges, w=w, zeta=zeta, W=W)


def point_lines(L: Library, th, cols, W):
    """Step 3: line luminosities [erg/s per Msun of the weights]."""
    if L.lines is None:
        return np.zeros(0), None
    lhat = nebular.line_table_interp(L.lines["line_table"], L.lines["zg_nodes"],
                                     L.lines["u_nodes"], th[cols["gas_logz"]], th[cols["gas_logu"]])
    return nebular.line_luminosity(W, L.Q, lhat, L.n_neb), lhat


def rest_frame(L: Library, theta, lines_on_grid=True):
    """Steps 1-5 for the whole batch: W, lines, Y, O and attenuated F [B, n_wave]."""
    theta = np.atleast_2d(theta)
    B = theta.shape[0]
    cols = columns(L.n_sfh, L.n_zh)
    n_k = L.flux.shape[0] * L.flux.shape[1] * L.flux.shape[2]
    Wk = np.zeros((B, n_k))
    per = []
    Lline = np.zeros((B, 0 if L.lines is None else len(L.lines["line_wave"])))
    for b in range(B):
        p = point_weights(L, theta[b], cols)
        Wk[b] = p["W"].reshape(-1)
        Lline[b], p["lhat"] = point_lines(L, theta[b], cols, p["W"])
        per.append(p)
    young_k = np.broadcast_to(L.young, L.flux.shape[:3]).reshape(-1)
    f = L.flux.reshape(n_k, -1)
    Y = Wk[:, young_k] @ f[young_k]
    O = Wk[:, ~young_k] @ f[~young_k]
    if L.lines is not None and lines_on_grid:
        Y = Y + (Lline / LSUN) @ L.G
    wave = L.wave
    F = np.empty_like(Y)
    for b in range(B):
        th = theta[b]
        F[b] = dust.attenuate(Y[b], O[b], wave, th[cols["tau_bc"]], th[cols["alpha_bc"]],
                              th[cols["tau_diff"]], th[cols["delta"]], L.dust_a, L.dust_d)
    return dict(per=per, W=Wk, Lline=Lline, Y=Y, O=O, F=F, cols=cols)


def observer_scale(L: Library, th, cols):
    """10^logmass * (1+z) / (4 pi D_L^2) [cm^-2] and D_L [cm]."""
    z = th[cols["zred"]]
    dl = float(cosmology.luminosity_distance_cm(z, L.H0, L.Om))
    return 10.0 ** th[cols["logmass"]] * (1.0 + z) / (4.0 * math.pi * dl * dl), dl


def fnu_observed(L: Library, F_row, scale):
    """F_nu^obs on the rest grid: scale * Lsun F_lambda[per cm] lambda^2 / c (Sec. 2.6)."""
    return scale * LSUN * F_row * L.wave ** 2 * ANG_CM / C_CMS


def line_fluxes(L: Library, th, cols, Lline, dl):
    """F_l = L_l T_BC(lambda_l) T_d(lambda_l) 10^logmass / (4 pi D_L^2) (App. I.1)."""
    lw = L.lines["line_wave"]
    a = np.interp(lw, L.wave, L.dust_a)
    d = np.interp(lw, L.wave, L.dust_d)
    T = np.exp(-dust.birth_cloud_tau(lw, th[cols["tau_bc"]], th[cols["alpha_bc"]])
               - dust.diffuse_tau(lw, th[cols["tau_diff"]], th[cols["delta"]], a, d))
    return Lline * T * 10.0 ** th[cols["logmass"]] / (4.0 * math.pi * dl * dl)


def predict(L: Library, obs, theta, rf=None, trunc=5.0):
    """Model observables [B, n] (maggies) for photometry or a spectrum."""
    theta = np.atleast_2d(theta)
    spec = obs.kind == "spec"
    if rf is None:
        rf = rest_frame(L, theta, lines_on_grid=not spec)
    cols = rf["cols"]
    out = []
    if spec:
        sig_k = projection.kernel_sigma_kms(obs.pix_wave, obs.lsf_mode, obs.lsf_value, L.wave,
                                            obs.z_ref, obs.sigma_gal_kms)
    for b in range(theta.shape[0]):
        th = theta[b]
        scale, dl = observer_scale(L, th, cols)
        fnu = fnu_observed(L, rf["F"][b], scale)
        z = th[cols["zred"]]
        if not spec:
            out.append(projection.band_maggies(L.wave, fnu, z, obs.filters))
            continue
        cont = projection.spectrum_continuum(obs.pix_wave, sig_k, L.wave, fnu, z, trunc)
        if L.lines is not None:
            Fl = line_fluxes(L, th, cols, rf["Lline"][b], dl)
            lobs = (1.0 + z) * L.lines["line_wave"]
            s_l = np.sqrt(obs.sigma_gas_kms ** 2
                          + projection.sigma_inst_kms(lobs, obs.lsf_mode,
                                                      _lsf_at(obs, lobs)) ** 2) / C_KMS
            cont = cont + projection.line_profile_pixels(obs.pix_wave, Fl, lobs, s_l)
        out.append(cont / FNU_AB)
    return np.array(out)


def _lsf_at(obs, lam_obs):
    """LSF parameter at arbitrary observed wavelengths (curves interpolate in lambda)."""
    v = np.asarray(obs.lsf_value, dtype=np.float64)
    if v.ndim == 0:
        return np.full(np.shape(lam_obs), float(v))
    return np.interp(lam_obs, obs.pix_wave, v)


def noise_terms(obs, th, cols):
    nz = obs.noise or {}
    s = math.exp(th[cols["log_err_scale"]]) if nz.get("err_scale") else 1.0
    fc = math.exp(th[cols["log_f_calib"]]) if nz.get("f_calib") else None
    fd = math.exp(th[cols["log_f_data"]]) if nz.get("f_data") else None
    j = math.exp(th[cols["log_jitter"]]) if nz.get("jitter") else None
    return s, fc, fd, j


def logl(L: Library, obs, theta, model=None, trunc=5.0):
    """logL[B] of eq. (6) with the noise floor of eq. G1."""
    theta = np.atleast_2d(theta)
    if model is None:
        model = predict(L, obs, theta, trunc=trunc)
    cols = columns(L.n_sfh, L.n_zh)
    mask = likelihood.inclusion_mask(obs.data, obs.sigma, obs.mask)
    out = np.empty(theta.shape[0])
    for b in range(theta.shape[0]):
        s, fc, fd, j = noise_terms(obs, theta[b], cols)
        out[b] = likelihood.lnlike(obs.data, model[b], obs.sigma, mask, s, fc, fd, j)
    return out
