"""The whole forward model and logL for a batch of parameter vectors (FP64).

Order of operations (Fig. A1, Tiers A-D):
  1. per point: z -> t_univ(z), D_L(z) (Sec. 2.6); SFH edges rescaled to t_univ.
  2. SFH (step scheme) and ZH -> SSP weights W[alpha, m, a] (App. B).
  3. nebular line luminosities and continuum from the weights and Q_ma (App. C),
     each cube interpolated trilinearly in (Z_gas, age, log U).
  4. contraction with the SSP grid, young and old parts kept apart (eq. 1, D2);
     on the photometric path the lines are added to the young part on the model
     grid (Sec. 2.3.1); the ionising continuum of nebular-covered ages is
     removed from the young part (Fig. A1 "combine" step) and, with an escape
     geometry, a fraction f_ob of it restored (Sec. 2.3.2, App. D.1).
  5. attenuation F = e^{-tau_d}(Y e^{-tau_BC} + O) (App. D.1), or its escape-geometry
     forms (eq. runaway_mix; the picket fence of Sec. 2.3.2).
  6. observer frame: F_nu^obs = 10^logmass (1+z) Lsun F_lambda lambda^2 / (c 4 pi D_L^2) (Sec. 2.6).
  7. projection onto the observation (App. E or App. F) and logL (eq. 6, G1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import cosmology, dust, igm, kinematics, likelihood, nebular, projection, sfh
from .constants import ANG_CM, C_CMS, C_KMS, FNU_AB, LAM_LYMAN, LSUN

SCALARS = ("logmass", "zred", "tau_bc", "alpha_bc", "tau_diff", "delta", "logzsol",
           "gas_logz", "gas_logu", "afe", "log_err_scale", "log_f_calib", "log_f_data",
           "log_jitter")


ESCAPE_GEOMETRIES = ("none", "runaway_bc", "picket")


def columns(n_sfh, n_zh, escape=False, igm=0, vdisp=False):
    """Column offsets of theta: the scalars, the SFH values (bin masses, or node SFRs under
    the linear scheme), the enrichment nodes, then frac_obrun = f_ob for a library with an
    escape geometry (Sec. 2.3.2); for one with IGM transmission (Sec. 2.6; igm a bit mask,
    IGM_* below) igm_factor, then x_HI with the damping wing and logN_HI, z_dla with the
    absorber; sigma_gal [km/s] for one with a free stellar velocity dispersion (Sec. 2.5)."""
    c = {n: i for i, n in enumerate(SCALARS)}
    c["sfh"] = len(SCALARS)
    c["zh"] = len(SCALARS) + n_sfh
    c["P"] = len(SCALARS) + n_sfh + n_zh
    if escape:
        c["frac_obrun"] = c["P"]
        c["P"] += 1
    igm = int(igm)
    if igm & IGM_MADAU:
        c["igm_factor"] = c["P"]
        c["P"] += 1
    if igm & IGM_DAMPING:
        c["x_hi"] = c["P"]
        c["P"] += 1
    if igm & IGM_DLA:
        c["log_nhi"] = c["P"]
        c["z_dla"] = c["P"] + 1
        c["P"] += 2
    if vdisp:
        c["sigma_gal"] = c["P"]
        c["P"] += 1
    return c


IGM_MADAU, IGM_DAMPING, IGM_DLA = 1, 2, 4   # IGM bit mask: the additions need the Madau IGM


def lib_columns(L):
    """columns() for a library."""
    return columns(L.n_sfh, L.n_zh, L.escape != "none", L.igm, L.sigma_gal_max > 0.0)


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
    n_neb: int = 0            # nebular-covered ages are [neb_a0, n_neb)
    neb_a0: int = 0
    cont: dict | None = None  # nebular continuum cube (App. C) or None
    escape: str = "none"      # fesc_geometry: "none" (f_ob = 0), "runaway_bc", "picket"
    sfh_scheme: str = "step"  # SFH -> age weights: "step" or "linear" (App. B)
    igm: int = 0              # IGM bit mask: Madau (1995) with theta[igm_factor], + damping wing, + DLA
    sigma_gal_max: float = 0.0  # > 0: theta[sigma_gal] in [0, sigma_gal_max] km/s, Fourier stage
    flux_ion: np.ndarray | None = None   # raw ionising continuum of nebular-covered ages


def build_library(cfg, lib, lines=None, dust_tab=None, cont=None, escape="none", sfh_scheme="step",
                  igm=False, sigma_gal_max=0.0) -> Library:
    """Static, parameter-independent preparation of the SSP grid (done once).

    ``lines``: line_wave, line_table [n_line][n_tau][n_zg][n_u] of log10(L_l/Q), zg_nodes,
    u_nodes and, optionally, line_tau (the table's own age axis; without it the age axis
    is the set of birth-cloud SSP ages).  ``cont``: cont_table [n_tau][n_zg][n_u][n_wave]
    of log10(L_nu/Q) on the library's wavelengths with its own tau_nodes, zg_nodes and
    u_nodes (App. C).  Nebular emission goes to the SSP ages inside every cube's age
    range; they must be birth-cloud ages.  ``escape`` selects the f_ob geometry,
    ``sfh_scheme`` the step or linear (tent-integral) weights, ``igm`` the IGM transmission
    (True or IGM_MADAU, optionally | IGM_DAMPING, | IGM_DLA),
    ``sigma_gal_max`` > 0 a free stellar velocity dispersion up to that value [km/s],
    applied in the Fourier stage (the grid must then be uniform in ln lambda).
    """
    ages, wave = lib["ages"], lib["wave"]
    flux_raw = np.asarray(lib["flux"], dtype=np.float64)
    H0, Om = cfg.cosmo
    if dust_tab is None:
        dust_tab = dict(dust_a=np.zeros_like(wave), dust_d=np.zeros_like(wave))
    if escape not in ESCAPE_GEOMETRIES:
        raise ValueError(f"escape geometry must be one of {ESCAPE_GEOMETRIES}")
    L = Library(ages=ages, logz=np.asarray(lib["logz"]), afe=np.asarray(lib["afe"]), wave=wave,
                flux=flux_raw.copy(), flux_raw=flux_raw, t_young=lib["t_young"],
                n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, H0=H0, Om=Om,
                dust_a=dust_tab["dust_a"], dust_d=dust_tab["dust_d"])
    L.young = ages < L.t_young
    L.lo, L.hi = sfh.age_cells(ages)
    L.Q = nebular.ionising_rate(wave, flux_raw)
    L.escape = escape
    if sfh_scheme not in ("step", "linear"):
        raise ValueError("sfh_scheme must be 'step' or 'linear'")
    L.sfh_scheme = sfh_scheme
    L.igm = int(igm)
    if L.igm not in (0, 1, 3, 5, 7):
        raise ValueError("igm: 0, or IGM_MADAU with optional IGM_DAMPING and IGM_DLA")
    if sigma_gal_max < 0.0 or not math.isfinite(sigma_gal_max):
        raise ValueError("sigma_gal_max must be finite and >= 0")
    if sigma_gal_max > 0.0:
        kinematics.log_step(wave)
    L.sigma_gal_max = float(sigma_gal_max)
    ranges = []
    if lines is not None:
        L.lines = dict(lines)
        if "line_tau" not in lines or lines["line_tau"] is None:
            n_y = int(L.young.sum())
            if lines["line_table"].shape[1] != n_y:
                raise ValueError("a line table without its own age axis must be on the birth-cloud ages")
            L.lines["line_tau"] = ages[:n_y].copy()
        lt = L.lines["line_tau"]
        ranges.append((lt[0], lt[-1]))
        L.G = nebular.line_profiles_grid(wave, lines["line_wave"])
    if cont is not None:
        if cont["cont_table"].shape[-1] != len(wave):
            raise ValueError("the continuum cube must be tabulated on the library wavelengths")
        L.cont = dict(cont)
        ranges.append((cont["tau_nodes"][0], cont["tau_nodes"][-1]))
    if ranges:
        sel = nebular.nebular_age_mask(ages, ranges)
        idx = np.flatnonzero(sel)
        if len(idx) == 0:
            raise ValueError("no SSP age falls inside the nebular grids' age range")
        if np.any(~L.young[idx]):
            raise ValueError("nebular-covered SSP ages must be birth-cloud ages")
        L.neb_a0, L.n_neb = int(idx[0]), int(idx[-1]) + 1
        ion = wave < LAM_LYMAN
        # the ionising continuum of nebular-covered ages is reprocessed (absent from the
        # young stellar light); an escape geometry restores a fraction f_ob of it
        L.flux_ion = np.zeros_like(flux_raw)
        L.flux_ion[:, :, L.neb_a0:L.n_neb, ion] = flux_raw[:, :, L.neb_a0:L.n_neb, ion]
        L.flux[:, :, L.neb_a0:L.n_neb, ion] = 0.0
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
    # spectrophotometric calibration polynomial (Sec. 3.2, App. H.3): None, "marginal" or
    # "optimise", the Chebyshev order and the prior widths s_m of the coefficients
    calib: str | None = None
    calib_order: int = 0
    calib_prior: np.ndarray | None = None
    # analytic marginalisation of the line fluxes (Sec. 4.1, App. I.3): None, "gauss" (prior
    # N(F_l, (frac F_l)^2) around the grid flux, flat for the lines flagged in line_flat) or
    # "flat" (every line flat)
    line_marg: str | None = None
    line_prior_frac: float = 0.0
    line_flat: np.ndarray | None = None


@dataclass
class Lines:
    """Emission-line catalogue (Sec. 3.3, App. I): entry k is the sum of the library lines
    blends[k] (an unresolved blend); integrated fluxes in erg/s/cm^2; upper[k] flags an
    upper limit."""
    blends: list
    data: np.ndarray | None = None
    sigma: np.ndarray | None = None
    mask: np.ndarray | None = None
    upper: np.ndarray | None = None
    kind: str = "lines"


def point_weights(L: Library, th, cols):
    """Steps 1-2 for one parameter vector: t_univ, edges, W[alpha, m, a]."""
    z = th[cols["zred"]]
    t_univ = float(cosmology.age_of_universe_yr(z, L.H0, L.Om))
    edges = sfh.sfh_edges(t_univ, L.n_sfh, L.T1)
    vals = th[cols["sfh"]:cols["sfh"] + L.n_sfh]
    if L.sfh_scheme == "linear":
        w = sfh.tent_weights(edges, vals, L.ages)
    else:
        w = sfh.step_weights(edges, vals, L.lo, L.hi)
    if L.n_zh:
        zeta = sfh.bin_metallicity_hist(th[cols["zh"]:cols["zh"] + L.n_zh], edges, L.T1, t_univ)
    else:
        zeta = np.full(L.n_sfh, th[cols["logzsol"]])
    W = sfh.ssp_weights(w, zeta, L.logz, th[cols["afe"]], L.afe)
    return dict(t_univ=t_univ, edges=edges, w=w, zeta=zeta, W=W)


def point_lines(L: Library, th, cols, W):
    """Step 3: line luminosities [erg/s per Msun of the weights] and Lhat [n_line, n_neb]."""
    if L.lines is None:
        return np.zeros(0), None
    ages = L.ages[L.neb_a0:L.n_neb]
    lhat = nebular.line_table_at_ages(L.lines["line_table"], L.lines["zg_nodes"], L.lines["line_tau"],
                                      L.lines["u_nodes"], th[cols["gas_logz"]], th[cols["gas_logu"]], ages)
    return nebular.line_luminosity(W, L.Q, lhat, L.n_neb, L.neb_a0), lhat


def point_continuum(L: Library, th, cols, W):
    """Step 3, continuum: the nebular continuum [Lsun/A per Msun of the weights] or 0."""
    if L.cont is None:
        return 0.0
    c = L.cont
    sel = np.zeros(len(L.ages), dtype=bool)
    sel[L.neb_a0:L.n_neb] = True
    chat = nebular.continuum_at_ages(c["cont_table"], c["zg_nodes"], c["tau_nodes"], c["u_nodes"],
                                     th[cols["gas_logz"]], th[cols["gas_logu"]], L.ages[sel])
    return nebular.continuum_luminosity(W, L.Q, chat, sel, L.wave)


def escape_fraction(L: Library, th, cols):
    """f_ob = theta[frac_obrun] clamped to [0, 1], or 0 without an escape geometry."""
    if L.escape == "none":
        return 0.0
    return min(max(float(th[cols["frac_obrun"]]), 0.0), 1.0)


def young_factors(L: Library, f):
    """(p, q, s): the young light crosses the birth cloud with transmission
    p e^{-tau_BC} + q and the nebular emission is scaled by s (Sec. 2.3.2, App. C, D.1):
    no geometry (1, 0, 1); runaway_bc (1 - f, f, 1 - f), the runaway mixture on the young
    array whose nebular part carries the covered fraction; picket (1 - f, 0, 1), only the
    covered fraction (1 - f) of the young light, nebular emission included, is attenuated."""
    if L.escape == "runaway_bc":
        return 1.0 - f, f, 1.0 - f
    if L.escape == "picket":
        return 1.0 - f, 0.0, 1.0
    return 1.0, 0.0, 1.0


def rest_frame(L: Library, theta, lines_on_grid=True):
    """Steps 1-5 for the whole batch: W, lines, Y, O and attenuated F [B, n_wave]."""
    theta = np.atleast_2d(theta)
    B = theta.shape[0]
    cols = lib_columns(L)
    n_k = L.flux.shape[0] * L.flux.shape[1] * L.flux.shape[2]
    Wk = np.zeros((B, n_k))
    per = []
    Lline = np.zeros((B, 0 if L.lines is None else len(L.lines["line_wave"])))
    neb = np.zeros((B, len(L.wave)))
    for b in range(B):
        p = point_weights(L, theta[b], cols)
        Wk[b] = p["W"].reshape(-1)
        Lline[b], p["lhat"] = point_lines(L, theta[b], cols, p["W"])
        neb[b] = point_continuum(L, theta[b], cols, p["W"])
        per.append(p)
    young_k = np.broadcast_to(L.young, L.flux.shape[:3]).reshape(-1)
    f = L.flux.reshape(n_k, -1)
    Y = Wk[:, young_k] @ f[young_k]
    O = Wk[:, ~young_k] @ f[~young_k]
    I = np.zeros_like(Y) if L.flux_ion is None else Wk @ L.flux_ion.reshape(n_k, -1)
    lines_grid = np.zeros_like(Y)
    if L.lines is not None and lines_on_grid:
        lines_grid = (Lline / LSUN) @ L.G
    wave = L.wave
    F = np.empty_like(Y)
    Yn = np.empty_like(Y)
    fob = np.zeros(B)
    for b in range(B):
        th = theta[b]
        fob[b] = escape_fraction(L, th, cols)
        pf, qf, sf = young_factors(L, fob[b])
        # young light after the escape geometry's scaling of the nebular part
        Yb = Yn[b] = Y[b] + sf * (neb[b] + lines_grid[b])
        T_bc = np.exp(-dust.birth_cloud_tau(wave, th[cols["tau_bc"]], th[cols["alpha_bc"]]))
        T_d = np.exp(-dust.diffuse_tau(wave, th[cols["tau_diff"]], th[cols["delta"]], L.dust_a, L.dust_d))
        if L.escape == "picket":
            # the fraction f_ob of the young stars, ionising continuum included, sees no dust
            F[b] = T_d * ((pf * T_bc + qf) * Yb + O[b]) + fob[b] * (Y[b] + I[b])
        else:
            # the restored ionising continuum bypasses the birth cloud, then the screen
            F[b] = T_d * ((pf * T_bc + qf) * Yb + fob[b] * I[b] + O[b])
    # Y: the young light before the birth cloud (stars, then the scaled nebular emission);
    # Ystar: its stellar part alone
    return dict(per=per, W=Wk, Lline=Lline, Y=Yn, Ystar=Y, O=O, I=I, neb=neb, F=F, cols=cols, fob=fob)


def observer_scale(L: Library, th, cols):
    """10^logmass * (1+z) / (4 pi D_L^2) [cm^-2] and D_L [cm]."""
    z = th[cols["zred"]]
    dl = float(cosmology.luminosity_distance_cm(z, L.H0, L.Om))
    return 10.0 ** th[cols["logmass"]] * (1.0 + z) / (4.0 * math.pi * dl * dl), dl


def fnu_observed(L: Library, F_row, scale):
    """F_nu^obs on the rest grid: scale * Lsun F_lambda[per cm] lambda^2 / c (Sec. 2.6)."""
    return scale * LSUN * F_row * L.wave ** 2 * ANG_CM / C_CMS


def line_fluxes(L: Library, th, cols, Lline, dl):
    """F_l = s L_l (p T_BC + q)(lambda_l) T_d(lambda_l) 10^logmass / (4 pi D_L^2) (App. I.1),
    with the escape geometry's (p, q, s) (young_factors; (1, 0, 1) without one)."""
    lw = L.lines["line_wave"]
    a = np.interp(lw, L.wave, L.dust_a)
    d = np.interp(lw, L.wave, L.dust_d)
    pf, qf, sf = young_factors(L, escape_fraction(L, th, cols))
    T_bc = np.exp(-dust.birth_cloud_tau(lw, th[cols["tau_bc"]], th[cols["alpha_bc"]]))
    T_d = np.exp(-dust.diffuse_tau(lw, th[cols["tau_diff"]], th[cols["delta"]], a, d))
    F = sf * Lline * (pf * T_bc + qf) * T_d * 10.0 ** th[cols["logmass"]] / (4.0 * math.pi * dl * dl)
    return F * igm_transmission(L, th, cols, (1.0 + th[cols["zred"]]) * lw)


def igm_transmission(L: Library, th, cols, lam_obs):
    """IGM transmission at observed wavelengths (1 without IGM): Madau (1995) with the
    optical depth scaled by theta[igm_factor], plus the damping wing of theta[x_HI] and the
    absorber of theta[logN_HI] at theta[z_dla] where the library has them (Sec. 2.6)."""
    if not L.igm:
        return np.ones_like(np.asarray(lam_obs, dtype=np.float64))
    return igm.transmission(lam_obs, th[cols["zred"]], th[cols["igm_factor"]],
                            x_hi=th[cols["x_hi"]] if L.igm & IGM_DAMPING else None,
                            log_nhi=th[cols["log_nhi"]] if L.igm & IGM_DLA else None,
                            z_dla=th[cols["z_dla"]] if L.igm & IGM_DLA else None)


def predict(L: Library, obs, theta, rf=None, trunc=5.0):
    """Model observables [B, n] (maggies) for photometry or a spectrum."""
    theta = np.atleast_2d(theta)
    spec = obs.kind == "spec"
    if obs.kind == "lines":
        # the line fluxes of App. I.1 summed over each entry's blend; no continuum
        if rf is None:
            rf = rest_frame(L, theta, lines_on_grid=False)
        cols = rf["cols"]
        out = []
        for b in range(theta.shape[0]):
            _, dl = observer_scale(L, theta[b], cols)
            Fl = line_fluxes(L, theta[b], cols, rf["Lline"][b], dl)
            out.append([float(np.sum(Fl[list(bl)])) for bl in obs.blends])
        return np.array(out)
    if rf is None:
        rf = rest_frame(L, theta, lines_on_grid=not spec)
    cols = rf["cols"]
    out = []
    if spec:
        sig_k = projection.kernel_sigma_kms(obs.pix_wave, obs.lsf_mode, obs.lsf_value, L.wave,
                                            obs.z_ref, obs.sigma_gal_kms)
    vd = fourier_stage_plan(L, obs, sig_k if spec else None)
    for b in range(theta.shape[0]):
        th = theta[b]
        scale, dl = observer_scale(L, th, cols)
        z = th[cols["zred"]]
        # observer frame: mass and flux factor (Sec. 2.6), then the free velocity dispersion
        # on the continuum (Sec. 2.5, App. F), then the IGM transmission at lambda (1 + z),
        # on the rest grid (the data-flow figure of App. A puts the IGM after sigma_gal and
        # before the instrument's kernel)
        fnu = fnu_observed(L, rf["F"][b], scale)
        if vd is not None:
            fnu = fourier_stage(L, vd, fnu, z, th[cols["sigma_gal"]])
        fnu = fnu * igm_transmission(L, th, cols, L.wave * (1.0 + z))
        if not spec:
            out.append(projection.band_maggies(L.wave, fnu, z, obs.filters))
            continue
        cont = projection.spectrum_continuum(obs.pix_wave, sig_k, L.wave, fnu, z, trunc)
        if L.lines is not None:
            Fl, lobs, s_l = spectrum_line_terms(L, obs, th, cols, rf["Lline"][b], dl)
            cont = cont + projection.line_profile_pixels(obs.pix_wave, Fl, lobs, s_l)
        out.append(cont / FNU_AB)
    return np.array(out)


def spectrum_line_terms(L: Library, obs, th, cols, Lline_row, dl):
    """Per library line: observer-frame flux F_l (App. I.1), observed wavelength and the
    profile width s_l in ln(lambda) (eq. app_line_profile)."""
    Fl = line_fluxes(L, th, cols, Lline_row, dl)
    lobs = (1.0 + th[cols["zred"]]) * L.lines["line_wave"]
    s_l = np.sqrt(obs.sigma_gas_kms ** 2
                  + projection.sigma_inst_kms(lobs, obs.lsf_mode, _lsf_at(obs, lobs)) ** 2) / C_KMS
    return Fl, lobs, s_l


def line_marg_terms(L: Library, obs, th, cols, Lline_row):
    """The lines fitted by the marginalisation of a spectrum (App. I.3) at one point: those
    whose observed wavelength lies within the pixel range, less the Gaussian-prior lines
    with no grid flux (fixed at zero); their unit-flux profiles on the pixels (maggies per
    erg/s/cm^2), grid fluxes, prior widths frac * F_l and flat flags."""
    _, dl = observer_scale(L, th, cols)
    Fl, lobs, s_l = spectrum_line_terms(L, obs, th, cols, Lline_row, dl)
    n_l = len(Fl)
    flat_all = obs.line_marg == "flat"
    flat = np.ones(n_l, dtype=bool) if flat_all else (
        np.zeros(n_l, dtype=bool) if obs.line_flat is None else np.asarray(obs.line_flat, dtype=bool))
    inwin = (lobs >= obs.pix_wave[0]) & (lobs <= obs.pix_wave[-1])
    sel = np.flatnonzero(inwin & (flat | (Fl > 0.0)))
    A = np.stack([projection.line_profile_pixels(obs.pix_wave, np.array([1.0]), lobs[[j]], s_l[[j]]) / FNU_AB
                  for j in sel], axis=1) if len(sel) else np.zeros((len(obs.pix_wave), 0))
    return dict(idx=sel, A=A, alpha_bar=Fl[sel], prior_sd=obs.line_prior_frac * Fl[sel], flat=flat[sel])


def joint_line_terms(L: Library, spec, cat, th, cols, Lline_row):
    """The lines fitted jointly by a spectrum (with its line_marg settings) and a line
    catalogue of the same object (Sec. 4.1, App. I.3): the spectrum's lines (observed
    wavelength within its pixel range) and the lines of the catalogue's detected, included
    entries, less the Gaussian-prior lines with no grid flux; their unit-flux profiles on
    the spectrum's pixels (zero where a line's profile misses them), the 0/1 blend matrix of
    every catalogue entry, grid fluxes, prior widths and flat flags."""
    _, dl = observer_scale(L, th, cols)
    Fl, lobs, s_l = spectrum_line_terms(L, spec, th, cols, Lline_row, dl)
    n_l = len(Fl)
    flat = np.ones(n_l, dtype=bool) if spec.line_marg == "flat" else (
        np.zeros(n_l, dtype=bool) if spec.line_flat is None else np.asarray(spec.line_flat, dtype=bool))
    inwin = (lobs >= spec.pix_wave[0]) & (lobs <= spec.pix_wave[-1])
    mask = likelihood.inclusion_mask(cat.data, cat.sigma, cat.mask)
    up = np.zeros(len(cat.blends), dtype=bool) if cat.upper is None else np.asarray(cat.upper, dtype=bool)
    in_cat = np.zeros(n_l, dtype=bool)
    for e, bl in enumerate(cat.blends):
        if mask[e] and not up[e]:
            in_cat[list(bl)] = True
    sel = np.flatnonzero((inwin | in_cat) & (flat | (Fl > 0.0)))
    A = np.stack([projection.line_profile_pixels(spec.pix_wave, np.array([1.0]), lobs[[j]], s_l[[j]]) / FNU_AB
                  for j in sel], axis=1) if len(sel) else np.zeros((len(spec.pix_wave), 0))
    Ac = np.array([[1.0 if j in set(bl) else 0.0 for j in sel] for bl in cat.blends]).reshape(len(cat.blends), len(sel))
    return dict(idx=sel, A=A, Ac=Ac, alpha_bar=Fl[sel], prior_sd=spec.line_prior_frac * Fl[sel], flat=flat[sel])


def line_band_response(L: Library, phot, th, cols, Lline_row, idx):
    """A[b, j]: the photometric model of library line idx[j] alone (its profile on the model
    grid through the birth cloud with the escape geometry's factors, the diffuse screen,
    the observer frame, the IGM and the filters: eq. E1), per unit of its observed flux
    F_l (App. I.1), so that a fitted flux alpha_j adds A[b, j] alpha_j to band b."""
    scale, dl = observer_scale(L, th, cols)
    z = th[cols["zred"]]
    wave = L.wave
    pf, qf, sf = young_factors(L, escape_fraction(L, th, cols))
    T_bc = np.exp(-dust.birth_cloud_tau(wave, th[cols["tau_bc"]], th[cols["alpha_bc"]]))
    T_d = np.exp(-dust.diffuse_tau(wave, th[cols["tau_diff"]], th[cols["delta"]], L.dust_a, L.dust_d))
    igm_t = igm_transmission(L, th, cols, wave * (1.0 + z))
    Fl = line_fluxes(L, th, cols, Lline_row, dl)
    A = np.zeros((len(phot.filters), len(idx)))
    for c, l in enumerate(idx):
        F_rest = T_d * (pf * T_bc + qf) * sf * (Lline_row[l] / LSUN) * L.G[l]
        fnu = fnu_observed(L, F_rest, scale) * igm_t
        A[:, c] = projection.band_maggies(wave, fnu, z, phot.filters) / Fl[l]
    return A


def logl_lines_joint(L: Library, spec, cat, theta, phot=None):
    """logL[B] of a spectrum, a line catalogue (or None) and a photometric observation (or
    None) of one object with the line fluxes marginalised jointly (eq. app_line_marg summed
    over the observations).  The fitted lines are the spectrum's and the catalogue's
    detections' (joint_line_terms); the photometry sees every line on the model grid, the
    fitted ones through line_band_response, the others at their grid fluxes.  Reading: a
    free sigma_gal (which broadens the photometric lines) is not combined with it."""
    theta = np.atleast_2d(theta)
    cols = lib_columns(L)
    if phot is not None and L.sigma_gal_max > 0.0:
        raise ValueError("joint marginalisation with photometry and a free sigma_gal is not supported")
    ms = predict(L, spec, theta)
    cat_in = cat if cat is not None else Lines(blends=[], data=np.zeros(0), sigma=np.zeros(0))
    mc = predict(L, cat, theta) if cat is not None else np.zeros((theta.shape[0], 0))
    mp = predict(L, phot, theta) if phot is not None else None
    rf = rest_frame(L, theta, lines_on_grid=False)
    mask_s = likelihood.inclusion_mask(spec.data, spec.sigma, spec.mask)
    mask_c = likelihood.inclusion_mask(cat_in.data, cat_in.sigma, cat_in.mask)
    up = np.zeros(len(cat_in.blends), dtype=bool) if cat_in.upper is None else np.asarray(cat_in.upper, dtype=bool)
    mask_p = likelihood.inclusion_mask(phot.data, phot.sigma, phot.mask) if phot is not None else None
    out = np.empty(theta.shape[0])
    for b in range(theta.shape[0]):
        s, fc, fd, j = noise_terms(spec, theta[b], cols)
        t = joint_line_terms(L, spec, cat_in, theta[b], cols, rf["Lline"][b])
        pdict = None
        if phot is not None:
            sp_, fcp, fdp, jp = noise_terms(phot, theta[b], cols)
            pdict = dict(data=phot.data, model=mp[b], sigma=phot.sigma, mask=mask_p,
                         A=line_band_response(L, phot, theta[b], cols, rf["Lline"][b], t["idx"]),
                         s=sp_, f_calib=fcp, f_data=fdp, jitter=jp)
        out[b] = likelihood.joint_line_marginal_lnlike(
            dict(data=spec.data, model=ms[b], sigma=spec.sigma, mask=mask_s, A=t["A"], s=s, f_calib=fc, f_data=fd,
                 jitter=j),
            dict(data=cat_in.data, model=mc[b], sigma=cat_in.sigma, mask=mask_c, upper=up, A=t["Ac"]),
            t["alpha_bar"], t["prior_sd"], t["flat"], phot=pdict)
    return out


def fourier_stage_plan(L: Library, obs, sig_k=None):
    """Window rule and transform length of an observation's Fourier stage (Sec. 2.5,
    App. F): the observed range it covers (the pixels, or every filter node) and the
    margin M in nodes; None without a free sigma_gal."""
    if L.sigma_gal_max <= 0.0:
        return None
    dlnl = kinematics.log_step(L.wave)
    mg = kinematics.margin_nodes(L.sigma_gal_max, dlnl)
    if obs.kind == "spec":
        lo, hi = float(obs.pix_wave[0]), float(obs.pix_wave[-1])
        M = kinematics.margin_nodes(np.max(sig_k), dlnl) + mg + 2
    else:
        lo = min(float(np.min(f[0])) for f in obs.filters)
        hi = max(float(np.max(f[0])) for f in obs.filters)
        M = mg + 2
    return dict(lo=lo, hi=hi, M=M, dlnl=dlnl, n_fft=kinematics.fft_length(lo, hi, dlnl, M, L.sigma_gal_max))


def fourier_stage(L: Library, vd, fnu, z, sigma):
    """The continuum on the rest grid with its window broadened by sigma [km/s]; NaN
    everywhere for sigma outside [0, sigma_gal_max]."""
    if not (0.0 <= sigma <= L.sigma_gal_max):
        return np.full_like(fnu, np.nan)
    j0, j1 = kinematics.window(L.wave, vd["lo"], vd["hi"], z, vd["M"])
    out = fnu.copy()
    out[j0:j1] = kinematics.fourier_broaden(fnu[j0:j1], vd["n_fft"], sigma, vd["dlnl"])
    return out


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
    cols = lib_columns(L)
    mask = likelihood.inclusion_mask(obs.data, obs.sigma, obs.mask)
    if obs.kind == "lines":
        up = np.zeros(len(obs.blends), dtype=bool) if obs.upper is None else np.asarray(obs.upper, dtype=bool)
        return np.array([likelihood.lines_lnlike(obs.data, model[b], obs.sigma, mask, up)
                         for b in range(theta.shape[0])])
    calib = getattr(obs, "calib", None)
    A = likelihood.chebyshev_design(obs.pix_wave, obs.calib_order) if calib else None
    lmarg = getattr(obs, "line_marg", None)
    if lmarg is not None:
        if calib:
            raise ValueError("line marginalisation and a calibration polynomial together are not supported")
        rf = rest_frame(L, theta, lines_on_grid=False)
    out = np.empty(theta.shape[0])
    for b in range(theta.shape[0]):
        s, fc, fd, j = noise_terms(obs, theta[b], cols)
        if lmarg is not None:
            t = line_marg_terms(L, obs, theta[b], cols, rf["Lline"][b])
            out[b] = likelihood.line_marginal_lnlike(obs.data, model[b], obs.sigma, mask, t["A"], t["alpha_bar"],
                                                     t["prior_sd"], t["flat"], s, fc, fd, j)
        elif calib:
            out[b] = likelihood.calibrated_lnlike(obs.data, model[b], obs.sigma, mask, A, obs.calib_prior, calib,
                                                  s, fc, fd, j)
        else:
            out[b] = likelihood.lnlike(obs.data, model[b], obs.sigma, mask, s, fc, fd, j)
    return out
