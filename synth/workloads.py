"""Seeded synthetic workloads for the batched stellar-population forward model.

Every array here is drawn from ``numpy.random.default_rng(seed)``; nothing in this
module evaluates the forward model.  The shapes follow the paper's workloads:
SSP grids of ~100 ages x ~20 metallicities x ~6000 wavelengths (Sec. 2.1), SFHs
of up to ~120 lookback bins (Sec. 5.3), 8-25 photometric bands and prism-like
spectra of a few thousand pixels (Sec. 5.5, 6.1), 64-1024 live points per batch
(Sec. 4.3, 7).  The real FSPS/BPASS grids, sedpy filter curves, Byler et al.
photoionisation tables and JADES catalogues are not available, so these
generators stand in for them.

Units: ages in yr, wavelengths in Angstrom, SSP spectra in Lsun/A per Msun
formed, line tables in log10(L_line/Q) with L in erg/s and Q in photons/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Parameter-vector layout.  theta[B, P] is float64, row-major.  The scalar
# columns come first, then the SFH bin masses, then the enrichment-history nodes.
# The C library reports the same layout through sps_theta_layout().
# ----------------------------------------------------------------------------
THETA_SCALARS = (
    "logmass",        # log10 of the total formed stellar mass (Sec. 2.6)
    "zred",           # redshift
    "tau_bc",         # birth-cloud optical depth at 5500 A (Sec. 2.4)
    "alpha_bc",       # birth-cloud power-law slope
    "tau_diff",       # diffuse optical depth (Kriek & Conroy form)
    "delta",          # diffuse slope offset delta_dust
    "logzsol",        # constant-metallicity mode: log10(Z/Zsun)
    "gas_logz",       # nebular gas-phase metallicity
    "gas_logu",       # nebular ionisation parameter
    "afe",            # [alpha/Fe] for libraries with an alpha axis
    "log_err_scale",  # ln s   (noise floor, App. G)
    "log_f_calib",    # ln f_calib
    "log_f_data",     # ln f_data
    "log_jitter",     # ln j
)
N_SCALARS = len(THETA_SCALARS)


def theta_columns(n_sfh: int, n_zh: int, escape: bool = False, igm: int = 0, vdisp: bool = False) -> dict:
    """Column offsets of the theta layout (scalars, then sfh[n_sfh], then zh[n_zh], then,
    for a library with an ionising-photon escape geometry, frac_obrun, then, with IGM
    transmission (igm: bit mask, 1 Madau, 2 damping wing, 4 damped absorber), igm_factor,
    x_HI, logN_HI and z_dla as present, then, with a free stellar velocity dispersion,
    sigma_gal)."""
    cols = {name: i for i, name in enumerate(THETA_SCALARS)}
    cols["sfh"] = N_SCALARS
    cols["zh"] = N_SCALARS + n_sfh
    cols["P"] = N_SCALARS + n_sfh + n_zh
    if escape:
        cols["frac_obrun"] = cols["P"]
        cols["P"] += 1
    igm = int(igm)
    if igm & 1:
        cols["igm_factor"] = cols["P"]
        cols["P"] += 1
    if igm & 2:
        cols["x_hi"] = cols["P"]
        cols["P"] += 1
    if igm & 4:
        cols["log_nhi"] = cols["P"]
        cols["z_dla"] = cols["P"] + 1
        cols["P"] += 2
    if vdisp:
        cols["sigma_gal"] = cols["P"]
        cols["P"] += 1
    return cols


# ----------------------------------------------------------------------------
# Workload configurations
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Config:
    name: str
    n_age: int
    logz: tuple
    afe: tuple
    n_wave: int
    n_sfh: int
    T1: float            # first non-zero SFH edge (yr)
    n_zh: int            # 0 = constant-metallicity mode
    batch: int
    filters: str         # "tophat8" | "gauss20" | "none"
    n_lines: int
    dust: str            # "powerlaw" (single screen) | "kc13"
    z_range: tuple
    spectrum: bool = False
    n_pix: int = 0
    t_young: float = 1e7
    lam_min: float = 100.0
    lam_max: float = 5e4
    age_min: float = 1e6
    age_max: float = 1.3e10
    cosmo: tuple = (70.0, 0.3)
    sample_alpha_bc: bool = False
    extra: dict = field(default_factory=dict)


def _logz_grid(n, lo, hi):
    return tuple(float(x) for x in np.linspace(lo, hi, n))


CONFIGS = {
    # tiny FP64 parity case
    "c0": Config("c0", n_age=20, logz=(-2.0, -1.0, 0.0), afe=(0.0,), n_wave=1000,
                 n_sfh=10, T1=1e7, n_zh=0, batch=64, filters="tophat8", n_lines=0,
                 dust="powerlaw", z_range=(1.0, 8.0)),
    # full-size FP32 batch: time-varying enrichment, two-component dust, 128 lines
    "c1": Config("c1", n_age=107, logz=_logz_grid(22, -2.5, 0.5), afe=(0.0,), n_wave=5994,
                 n_sfh=120, T1=3e6, n_zh=24, batch=1024, filters="gauss20", n_lines=128,
                 dust="kc13", z_range=(0.5, 12.0)),
    # precision variant of c1 (same inputs; the library is stored in 16 bit)
    "c2": Config("c2", n_age=107, logz=_logz_grid(22, -2.5, 0.5), afe=(0.0,), n_wave=5994,
                 n_sfh=120, T1=3e6, n_zh=24, batch=1024, filters="gauss20", n_lines=128,
                 dust="kc13", z_range=(0.5, 12.0)),
    # spectroscopic gradient variant of c1: 3000-pixel R~100 prism-like spectrum
    "c3": Config("c3", n_age=107, logz=_logz_grid(22, -2.5, 0.5), afe=(0.0,), n_wave=5994,
                 n_sfh=120, T1=3e6, n_zh=24, batch=1024, filters="none", n_lines=128,
                 dust="kc13", z_range=(0.5, 12.0), spectrum=True, n_pix=3000,
                 sample_alpha_bc=True),
    # serving: alpha-enhanced library, constant metallicity, nebular emission off
    "c4": Config("c4", n_age=107, logz=_logz_grid(22, -2.5, 0.5), afe=(0.0, 0.2, 0.4),
                 n_wave=5994, n_sfh=120, T1=3e6, n_zh=0, batch=1024, filters="gauss20",
                 n_lines=0, dust="kc13", z_range=(0.5, 12.0)),
}


def reduced(cfg: Config, **kw) -> Config:
    """A copy of ``cfg`` with some fields replaced (small parity cases)."""
    d = dict(cfg.__dict__)
    d.update(kw)
    return Config(**d)


# ----------------------------------------------------------------------------
# SSP library: sum of three peak-normalised Planck curves per (age, Z, afe)
# ----------------------------------------------------------------------------
_HC_OVER_K_AK = 1.438776877e8   # h c / k_B in Angstrom * Kelvin (data generation only)
_WIEN_X = 4.965114231744276    # root of x = 5 (1 - e^-x): peak of x^5/(e^x - 1)


def _planck_shape(wave, T):
    """Planck B_lambda(T) shape normalised to a peak value of 1."""
    x = _HC_OVER_K_AK / (wave[None, :] * T[:, None])
    with np.errstate(over="ignore", under="ignore"):
        em = np.exp(-np.minimum(x, 700.0))
        val = x ** 5 * em / (-np.expm1(-x))
    peak = _WIEN_X ** 5 * math.exp(-_WIEN_X) / (-math.expm1(-_WIEN_X))
    return val / peak


def make_library(cfg: Config, seed: int = 0, noise: float = 0.1) -> dict:
    """SSP grid flux[n_afe, n_z, n_age, n_wave] in Lsun/A/Msun on a log-uniform grid.

    ``noise`` is the dispersion of the iid lognormal factor per element (0.1 for the
    workloads; 0 gives smooth spectra for finite-difference tests).
    """
    rng = np.random.default_rng(seed)
    ages = np.geomspace(cfg.age_min, cfg.age_max, cfg.n_age)
    wave = np.geomspace(cfg.lam_min, cfg.lam_max, cfg.n_wave)
    logz = np.asarray(cfg.logz, dtype=np.float64)
    afe = np.asarray(cfg.afe, dtype=np.float64)
    tm = ages / 1e6
    flux = np.empty((len(afe), len(logz), cfg.n_age, cfg.n_wave))
    for ia, al in enumerate(afe):
        for iz, lz in enumerate(logz):
            tfac = (1.0 - 0.05 * lz) * (1.0 + 0.03 * al)
            T1 = 4e4 * tm ** -0.3 * tfac
            T2 = 7e3 * tm ** -0.05 * tfac
            T3 = np.full_like(tm, 3.5e3) * tfac
            A1 = tm ** -1.0
            A2 = tm ** -0.5 * (1.0 - 0.2 * al)
            A3 = 0.1 * tm ** -0.2
            flux[ia, iz] = (A1[:, None] * _planck_shape(wave, T1)
                            + A2[:, None] * _planck_shape(wave, T2)
                            + A3[:, None] * _planck_shape(wave, T3))
    flux *= np.exp(rng.normal(0.0, noise, size=flux.shape))
    flux *= 1e2 / flux.max()
    np.maximum(flux, 1e-8, out=flux)
    return dict(ages=ages, logz=logz, afe=afe, wave=wave, flux=flux, t_young=cfg.t_young)


def make_lines(cfg: Config, lib: dict, seed: int = 1, line_tau=None) -> dict | None:
    """Synthetic photoionisation line table log10(L_line/Q) [n_line, n_tau, n_zg, n_u].

    Without ``line_tau`` the table's age axis is the set of SSP ages younger than
    ``t_young``; with it, the table is on those ages (yr) and carries them as
    ``line_tau`` (a grid of its own, as the photoionisation grids have).
    """
    if cfg.n_lines == 0:
        return None
    rng = np.random.default_rng(seed)
    if line_tau is None:
        n_tau = int(np.sum(lib["ages"] < cfg.t_young))
        an = np.arange(n_tau) / max(n_tau - 1, 1)
    else:
        line_tau = np.asarray(line_tau, dtype=np.float64)
        n_tau = len(line_tau)
        an = (line_tau - line_tau[0]) / (line_tau[-1] - line_tau[0])
    line_wave = np.sort(np.exp(rng.uniform(np.log(1000.0), np.log(2e4), cfg.n_lines)))
    zg = np.linspace(-1.3, 0.3, 7)
    lu = np.linspace(-4.0, -1.0, 7)
    base = rng.uniform(-14.0, -11.5, cfg.n_lines)
    sz = rng.uniform(-0.6, 0.6, cfg.n_lines)
    su = rng.uniform(-0.8, 0.8, cfg.n_lines)
    sa = rng.uniform(-1.0, 0.0, cfg.n_lines)
    zn = (zg - zg.mean()) / np.ptp(zg)
    un = (lu - lu.mean()) / np.ptp(lu)
    table = (base[:, None, None, None]
             + sa[:, None, None, None] * an[None, :, None, None]
             + sz[:, None, None, None] * zn[None, None, :, None]
             + su[:, None, None, None] * un[None, None, None, :]
             + 0.3 * (zn[None, None, :, None] * un[None, None, None, :])
             + rng.normal(0.0, 0.05, size=(cfg.n_lines, n_tau, len(zg), len(lu))))
    out = dict(line_wave=line_wave, line_table=table, zg_nodes=zg, u_nodes=lu)
    if line_tau is not None:
        out["line_tau"] = line_tau
    return out


CONT_TAU = (5e5, 1e6, 2e6, 3e6, 5e6, 7e6, 1e7)   # yr: ages of the continuum cube
LINE_TAU = (5e5, 1e6, 2e6, 3e6, 4e6, 6e6, 1e7)   # yr: ages of a line cube with its own axis


def make_nebular_continuum(wave: np.ndarray, seed: int = 3, tau_nodes=CONT_TAU) -> dict:
    """Synthetic nebular continuum cube log10(L_nu/Q) [n_tau, n_zg, n_u, n_wave] on the
    library wavelengths (L_nu in erg/s/Hz, Q in photons/s), standing in for the
    photoionisation grids (App. C).  Its axes differ from the line table's.

    Shape: a smooth level with Balmer (3646 A) and Paschen (8204 A) jumps, nothing
    below the Lyman limit (-38), linear trends and a cross term in the normalised
    (Z_gas, age, log U) coordinates and 0.03 dex of iid scatter.  The level, -25.2 at
    5000 A, makes the continuum a sizeable fraction (tens of per cent) of the young
    stellar light of ``make_library``'s spectra at optical wavelengths.
    """
    rng = np.random.default_rng(seed)
    tau = np.asarray(tau_nodes, dtype=np.float64)
    zg = np.linspace(-2.0, 0.4, 5)
    lu = np.linspace(-4.0, -1.0, 4)
    lw = np.log10(np.asarray(wave, dtype=np.float64) / 5000.0)
    c0 = -25.2 - 0.2 * lw ** 2 + 0.35 * (wave < 3646.0) + 0.15 * (wave < 8204.0)
    c0 = np.where(wave < 912.0, -38.0, c0)
    tn = (tau - tau[0]) / (tau[-1] - tau[0])
    zn = (zg - zg.mean()) / np.ptp(zg)
    un = (lu - lu.mean()) / np.ptp(lu)
    cube = (c0[None, None, None, :]
            - 0.3 * tn[:, None, None, None]
            + 0.25 * zn[None, :, None, None]
            - 0.15 * un[None, None, :, None]
            + 0.2 * (zn[None, :, None, None] * un[None, None, :, None])
            + rng.normal(0.0, 0.03, size=(len(tau), len(zg), len(lu), len(wave))))
    return dict(cont_table=cube, tau_nodes=tau, zg_nodes=zg, u_nodes=lu)


def make_dust_tables(cfg: Config, wave: np.ndarray) -> dict:
    """Static attenuation-curve tables a(lambda), d(lambda) on the library grid.

    ``powerlaw``: a = (lambda/5500)^-0.7, d = 0 (single power-law screen).
    ``kc13``: a = (lambda/5500)^-0.7 and d = a Drude profile at 2175 A, FWHM 350 A.
    """
    a = (wave / 5500.0) ** -0.7
    if cfg.dust == "powerlaw":
        d = np.zeros_like(wave)
    else:
        l0, dl = 2175.0, 350.0
        d = (wave * dl) ** 2 / ((wave ** 2 - l0 ** 2) ** 2 + (wave * dl) ** 2)
    return dict(dust_a=a, dust_d=d)


# ----------------------------------------------------------------------------
# Filters and spectral pixel grids
# ----------------------------------------------------------------------------
_FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


def _gauss_filter(centre, lam_over_fwhm, n=128):
    sig = centre / lam_over_fwhm / _FWHM_PER_SIGMA
    lam = np.linspace(centre - 3 * sig, centre + 3 * sig, n)
    R = np.exp(-0.5 * ((lam - centre) / sig) ** 2)
    R[0] = R[-1] = 0.0
    return lam, R


def make_filters(kind: str, n_band: int | None = None) -> list:
    """List of (lambda_nodes [A], transmission) pairs; every curve has zero end nodes."""
    out = []
    if kind == "tophat8":
        edges = np.geomspace(9000.0, 44000.0, 9)
        for i in range(8):
            lam = np.linspace(edges[i], edges[i + 1], 64)
            R = np.ones(64)
            R[0] = R[-1] = 0.0
            out.append((lam, R))
    elif kind == "gauss20":
        cen = np.geomspace(7000.0, 48000.0, 16)
        for i, c in enumerate(cen):
            out.append(_gauss_filter(c, 4.0 if i % 2 == 0 else 10.0))
        for c in (52000.0, 56000.0, 61000.0, 66000.0):
            out.append(_gauss_filter(c, 10.0))
    elif kind == "gaussN":
        cen = np.geomspace(7000.0, 66000.0, n_band)
        for i, c in enumerate(cen):
            r = 10.0 if (c > 48000.0 or i % 2 == 1) else 4.0
            out.append(_gauss_filter(c, r))
    elif kind == "none":
        pass
    else:
        raise ValueError(kind)
    return out


def make_spectrum_grid(n_pix: int, lam_lo=6000.0, lam_hi=53000.0) -> dict:
    """Prism-like pixel grid, log-uniform in wavelength, with a constant R_fwhm=100 LSF."""
    return dict(pix_wave=np.geomspace(lam_lo, lam_hi, n_pix), lsf_mode="R_fwhm",
                lsf_value=100.0, sigma_gas_kms=100.0, sigma_gal_kms=0.0)


# ----------------------------------------------------------------------------
# Parameter batches
# ----------------------------------------------------------------------------
def _trunc_normal(rng, mu, sd, lo, hi, size):
    out = rng.normal(mu, sd, size)
    bad = (out < lo) | (out > hi)
    while bad.any():
        out[bad] = rng.normal(mu, sd, int(bad.sum()))
        bad = (out < lo) | (out > hi)
    return out


def _clipped_t(rng, nu, scale, clip, size):
    return np.clip(rng.standard_t(nu, size) * scale, -clip, clip)


def make_theta(cfg: Config, B: int | None = None, seed: int = 2, escape: bool = False, igm: bool = False,
               sfh_scheme: str = "step", vdisp: float = 0.0) -> np.ndarray:
    """Draw theta[B, P] from the configuration's priors.

    SFH: c0 uses Dirichlet(1,...,1) bin masses; the others draw clipped Student-t
    (nu=2, sigma=0.3, |d|<=1) log10 ratios between adjacent bins and normalise to
    one solar mass (the continuity-prior shape of Sec. 4.2, applied to masses).
    Enrichment history: zeta_0 ~ U(-2.2, 0.3) plus a clipped Student-t random
    walk with sigma 0.2, clamped to the grid.  With ``escape``, a column frac_obrun ~
    U(0, 1) and with ``igm`` a column igm_factor ~ U(0.5, 1.5) (with the damping wing x_HI ~
    U(0, 1); with the damped absorber logN_HI ~ U(20, 22) and z_dla = z - U(0, 0.5),
    floored at 0), each from a stream of its own (the other columns are unchanged); with
    ``vdisp`` > 0 a column sigma_gal ~
    U(0, vdisp) km/s.  Under the linear SFH scheme the SFH values are node SFRs: the bin
    masses divided by 1e10 / n_sfh years.
    """
    B = cfg.batch if B is None else B
    rng = np.random.default_rng(seed)
    cols = theta_columns(cfg.n_sfh, cfg.n_zh, escape, igm, vdisp > 0.0)
    th = np.zeros((B, cols["P"]))
    if vdisp > 0.0:
        th[:, cols["sigma_gal"]] = np.random.default_rng(seed + 15485863).uniform(0.0, vdisp, B)
    if escape:
        th[:, cols["frac_obrun"]] = np.random.default_rng(seed + 7919).uniform(0.0, 1.0, B)
    igm = int(igm)
    if igm & 1:
        th[:, cols["igm_factor"]] = np.random.default_rng(seed + 104729).uniform(0.5, 1.5, B)
    if igm & 2:
        th[:, cols["x_hi"]] = np.random.default_rng(seed + 1299709).uniform(0.0, 1.0, B)
    zlo, zhi = cfg.z_range
    th[:, cols["logmass"]] = rng.uniform(8.0, 11.0, B)
    th[:, cols["zred"]] = rng.uniform(zlo, zhi, B)
    if igm & 4:
        r4 = np.random.default_rng(seed + 15485867)
        th[:, cols["log_nhi"]] = r4.uniform(20.0, 22.0, B)
        th[:, cols["z_dla"]] = np.maximum(th[:, cols["zred"]] - r4.uniform(0.0, 0.5, B), 0.0)
    th[:, cols["gas_logz"]] = -0.5
    th[:, cols["gas_logu"]] = -2.5
    th[:, cols["alpha_bc"]] = -0.7
    if cfg.name == "c0":
        th[:, cols["logzsol"]] = rng.uniform(-2.0, 0.0, B)
        th[:, cols["tau_diff"]] = rng.uniform(0.0, 2.0, B)
        m = rng.dirichlet(np.ones(cfg.n_sfh), B)
    else:
        th[:, cols["tau_bc"]] = _trunc_normal(rng, 0.3, 0.5, 0.0, 4.0, B)
        th[:, cols["tau_diff"]] = _trunc_normal(rng, 0.3, 1.0, 0.0, 4.0, B)
        th[:, cols["delta"]] = rng.uniform(-1.0, 0.4, B)
        if cfg.sample_alpha_bc:
            th[:, cols["alpha_bc"]] = rng.uniform(-1.5, -0.3, B)
        if cfg.n_lines:
            th[:, cols["gas_logz"]] = rng.uniform(-1.3, 0.3, B)
            th[:, cols["gas_logu"]] = rng.uniform(-4.0, -1.0, B)
        steps = _clipped_t(rng, 2, 0.3, 1.0, (B, cfg.n_sfh - 1))
        logm = np.concatenate([np.zeros((B, 1)), np.cumsum(steps, axis=1)], axis=1)
        m = 10.0 ** logm
        m /= m.sum(axis=1, keepdims=True)
        zlo_g, zhi_g = min(cfg.logz), max(cfg.logz)
        if cfg.n_zh:
            z0 = rng.uniform(-2.2, 0.3, B)
            walk = _clipped_t(rng, 2, 0.2, 1.0, (B, cfg.n_zh - 1))
            zh = np.concatenate([z0[:, None], z0[:, None] + np.cumsum(walk, axis=1)], axis=1)
            th[:, cols["zh"]:cols["zh"] + cfg.n_zh] = np.clip(zh, zlo_g, zhi_g)
        else:
            th[:, cols["logzsol"]] = rng.uniform(-2.2, 0.3, B)
        if len(cfg.afe) > 1:
            th[:, cols["afe"]] = rng.uniform(min(cfg.afe), max(cfg.afe), B)
    th[:, cols["sfh"]:cols["sfh"] + cfg.n_sfh] = m if sfh_scheme == "step" else m * cfg.n_sfh / 1e10
    return th


def perturb_theta(cfg: Config, theta: np.ndarray, scale: float, seed: int) -> np.ndarray:
    """Small seeded perturbations of theta (live points near a reference point).

    Masses are perturbed multiplicatively and renormalised; everything stays in
    its prior range.
    """
    rng = np.random.default_rng(seed)
    cols = theta_columns(cfg.n_sfh, cfg.n_zh)
    th = theta.copy()
    B = th.shape[0]
    for name, lo, hi in (("logmass", 6.0, 12.5), ("tau_bc", 0.0, 4.0), ("tau_diff", 0.0, 4.0),
                         ("delta", -1.0, 0.4)):
        th[:, cols[name]] = np.clip(th[:, cols[name]] + scale * rng.normal(size=B), lo, hi)
    zlo, zhi = cfg.z_range
    th[:, cols["zred"]] = np.clip(th[:, cols["zred"]] + 0.1 * scale * rng.normal(size=B), zlo, zhi)
    s0, n = cols["sfh"], cfg.n_sfh
    m = th[:, s0:s0 + n] * np.exp(scale * rng.normal(size=(B, n)))
    th[:, s0:s0 + n] = m / m.sum(axis=1, keepdims=True)
    # metallicities stay strictly inside the grid (away from the clamp at its ends)
    zlo_g, zhi_g = min(cfg.logz), max(cfg.logz)
    margin = 1e-3 * (zhi_g - zlo_g)
    zlo_g, zhi_g = zlo_g + margin, zhi_g - margin
    if cfg.n_zh:
        z0 = cols["zh"]
        th[:, z0:z0 + cfg.n_zh] = np.clip(th[:, z0:z0 + cfg.n_zh]
                                         + scale * rng.normal(size=(B, cfg.n_zh)), zlo_g, zhi_g)
    else:
        th[:, cols["logzsol"]] = np.clip(th[:, cols["logzsol"]] + scale * rng.normal(size=B),
                                         zlo_g, zhi_g)
    if len(cfg.afe) > 1:
        alo, ahi = min(cfg.afe), max(cfg.afe)
        am = 1e-3 * (ahi - alo)
        th[:, cols["afe"]] = np.clip(th[:, cols["afe"]], alo + am, ahi - am)
    return th


def noisy_photometry(model: np.ndarray, seed: int, frac: float = 0.05):
    """Data = model + frac*model*N(0,1); sigma = frac*|model| (per band)."""
    rng = np.random.default_rng(seed)
    sig = frac * np.abs(model)
    return model + sig * rng.normal(size=model.shape), sig


def noisy_spectrum(model: np.ndarray, seed: int):
    """sigma_i = 0.05|m_i| + 0.01 median|m|; data = model + sigma N(0,1)."""
    rng = np.random.default_rng(seed)
    sig = 0.05 * np.abs(model) + 0.01 * np.median(np.abs(model))
    return model + sig * rng.normal(size=model.shape), sig


# ----------------------------------------------------------------------------
# Serving stream
# ----------------------------------------------------------------------------
def make_requests(n: int, rate_hz: float = 50.0, seed: int = 7, max_points: int = 1024):
    """Poisson arrivals; half photometry (8-25 bands), half prism spectra (400-3000 px).

    Each request carries B_r in {64, 128, ..., max_points} live points and its own seed.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    reqs = []
    for i in range(n):
        kind = "phot" if rng.uniform() < 0.5 else "spec"
        size = int(rng.integers(8, 26)) if kind == "phot" else int(rng.integers(400, 3001))
        B_r = 64 * int(rng.integers(1, max_points // 64 + 1))
        reqs.append(dict(id=i, arrival_s=float(t[i]), kind=kind, size=size, B=B_r,
                         seed=int(rng.integers(0, 2 ** 31 - 1))))
    return reqs
