"""Observation projections: photometry (Sec. 3.1, App. E) and spectra (Sec. 3.2, App. F).

Photometry follows eq. E1-E2 literally: the observer-frame F_nu on the shifted
model grid is turned into f_lambda (the diag(c/lambda_obs^2) factor), linearly
interpolated in wavelength onto each filter's nodes (H; zero outside the model
grid), and summed with the photon-counting weights R_b lambda_j dlambda_j
(Riemann, local spacing by central differences, one-sided at the ends) over
the AB zero point integrated with the trapezoid rule.

Spectra follow eq. F2-F6: per-pixel instrumental dispersion from the LSF mode,
library resolution from the stored grid's two-pixel width, fixed kernel width
with the library term removed, a banded Gaussian response in ln(lambda) shifted
by ln(1+z) (rows normalised, truncated at 5 sigma; rows narrower than half a
log pixel reduce to linear interpolation), plus analytic line profiles on the
detector pixels.
"""
import math

import numpy as np

from .constants import ANG_CM, C_CMS, C_KMS, FNU_AB, FWHM_PER_SIGMA
from .nebular import trapezoid_weights


def local_spacing(x):
    """Central differences (x_{j+1} - x_{j-1})/2, one-sided at the two ends."""
    x = np.asarray(x, dtype=np.float64)
    d = np.empty_like(x)
    d[1:-1] = 0.5 * (x[2:] - x[:-2])
    d[0] = x[1] - x[0]
    d[-1] = x[-1] - x[-2]
    return d


# ----------------------------------------------------------------------------
# Photometry (App. E)
# ----------------------------------------------------------------------------
def ab_zero_point(lam, R):
    """Denominator of eq. E1: sum_j R_j lambda_j dlambda^trap_j f_lambda^AB(lambda_j)."""
    f_ab = FNU_AB * C_CMS / (lam * ANG_CM) ** 2
    return np.sum(R * lam * trapezoid_weights(lam) * f_ab)


def band_maggies(rest_wave, fnu_obs, z, filters):
    """m_b = sum_k T_bk F_nu,k^obs with T = (R H) diag(c / lambda_obs^2) (eq. E2)."""
    lam_obs = (1.0 + z) * rest_wave
    f_lam = C_CMS * fnu_obs / (lam_obs * ANG_CM) ** 2
    out = np.empty(len(filters))
    for b, (lam, R) in enumerate(filters):
        f_nodes = np.interp(lam, lam_obs, f_lam, left=0.0, right=0.0)
        out[b] = np.sum(R * lam * local_spacing(lam) * f_nodes) / ab_zero_point(lam, R)
    return out


# ----------------------------------------------------------------------------
# Spectra (App. F)
# ----------------------------------------------------------------------------
def sigma_inst_kms(lam_obs, mode, value):
    """Instrumental dispersion [km/s] at observed wavelengths (eq. F2).

    ``value`` is a constant or an array tabulated on ``lam_obs``.  A bare ``R``
    is rejected because its convention is ambiguous.
    """
    lam_obs = np.asarray(lam_obs, dtype=np.float64)
    v = np.broadcast_to(np.asarray(value, dtype=np.float64), lam_obs.shape)
    if mode == "R_fwhm":
        return C_KMS / (FWHM_PER_SIGMA * v)
    if mode == "R_sigma":
        return C_KMS / v
    if mode == "fwhm_aa":
        return C_KMS * v / (FWHM_PER_SIGMA * lam_obs)
    if mode == "sigma_aa":
        return C_KMS * v / lam_obs
    if mode == "sigma_kms":
        return np.array(v, dtype=np.float64)
    if mode == "fwhm_kms":
        return v / FWHM_PER_SIGMA
    raise ValueError(f"LSF mode {mode!r} is not one of the six stated conventions")


def sigma_lib_kms(rest_wave):
    """Library resolution floor on its own grid: (c/2.3548) * 2 dlambda/lambda (eq. F3)."""
    return C_KMS / FWHM_PER_SIGMA * 2.0 * local_spacing(rest_wave) / rest_wave


def kernel_sigma_kms(pix_wave, lsf_mode, lsf_value, rest_wave, z_ref, sigma_gal_kms):
    """Continuum kernel width per pixel: sqrt(sigma_fix^2 + sigma_gal^2) (eq. 5, F4)."""
    s_inst = sigma_inst_kms(pix_wave, lsf_mode, lsf_value)
    s_lib = np.interp(pix_wave / (1.0 + z_ref), rest_wave, sigma_lib_kms(rest_wave))
    s_fix2 = np.maximum(s_inst ** 2 - s_lib ** 2, 0.0)
    return np.sqrt(s_fix2 + sigma_gal_kms ** 2)


def lsf_row(pix_lam, sigma_kms, ln_rest, z, trunc=5.0):
    """(indices, weights) of one row of the banded response W_ij (eq. F5).

    ``trunc`` is the truncation in dispersions (five in the paper); tests of the
    redshift gradient widen it so that no node enters or leaves the window.
    """
    x = math.log(pix_lam) - math.log1p(z)
    n = len(ln_rest)
    if x < ln_rest[0] or x > ln_rest[-1]:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    k = int(np.searchsorted(ln_rest, x, side="right")) - 1
    k = min(max(k, 0), n - 2)
    s = sigma_kms / C_KMS
    if s < 0.5 * (ln_rest[k + 1] - ln_rest[k]):
        t = (x - ln_rest[k]) / (ln_rest[k + 1] - ln_rest[k])
        return np.array([k, k + 1]), np.array([1.0 - t, t])
    idx = np.nonzero(np.abs(ln_rest - x) <= trunc * s)[0]
    w = np.exp(-0.5 * ((ln_rest[idx] - x) / s) ** 2)
    return idx, w / w.sum()


def spectrum_continuum(pix_wave, sigma_kms, rest_wave, fnu_obs, z, trunc=5.0):
    """F_nu(lambda_i) = sum_j W_ij F_nu^obs(lambda_j) for every detector pixel."""
    ln_rest = np.log(rest_wave)
    out = np.zeros(len(pix_wave))
    for i, (lam, s) in enumerate(zip(pix_wave, sigma_kms)):
        idx, w = lsf_row(lam, s, ln_rest, z, trunc)
        out[i] = np.dot(w, fnu_obs[idx])
    return out


def line_profile_pixels(pix_wave, line_flux, line_obs_wave, s_line):
    """f_nu^lines(lambda_i) = sum_l F_l (lambda_i/c) N(ln lambda_i; ln lambda_l^obs, s_l) (eq. F6)."""
    lnp = np.log(pix_wave)[:, None]
    lnl = np.log(line_obs_wave)[None, :]
    g = np.exp(-0.5 * ((lnp - lnl) / s_line[None, :]) ** 2) / (math.sqrt(2 * math.pi) * s_line[None, :])
    return (pix_wave * ANG_CM / C_CMS) * (g @ line_flux)
