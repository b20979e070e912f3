"""Nebular line emission (Sec. 2.3, App. C).

* Q_ma, the hydrogen-ionising photon rate of each unattenuated SSP (eq. C1).  The
  library stores f_lambda in Lsun/A/Msun, so the photon integral is written as
  (Lsun/(h c)) * integral_{lambda <= 912 A} f_lambda lambda d lambda, the same
  quantity as eq. C1's integral of f_nu/lambda; it is a trapezoid over the
  library's own nodes at or below 912 A.
* line luminosities L_l = sum over nebular-covered nodes of W_ma Q_ma 10^Lhat_l(a)
  (eq. C2), with Lhat bilinearly interpolated in (gas_logz, gas_logu) on the
  table at each SSP age (the table's age axis is the SSP ages it covers).
* on the model wavelength grid each line is a Gaussian of width two local pixels,
  normalised on the grid so that its flux is conserved (Sec. 2.3.1, App. C).
  Reading: sigma = 2 (lambda_{k+1} - lambda_k) for the pixel k containing the
  line, truncated at 5 sigma, normalised with trapezoid weights.
"""
import numpy as np

from .constants import ANG_CM, C_CMS, H_PLANCK, LAM_LYMAN, LSUN
from .sfh import grid_split


def trapezoid_weights(x):
    """Weights w_k with sum_k w_k f_k equal to the trapezoid rule on nodes x."""
    x = np.asarray(x, dtype=np.float64)
    w = np.zeros_like(x)
    dx = np.diff(x)
    w[:-1] += 0.5 * dx
    w[1:] += 0.5 * dx
    return w


def ionising_rate(wave, flux):
    """Q[..., a] in photons/s per Msun from flux[..., a, wave] (eq. C1)."""
    sel = wave <= LAM_LYMAN
    lam = wave[sel]
    integrand = flux[..., sel] * lam
    integral = np.trapezoid(integrand, lam, axis=-1)      # Lsun * A  (per Msun)
    return LSUN * ANG_CM * integral / (H_PLANCK * C_CMS)


def line_table_interp(table, zg_nodes, u_nodes, gas_logz, gas_logu):
    """Lhat[l, a_neb]: bilinear interpolation in (Z_gas, log U), clamped to the table."""
    jz, tz = grid_split(gas_logz, zg_nodes)
    ju, tu = grid_split(gas_logu, u_nodes)
    return ((1 - tz) * (1 - tu) * table[:, :, jz, ju]
            + (1 - tz) * tu * table[:, :, jz, ju + 1]
            + tz * (1 - tu) * table[:, :, jz + 1, ju]
            + tz * tu * table[:, :, jz + 1, ju + 1])


def line_luminosity(W, Q, lhat, n_neb):
    """L_l [erg/s per unit of the weights' mass] = sum_{alpha, m, a<n_neb} W Q 10^Lhat_l(a)."""
    WQ = (W[:, :, :n_neb] * Q[:, :, :n_neb]).sum(axis=(0, 1))   # [a_neb]
    return (10.0 ** lhat) @ WQ


def line_profiles_grid(wave, line_wave):
    """G[l, k]: per-Angstrom line profiles on the model grid (unit trapezoid integral)."""
    wt = trapezoid_weights(wave)
    G = np.zeros((len(line_wave), len(wave)))
    for l, lam in enumerate(line_wave):
        k = int(np.searchsorted(wave, lam, side="right")) - 1
        k = min(max(k, 0), len(wave) - 2)
        sig = 2.0 * (wave[k + 1] - wave[k])
        g = np.exp(-0.5 * ((wave - lam) / sig) ** 2)
        g[np.abs(wave - lam) > 5.0 * sig] = 0.0
        G[l] = g / np.sum(g * wt)
    return G
