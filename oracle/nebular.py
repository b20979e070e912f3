"""Nebular line emission (Sec. 2.3, App. C).

* Q_ma, the hydrogen-ionising photon rate of each unattenuated SSP (eq. C1).  The
  library stores f_lambda in Lsun/A/Msun, so the photon integral is written as
  (Lsun/(h c)) * integral_{lambda <= 912 A} f_lambda lambda d lambda, the same
  quantity as eq. C1's integral of f_nu/lambda; it is a trapezoid over the
  library's own nodes at or below 912 A.
* line luminosities L_l = sum over nebular-covered nodes of W_ma Q_ma 10^Lhat_l(a)
  (eq. C2), with Lhat interpolated trilinearly in (gas_logz, age, gas_logu) on the
  table's own axes (a table without an age axis of its own is on the birth-cloud
  SSP ages, where the age weights are 0 and 1).
* the nebular continuum, likewise: sum over the same nodes of W_ma Q_ma 10^Chat(a, lambda)
  with Chat trilinear in the continuum cube (eq. C2).
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


def line_luminosity(W, Q, lhat, n_neb, a0=0):
    """L_l [erg/s per unit of the weights' mass] = sum_{alpha, m, a0<=a<n_neb} W Q 10^Lhat_l(a)."""
    WQ = (W[:, :, a0:n_neb] * Q[:, :, a0:n_neb]).sum(axis=(0, 1))   # [a_neb]
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


# ---------------------------------------------------------------------------------
# Full grid evaluation: trilinear cubes and the nebular continuum (App. C)
# ---------------------------------------------------------------------------------
def trilinear(cube, zg_nodes, tau_nodes, u_nodes, gas_logz, tau, gas_logu):
    """Trilinear interpolation of cube[..., i_zg, j_tau, k_u] (trailing three axes) at
    (gas_logz, tau, gas_logu), each coordinate clamped to its axis: the sum over the
    eight corners of the bracketing cell of the product of the three 1-D hat weights.

    Reading (App. C): the age coordinate is the age itself, linear in tau, like the
    other two axes, which are already logarithmic quantities (log Z_gas/Z_sun, log U).
    """
    jz, tz = grid_split(gas_logz, zg_nodes)
    jt, tt = grid_split(tau, tau_nodes)
    ju, tu = grid_split(gas_logu, u_nodes)
    out = 0.0
    for dz, wz in ((0, 1.0 - tz), (1, tz)):
        for dt, wt in ((0, 1.0 - tt), (1, tt)):
            for du, wu in ((0, 1.0 - tu), (1, tu)):
                out = out + wz * wt * wu * cube[..., jz + dz, jt + dt, ju + du]
    return out


def nebular_age_mask(ages, tau_ranges):
    """SSP ages that take nebular emission: those inside every cube's tabulated age range
    (the overlap of the continuum and line grids, App. C); the others get none."""
    ages = np.asarray(ages, dtype=np.float64)
    sel = np.ones(len(ages), dtype=bool)
    for lo, hi in tau_ranges:
        sel &= (ages >= lo) & (ages <= hi)
    return sel


def line_table_at_ages(line_cube, zg_nodes, tau_nodes, u_nodes, gas_logz, gas_logu, ages):
    """Lhat[l, a] = trilinear(log10(L_l/Q)) at (gas_logz, age a, gas_logu) for the given
    SSP ages; line_cube is [n_line][n_tau][n_zg][n_u] (the table's own axes)."""
    cube = np.moveaxis(line_cube, 1, 2)            # -> [l][zg][tau][u]
    return np.stack([trilinear(cube, zg_nodes, tau_nodes, u_nodes, gas_logz, t, gas_logu)
                     for t in ages], axis=1)


def continuum_at_ages(cont_cube, zg_nodes, tau_nodes, u_nodes, gas_logz, gas_logu, ages):
    """Chat[a, lambda] = trilinear(log10(L_nu/Q)) at (gas_logz, age a, gas_logu);
    cont_cube is [n_tau][n_zg][n_u][n_wave] (L_nu in erg/s/Hz, Q in photons/s)."""
    cube = np.moveaxis(cont_cube, (0, 1, 2), (-2, -3, -1))   # -> [wave][zg][tau][u]
    return np.stack([trilinear(cube, zg_nodes, tau_nodes, u_nodes, gas_logz, t, gas_logu)
                     for t in ages], axis=0)


def continuum_luminosity(W, Q, chat, sel, wave):
    """Nebular continuum added to the young light [Lsun/A per unit of the weights' mass]:
    sum over nebular ages a and nodes (alpha, m) of W Q 10^Chat(a, lambda) (App. C), the
    per-photon L_nu turned into L_lambda = L_nu c / lambda^2 and divided by Lsun."""
    WQ = (W[:, :, sel] * Q[:, :, sel]).sum(axis=(0, 1))      # [a_neb]
    lnu = WQ @ (10.0 ** chat)                                 # erg/s/Hz
    return lnu * (C_CMS / ANG_CM) / wave ** 2 / LSUN
