"""Intergalactic-medium transmission (Sec. 2.6, final paragraph): the Madau (1995) mean
transmission of the Lyman-series forest and of Lyman-limit systems, with the optional free
scaling theta[igm_factor] of the optical depth.

T(lambda_obs) = exp(-f tau(lambda_obs)),
  tau = sum over the series lines j (Ly alpha .. Ly delta, lambda_j = 1215.67, 1025.72,
        972.54, 949.74 A) with lambda_j < lambda_obs < lambda_j (1 + z) of
        A_j (lambda_obs / lambda_j)^3.46, A_j = 3.6e-3, 1.7e-3, 1.2e-3, 9.3e-4;
      + below the Lyman limit of the source (lambda_obs < 911.75 (1 + z)), with
        x_c = lambda_obs / 911.75 and x_e = 1 + z, the photoelectric term
        0.25 x_c^3 (x_e^0.46 - x_c^0.46) + 9.4 x_c^1.5 (x_e^0.18 - x_c^0.18)
        - 0.7 x_c^3 (x_c^-1.32 - x_e^-1.32) - 0.023 (x_e^1.68 - x_c^1.68).
These are the published coefficients of Madau (1995); the higher series lines are not
included.  Parity unpinned for the coefficients themselves (nothing outside the formula
fixes them here): the pins cover the structure (identity redward of Ly alpha and at f = 0,
the power-law dependence on f, the Lyman-limit onset).

The paper's two optional additions (Sec. 2.6), each on top of the Madau IGM:

* the damping wing of a partly neutral IGM (Miralda-Escude 1998; Totani et al. 2006) with
  neutral fraction theta[x_HI]: redward of the source's Lyman alpha,
    tau_DW = x_HI tau_GP(z) (R_alpha / pi) (1 + z_o)^{3/2} / (1 + z)^{3/2} [I(x_u) - I(x_l)],
  1 + z_o = lambda_obs / lambda_alpha, x_u = (1 + z) / (1 + z_o), x_l = (1 + z_l) / (1 + z_o)
  (0 where z <= z_l), I(x) = x^{9/2} / (1 - x) + 9/7 x^{7/2} + 9/5 x^{5/2} + 3 x^{3/2}
  + 9 x^{1/2} - 9/2 ln((1 + x^{1/2}) / (1 - x^{1/2})) (the antiderivative of
  x^{9/2} / (1 - x)^2: the scattering wing K Gamma (nu / nu_alpha)^4 / (4 pi^2 (nu -
  nu_alpha)^2) integrated through a matter-dominated IGM), R_alpha = Gamma_alpha
  lambda_alpha / (4 pi c); blueward of it, where
  the photon redshifts through Lyman alpha inside the neutral region (z_l < z_o < z), the
  resonant Gunn-Peterson depth x_HI tau_GP(z_o).
  Readings: the neutral region extends from the source down to z_l = 6 (the end of
  reionisation, as in Totani et al.), and tau_GP(z) = 3.88e5 ((1 + z) / 7)^{3/2};
* a damped Lyman-alpha absorber (Tepper-Garcia 2006) of column density 10^theta[logN_HI]
  cm^-2 at redshift theta[z_dla]: tau = N sigma(lambda_obs / (1 + z_dla)) with the Voigt
  cross-section sigma = (pi e^2 / (m_e c)) f_alpha H(a, x) / (sqrt(pi) dnu_D), dnu_D = b /
  lambda_alpha, x = (nu - nu_alpha) / dnu_D, a = Gamma_alpha / (4 pi dnu_D), and Tepper-
  Garcia's approximation H(a, x) = H0 - a / (sqrt(pi) x^2) [H0^2 (4 x^4 + 7 x^2 + 4 + 1.5
  x^-2) - 1.5 x^-2 - 1], H0 = exp(-x^2) (for x^2 < 1e-4 its limit H0 - a (2 - 4 x^2 +
  5/3 x^4) / sqrt(pi), the same expression without the cancellation).
  Reading: Lyman alpha only, with a Doppler parameter b = 10 km/s.
"""
import numpy as np

LYMAN_SERIES = (1215.67, 1025.72, 972.54, 949.74)   # A
LYMAN_A = (3.6e-3, 1.7e-3, 1.2e-3, 9.3e-4)
LYMAN_LIMIT = 911.75                                # A


def madau_tau(lam_obs, z):
    """Optical depth tau(lambda_obs) of the Madau (1995) mean IGM for a source at z."""
    lam = np.asarray(lam_obs, dtype=np.float64)
    tau = np.zeros_like(lam)
    for lj, aj in zip(LYMAN_SERIES, LYMAN_A):
        on = (lam > lj) & (lam < lj * (1.0 + z))
        tau = tau + np.where(on, aj * (lam / lj) ** 3.46, 0.0)
    xe = 1.0 + z
    xc = lam / LYMAN_LIMIT
    on = (xc > 1.0) & (xc < xe)
    xs = np.where(on, xc, 1.0)
    cont = (0.25 * xs ** 3 * (xe ** 0.46 - xs ** 0.46) + 9.4 * xs ** 1.5 * (xe ** 0.18 - xs ** 0.18)
            - 0.7 * xs ** 3 * (xs ** -1.32 - xe ** -1.32) - 0.023 * (xe ** 1.68 - xs ** 1.68))
    return tau + np.where(on, cont, 0.0)


# Lyman alpha: wavelength, rest-frame Einstein A (damping constant) and oscillator strength
LYA_CM = 1215.67e-8
LYA_GAMMA = 6.265e8                # s^-1
LYA_F = 0.4164
E_ESU = 4.80320471e-10             # electron charge [esu]
ME_G = 9.1093837015e-28            # electron mass [g]
C_CMS = 2.99792458e10
Z_NEUTRAL_END = 6.0                # low-redshift edge of the neutral region (reading)
DLA_B_KMS = 10.0                   # Doppler parameter of the absorber (reading)


def tau_gp(z):
    """Gunn-Peterson optical depth of a fully neutral IGM at z (reading: 3.88e5 ((1+z)/7)^1.5)."""
    return 3.88e5 * ((1.0 + np.asarray(z, dtype=np.float64)) / 7.0) ** 1.5


def _I(x):
    s = np.sqrt(x)
    return (x ** 4.5 / (1.0 - x) + 9.0 / 7.0 * x ** 3.5 + 9.0 / 5.0 * x ** 2.5 + 3.0 * x ** 1.5 + 9.0 * s
            - 4.5 * np.log((1.0 + s) / (1.0 - s)))


def damping_wing_tau(lam_obs, z, x_hi):
    """Optical depth of a neutral IGM of fraction x_hi between z_l = 6 and the source at z:
    the Lorentzian wing of Lyman alpha redward of the source's line, the resonant
    Gunn-Peterson depth where the photon crosses Lyman alpha inside the region."""
    lam = np.asarray(lam_obs, dtype=np.float64)
    tau = np.zeros_like(lam)
    if z <= Z_NEUTRAL_END or x_hi == 0.0:
        return tau
    r_alpha = LYA_GAMMA * LYA_CM / (4.0 * np.pi * C_CMS)
    opz_o = lam * 1e-8 / LYA_CM
    red = opz_o > 1.0 + z
    o = np.where(red, opz_o, 2.0 * (1.0 + z))
    xu = (1.0 + z) / o
    xl = (1.0 + Z_NEUTRAL_END) / o
    wing = x_hi * tau_gp(z) * r_alpha / np.pi * (o / (1.0 + z)) ** 1.5 * (_I(xu) - _I(xl))
    tau = np.where(red, wing, tau)
    trough = (opz_o > 1.0 + Z_NEUTRAL_END) & (opz_o < 1.0 + z)
    return np.where(trough, x_hi * tau_gp(opz_o - 1.0), tau)


def voigt_tepper_garcia(a, x):
    """Tepper-Garcia (2006) approximation of the Voigt-Hjerting function H(a, x)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    u = x * x
    h0 = np.exp(-u)
    small = u < 1e-4
    us = np.where(small, 1.0, u)
    full = (h0 * h0 * (4.0 * us * us + 7.0 * us + 4.0 + 1.5 / us) - 1.5 / us - 1.0) / us
    series = 2.0 - 4.0 * u + 5.0 / 3.0 * u * u
    return h0 - a / np.sqrt(np.pi) * np.where(small, series, full)


def dla_tau(lam_obs, z_dla, log_nhi, b_kms=DLA_B_KMS):
    """Optical depth of a damped Lyman-alpha absorber of column 10^log_nhi cm^-2 at z_dla."""
    lam_r = np.asarray(lam_obs, dtype=np.float64) * 1e-8 / (1.0 + z_dla)     # absorber frame [cm]
    dnu_d = b_kms * 1e5 / LYA_CM
    x = (C_CMS / lam_r - C_CMS / LYA_CM) / dnu_d
    a = LYA_GAMMA / (4.0 * np.pi * dnu_d)
    sigma = np.pi * E_ESU ** 2 / (ME_G * C_CMS) * LYA_F * voigt_tepper_garcia(a, x) / (np.sqrt(np.pi) * dnu_d)
    return 10.0 ** log_nhi * sigma


def transmission(lam_obs, z, factor=1.0, x_hi=None, log_nhi=None, z_dla=None):
    """T = exp(-(factor tau_Madau + tau_DW + tau_DLA)); the damping wing with x_hi given,
    the absorber with log_nhi and z_dla given."""
    tau = factor * madau_tau(lam_obs, z)
    if x_hi is not None:
        tau = tau + damping_wing_tau(lam_obs, z, x_hi)
    if log_nhi is not None:
        tau = tau + dla_tau(lam_obs, z_dla, log_nhi)
    return np.exp(-tau)
