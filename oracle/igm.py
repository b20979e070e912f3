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
These are the published coefficients of Madau (1995); the higher series lines and the
damping wing / DLA options of the paper are not included.  Parity unpinned for the
coefficients themselves (nothing outside the formula fixes them here): the pins cover
the structure (identity redward of Ly alpha and at f = 0, the power-law dependence on f,
the Lyman-limit onset).
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


def transmission(lam_obs, z, factor=1.0):
    """T = exp(-factor tau)."""
    return np.exp(-factor * madau_tau(lam_obs, z))
