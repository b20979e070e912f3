"""Flat LambdaCDM luminosity distance and age of the Universe (Sec. 2.6).

The paper evaluates D_L(z) and the age of the Universe with a flat-LambdaCDM
cosmology (no radiation term) chosen at construction; the workloads use
H0 = 70 km/s/Mpc and Omega_m = 0.3.  Here the comoving distance is an adaptive
quadrature of 1/E(z) and the age has its closed form.
"""
import math

import numpy as np
from scipy import integrate

from .constants import C_KMS, MPC_CM, MPC_KM, YR_S


def E(z, Om):
    """Dimensionless Hubble rate of a flat universe: sqrt(Om (1+z)^3 + 1 - Om)."""
    return np.sqrt(Om * (1.0 + z) ** 3 + (1.0 - Om))


def comoving_distance_mpc(z, H0, Om):
    """D_C(z) = (c/H0) * integral_0^z dz'/E(z') [Mpc], adaptive quadrature, rtol 1e-13."""
    zs = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.empty_like(zs)
    for i, zi in enumerate(zs):
        val, _ = integrate.quad(lambda x: 1.0 / E(x, Om), 0.0, float(zi),
                                epsabs=0.0, epsrel=1e-13, limit=400)
        out[i] = (C_KMS / H0) * val
    return out if np.ndim(z) else out[0]


def luminosity_distance_cm(z, H0, Om):
    """D_L(z) = (1+z) D_C(z) [cm]."""
    return (1.0 + np.asarray(z)) * comoving_distance_mpc(z, H0, Om) * MPC_CM


def hubble_time_yr(H0):
    """1/H0 in years."""
    return MPC_KM / H0 / YR_S


def age_of_universe_yr(z, H0, Om):
    """Closed form for a flat universe: t(z) = 2/(3 H0 sqrt(OL)) asinh(sqrt(OL/Om) (1+z)^-3/2)."""
    OL = 1.0 - Om
    z = np.asarray(z, dtype=np.float64)
    return (hubble_time_yr(H0) * 2.0 / (3.0 * math.sqrt(OL))
            * np.arcsinh(math.sqrt(OL / Om) * (1.0 + z) ** -1.5))


def d_age_dz_yr(z, H0, Om):
    """dt/dz = -1/(H0 (1+z) E(z)) (the defining integrand of the age)."""
    z = np.asarray(z, dtype=np.float64)
    return -hubble_time_yr(H0) / ((1.0 + z) * E(z, Om))


def d_luminosity_distance_dz_cm(z, H0, Om):
    """dD_L/dz = D_C + (1+z) (c/H0)/E(z) [cm]."""
    z = np.asarray(z, dtype=np.float64)
    return (comoving_distance_mpc(z, H0, Om) + (1.0 + z) * (C_KMS / H0) / E(z, Om)) * MPC_CM
