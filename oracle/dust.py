"""Two-component dust attenuation (Sec. 2.4, App. D.1, eq. D1-D2).

Birth cloud: power law tau_BC(lambda) = tau_bc (lambda/5500 A)^alpha_bc on SSP
ages younger than the birth-cloud edge.  Diffuse screen on all ages, in the
Kriek & Conroy form tau_d = tau_diff (lambda/5500)^delta [a(lambda) + E_b(delta) d(lambda)]
with E_b = 0.85 - 1.9 delta.  The shape tables a and d are static inputs
(the paper's sedpy/FSPS curves are not available).  With the two-bin one-hot
age-to-bin matrix, eq. D2 becomes F = e^{-tau_d} (Y e^{-tau_BC} + O).
"""
import numpy as np

from .constants import LAM_V


def birth_cloud_tau(wave, tau_bc, alpha_bc):
    return tau_bc * (np.asarray(wave) / LAM_V) ** alpha_bc


def diffuse_tau(wave, tau_diff, delta, a_tab, d_tab):
    Eb = 0.85 - 1.9 * delta
    return tau_diff * (np.asarray(wave) / LAM_V) ** delta * (a_tab + Eb * d_tab)


def attenuate(young, old, wave, tau_bc, alpha_bc, tau_diff, delta, a_tab, d_tab):
    """F = exp(-tau_d) * (Y exp(-tau_BC) + O) on one rest-frame spectrum."""
    T_bc = np.exp(-birth_cloud_tau(wave, tau_bc, alpha_bc))
    T_d = np.exp(-diffuse_tau(wave, tau_diff, delta, a_tab, d_tab))
    return T_d * (young * T_bc + old)
