"""Pins for the oracle's flat-LambdaCDM distances and ages (Sec. 2.6).

Each check uses something other than the oracle's own formula: the Einstein-de
Sitter and pure-Lambda limits, an independent quadrature rule, the age as a
numerical integral of dt = -dz/((1+z) H(z)), and finite differences.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import cosmology as co
from oracle.constants import C_KMS, MPC_CM, MPC_KM, YR_S

H0 = 70.0


@pytest.mark.parametrize("z", [0.1, 1.0, 3.5, 8.0, 12.0])
def test_einstein_de_sitter_limit(z):
    # Omega_m = 1: D_C = 2c/H0 (1 - (1+z)^-1/2), t = 2/(3 H0) (1+z)^-3/2
    dc = co.comoving_distance_mpc(z, H0, 1.0)
    assert dc == pytest.approx(2 * C_KMS / H0 * (1 - (1 + z) ** -0.5), rel=1e-13, abs=0.0)
    t = co.age_of_universe_yr(z, H0, 1.0 - 1e-13)
    t_eds = 2.0 / 3.0 * (MPC_KM / H0 / YR_S) * (1 + z) ** -1.5
    assert t == pytest.approx(t_eds, rel=1e-9, abs=0.0)


@pytest.mark.parametrize("z", [0.5, 2.0, 9.0])
def test_pure_lambda_limit(z):
    # Omega_m -> 0: E = 1, D_C = c z / H0
    assert co.comoving_distance_mpc(z, H0, 0.0) == pytest.approx(C_KMS * z / H0, rel=1e-13, abs=0.0)


@pytest.mark.parametrize("z", [0.5, 1.0, 4.43, 8.0, 12.0])
def test_distance_two_independent_rules(z):
    # adaptive quadrature vs a 400-node Gauss-Legendre rule
    x, w = np.polynomial.legendre.leggauss(400)
    zz = 0.5 * z * (x + 1.0)
    gl = 0.5 * z * np.sum(w / np.sqrt(0.3 * (1 + zz) ** 3 + 0.7)) * C_KMS / H0
    assert co.comoving_distance_mpc(z, H0, 0.3) == pytest.approx(gl, rel=1e-13, abs=0.0)


@pytest.mark.parametrize("z", [0.0, 0.5, 3.0, 12.0])
def test_age_equals_time_integral(z):
    # t(z) = (1/H0) * integral_z^inf dz' / ((1+z') E(z')), with a = 1/(1+z) substitution
    f = lambda a: 1.0 / (a * math.sqrt(0.3 / a ** 3 + 0.7))
    val, _ = integrate.quad(f, 0.0, 1.0 / (1.0 + z), epsabs=0, epsrel=1e-13, limit=400)
    t_int = val * MPC_KM / H0 / YR_S
    assert co.age_of_universe_yr(z, H0, 0.3) == pytest.approx(t_int, rel=1e-11, abs=0.0)


@pytest.mark.parametrize("z", [0.7, 3.0, 11.0])
def test_derivatives_by_finite_difference(z):
    h = 1e-5
    fd_t = (co.age_of_universe_yr(z + h, H0, 0.3) - co.age_of_universe_yr(z - h, H0, 0.3)) / (2 * h)
    assert co.d_age_dz_yr(z, H0, 0.3) == pytest.approx(fd_t, rel=1e-8, abs=0.0)
    fd_d = (co.luminosity_distance_cm(z + h, H0, 0.3) - co.luminosity_distance_cm(z - h, H0, 0.3)) / (2 * h)
    assert co.d_luminosity_distance_dz_cm(z, H0, 0.3) == pytest.approx(fd_d, rel=1e-8, abs=0.0)


def test_luminosity_distance_is_one_plus_z_times_comoving():
    z = 2.7
    assert co.luminosity_distance_cm(z, H0, 0.3) == pytest.approx(
        (1 + z) * co.comoving_distance_mpc(z, H0, 0.3) * MPC_CM, rel=1e-15, abs=0.0)
