"""Pins for the oracle's spectrophotometric calibration polynomial (Sec. 3.2, App. H.3,
eq. app_polymarg).

The marginal likelihood is checked against direct numerical integration of its definition,
the product of the Gaussian likelihood of the calibrated model and the Gaussian prior of the
coefficients, over a grid of coefficients (one and two coefficients); its s_m -> 0 limit is
the uncalibrated likelihood (the paper states the reduction); the Occam term is never
positive; and the optimised polynomial recovers a known calibration from noise-free data.
"""
import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import likelihood as lk


def _toy(n=60, seed=0):
    rng = np.random.default_rng(seed)
    lam = np.linspace(6000.0, 9000.0, n)
    mu = 1.0 + 0.3 * np.sin(lam / 500.0)
    sigma = 0.05 + 0.02 * rng.random(n)
    data = mu * (1.0 + 0.04 - 0.03 * (2 * (lam - lam[0]) / (lam[-1] - lam[0]) - 1)) + sigma * rng.normal(size=n)
    mask = np.ones(n, dtype=bool)
    mask[[3, 17]] = False
    return lam, mu, sigma, data, mask


def _direct(lam, mu, sigma, data, mask, order, sd, grids):
    """ln of the integral over c of N(d; mu (1 + A c), C) N(c; 0, diag(sd^2)) on a grid."""
    A = lk.chebyshev_design(lam, order)
    mesh = np.meshgrid(*grids, indexing="ij")
    cs = np.stack([m.ravel() for m in mesh], axis=1)
    dv = np.prod([g[1] - g[0] for g in grids])
    vals = []
    for c in cs:
        model = mu * (1.0 + A @ c)
        # the likelihood of the calibrated model with the noise fixed at the uncalibrated one
        r = np.where(mask, data - model, 0.0)
        v = np.where(mask, sigma, 1.0) ** 2
        ll = np.sum(np.where(mask, -0.5 * r * r / v - 0.5 * np.log(2 * np.pi * v), 0.0))
        lp = np.sum(-0.5 * (c / sd) ** 2 - 0.5 * np.log(2 * np.pi * sd ** 2))
        vals.append(ll + lp)
    return logsumexp(vals) + np.log(dv)


def test_marginal_likelihood_matches_direct_integration_one_coefficient():
    lam, mu, sigma, data, mask = _toy()
    sd = np.array([0.1])
    closed = lk.calibrated_lnlike(data, mu, sigma, mask, lk.chebyshev_design(lam, 0), sd, "marginal")
    g = np.linspace(-0.1, 0.2, 6001)
    assert closed == pytest.approx(_direct(lam, mu, sigma, data, mask, 0, sd, [g]), rel=0.0, abs=1e-7)


def test_marginal_likelihood_matches_direct_integration_two_coefficients():
    lam, mu, sigma, data, mask = _toy(seed=1)
    sd = np.array([0.1, 0.05])
    closed = lk.calibrated_lnlike(data, mu, sigma, mask, lk.chebyshev_design(lam, 1), sd, "marginal")
    g0 = np.linspace(-0.05, 0.12, 701)
    g1 = np.linspace(-0.12, 0.07, 701)
    assert closed == pytest.approx(_direct(lam, mu, sigma, data, mask, 1, sd, [g0, g1]), rel=0.0, abs=1e-5)


def test_tight_prior_reduces_to_the_uncalibrated_likelihood():
    lam, mu, sigma, data, mask = _toy(seed=2)
    base = lk.lnlike(data, mu, sigma, mask)
    A = lk.chebyshev_design(lam, 3)
    got = lk.calibrated_lnlike(data, mu, sigma, mask, A, np.full(4, 1e-9), "marginal")
    assert got == pytest.approx(base, rel=0.0, abs=1e-9)
    got = lk.calibrated_lnlike(data, mu, sigma, mask, A, np.full(4, 1e-9), "optimise")
    assert got == pytest.approx(base, rel=0.0, abs=1e-9)


def test_occam_term_is_never_positive_and_the_gain_never_negative():
    lam, mu, sigma, data, mask = _toy(seed=3)
    for order, sd in ((0, [0.3]), (2, [0.1, 0.2, 0.05]), (5, np.full(6, 1.0))):
        A = lk.chebyshev_design(lam, order)
        sd = np.asarray(sd, dtype=float)
        iv = np.where(mask, 1.0 / sigma ** 2, 0.0)
        D = mu[:, None] * A
        M = D.T @ (iv[:, None] * D) + np.diag(1.0 / sd ** 2)
        _, ld = np.linalg.slogdet(M * sd[None, :] ** 2)
        assert -0.5 * ld <= 0.0
        got = lk.calibrated_lnlike(data, mu, sigma, mask, A, sd, "marginal")
        r = np.where(mask, data - mu, 0.0)
        b = D.T @ (iv * r)
        assert got - lk.lnlike(data, mu, sigma, mask) + 0.5 * ld == pytest.approx(
            0.5 * b @ np.linalg.solve(M, b), rel=1e-10, abs=0.0)


def test_optimised_polynomial_recovers_a_known_calibration():
    lam = np.linspace(6000.0, 9000.0, 200)
    mu = 1.0 + 0.3 * np.sin(lam / 500.0)
    c_true = np.array([0.05, -0.02, 0.01, 0.004])
    A = lk.chebyshev_design(lam, 3)
    data = mu * (1.0 + A @ c_true)
    sigma = np.full(lam.size, 1e-3)
    mask = np.ones(lam.size, dtype=bool)
    got = lk.calibrated_lnlike(data, mu, sigma, mask, A, np.full(4, 1e4), "optimise")
    # the residual left after the fit is the prior's pull, ~ (sigma / s)^2: the likelihood is
    # the noise normalisation alone
    assert got == pytest.approx(np.sum(-0.5 * np.log(2 * np.pi * sigma ** 2)), rel=0.0, abs=1e-6)
    assert np.allclose(A[:, 0], 1.0) and np.allclose(A[[0, -1], 1], [-1.0, 1.0])
