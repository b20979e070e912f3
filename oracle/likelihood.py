"""Diagonal Gaussian log-likelihood with the systematic noise floor.

Eq. (6) summed over the inclusion mask, with the normalisation term kept
(App. G), and the effective variance of eq. G1:
  sigma_eff^2 = s^2 sigma^2 + (f_calib |m|)^2 + (f_data |d|)^2 + j^2.
Each term is switched on per observation; its parameter is sampled in log
space.  Reading: the natural log (App. G speaks of a uniform prior on ln f),
so s = exp(theta[log_err_scale]) and likewise for the others.
The mask is the user's mask AND finite data AND finite sigma AND sigma > 0
(App. H.1).
"""
import numpy as np


def inclusion_mask(data, sigma, user_mask=None):
    m = np.isfinite(data) & np.isfinite(sigma) & (sigma > 0)
    if user_mask is not None:
        m &= np.asarray(user_mask, dtype=bool)
    return m


def effective_variance(sigma, model, data, s=1.0, f_calib=None, f_data=None, jitter=None):
    v = (s * sigma) ** 2
    if f_calib is not None:
        v = v + (f_calib * np.abs(model)) ** 2
    if f_data is not None:
        v = v + (f_data * np.abs(data)) ** 2
    if jitter is not None:
        v = v + jitter ** 2
    return v


def lnlike(data, model, sigma, mask, s=1.0, f_calib=None, f_data=None, jitter=None):
    """sum_{i in mask} [ -(d_i - m_i)^2 / (2 v_i) - ln(2 pi v_i) / 2 ]."""
    d = np.where(mask, data, 0.0)
    sg = np.where(mask, sigma, 1.0)
    v = effective_variance(sg, model, d, s, f_calib, f_data, jitter)
    terms = -0.5 * (d - model) ** 2 / v - 0.5 * np.log(2.0 * np.pi * v)
    return float(np.sum(np.where(mask, terms, 0.0)))
