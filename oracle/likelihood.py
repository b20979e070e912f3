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


# ---------------------------------------------------------------------------------
# Spectrophotometric calibration polynomial (Sec. 3.2, App. H.3, eq. app_polymarg)
# ---------------------------------------------------------------------------------
def chebyshev_design(pix_wave, order):
    """A[i, m] = T_m(x_i), x the pixel wavelengths mapped linearly onto [-1, 1] (reading:
    the first and last pixel of the observation map to -1 and +1)."""
    lam = np.asarray(pix_wave, dtype=np.float64)
    x = 2.0 * (lam - lam[0]) / (lam[-1] - lam[0]) - 1.0
    return np.polynomial.chebyshev.chebvander(x, order)


def calibrated_lnlike(data, model, sigma, mask, A, prior_sd, mode, s=1.0, f_calib=None, f_data=None,
                      jitter=None):
    """The calibrated model mu (1 + sum_m c_m T_m(x)): the residual r = d - mu is linear in c,
    r = D c + n, D = diag(mu) A, n ~ N(0, C), C = diag(sigma_eff^2) at the uncalibrated model,
    prior c ~ N(0, diag(s_m^2)); with M = D^T C^-1 D + diag(s_m^-2) and b = D^T C^-1 r:

      mode "marginal" (eq. app_polymarg): lnL_diag(r) + b^T M^-1 b / 2 - ln|M| / 2 - ln|Lambda| / 2;
      mode "optimise": lnL_diag(r - D c_hat) at the regularised best fit c_hat = M^-1 b
      (Sec. 3.2: the polynomial optimised at each evaluation, with regularisation 1/s_m).
    """
    d = np.where(mask, data, 0.0)
    sg = np.where(mask, sigma, 1.0)
    v = effective_variance(sg, model, d, s, f_calib, f_data, jitter)
    r = np.where(mask, d - model, 0.0)
    iv = np.where(mask, 1.0 / v, 0.0)
    D = model[:, None] * A
    Mm = D.T @ (iv[:, None] * D) + np.diag(1.0 / np.asarray(prior_sd, dtype=np.float64) ** 2)
    b = D.T @ (iv * r)
    chat = np.linalg.solve(Mm, b)
    if mode == "marginal":
        base = lnlike(data, model, sigma, mask, s, f_calib, f_data, jitter)
        _, logdet = np.linalg.slogdet(Mm)
        return base + 0.5 * b @ chat - 0.5 * logdet - np.sum(np.log(prior_sd))
    if mode == "optimise":
        res = r - D @ chat
        terms = -0.5 * res ** 2 * iv - 0.5 * np.log(2.0 * np.pi * v)
        return float(np.sum(np.where(mask, terms, 0.0)))
    raise ValueError(mode)


# ---------------------------------------------------------------------------------
# Emission-line catalogues (App. I.2, eq. app_line_chi2_det / app_line_chi2_UL)
# ---------------------------------------------------------------------------------
def lines_lnlike(data, model, sigma, mask, upper):
    """-chi^2 / 2 over the mask: detections ((d - m)/sigma)^2; upper limits the same when the
    model exceeds the limit, else 0.  Reading: the noise floor and the normalisation term
    do not enter (App. I.2 adds -chi^2_lines / 2)."""
    d = np.where(mask, data, 0.0)
    sg = np.where(mask, sigma, 1.0)
    chi2 = ((d - model) / sg) ** 2
    chi2 = np.where(upper & (model <= d), 0.0, chi2)
    return float(-0.5 * np.sum(np.where(mask, chi2, 0.0)))


# ---------------------------------------------------------------------------------
# Analytic marginalisation of line fluxes (Sec. 4.1, App. I.3, eq. app_line_marg)
# ---------------------------------------------------------------------------------
def line_marginal_lnlike(data, model, sigma, mask, A, alpha_bar, prior_sd, flat, s=1.0, f_calib=None,
                         f_data=None, jitter=None, return_mean=False):
    """The data are linear in the fitted line fluxes alpha: d = mu + A alpha + n.  ``model`` is
    the full model at the grid fluxes alpha_bar (mu + A alpha_bar), A[i, j] the unit-flux
    profile of line j on pixel i, n ~ N(0, diag(sigma_eff^2)) with sigma_eff at that model.
    Line j takes a Gaussian prior N(alpha_bar_j, prior_sd_j^2), or a flat prior where
    flat[j] (its grid flux then does not enter the residual).  With r = d - mu - A alpha_0
    (alpha_0 = alpha_bar, 0 on flat lines), b = A^T W r, P = A^T W A + diag(prior_sd^-2) over
    the Gaussian lines:

      ln Z = lnL_diag(r) + b^T P^-1 b / 2 - ln|P| / 2 - sum_G ln s_j + (m_flat / 2) ln(2 pi),

    and the fluxes given theta are Gaussian with mean alpha_0 + P^-1 b (returned as well
    with ``return_mean``)."""
    A = np.asarray(A, dtype=np.float64)
    flat = np.asarray(flat, dtype=bool)
    alpha_bar = np.asarray(alpha_bar, dtype=np.float64)
    prior_sd = np.asarray(prior_sd, dtype=np.float64)
    d = np.where(mask, data, 0.0)
    sg = np.where(mask, sigma, 1.0)
    v = effective_variance(sg, model, d, s, f_calib, f_data, jitter)
    iv = np.where(mask, 1.0 / v, 0.0)
    alpha0 = np.where(flat, 0.0, alpha_bar)
    resid_model = model - A @ np.where(flat, alpha_bar, 0.0)      # mu + A alpha_0
    r = np.where(mask, d - resid_model, 0.0)
    base = float(np.sum(np.where(mask, -0.5 * r * r * iv - 0.5 * np.log(2.0 * np.pi * np.where(mask, v, 1.0)), 0.0)))
    b = A.T @ (iv * r)
    P = A.T @ (iv[:, None] * A) + np.diag(np.where(flat, 0.0, 1.0 / np.where(flat, 1.0, prior_sd) ** 2))
    x = np.linalg.solve(P, b)
    _, logdet = np.linalg.slogdet(P)
    lnz = base + 0.5 * b @ x - 0.5 * logdet - np.sum(np.log(prior_sd[~flat])) \
        + 0.5 * np.count_nonzero(flat) * np.log(2.0 * np.pi)
    return (lnz, alpha0 + x) if return_mean else lnz


def joint_line_marginal_lnlike(spec, cat, alpha_bar, prior_sd, flat, return_mean=False, phot=None):
    """Eq. app_line_marg over two observations that see the same fitted lines: a spectrum
    ``spec`` = dict(data, model, sigma, mask, A, s, f_calib, f_data, jitter) (A[i, j] the
    unit-flux profile of line j on pixel i, noise floor as in eq. G1) and a line catalogue
    ``cat`` = dict(data, model, sigma, mask, upper, A) (A[e, j] = 1 where fitted line j is in
    entry e's blend).  Each model is the full one at the grid fluxes; lnL_diag of the
    catalogue is its own -chi^2 / 2 (no normalisation term, App. I.2).  Reading: upper-limit
    entries are not Gaussian in the fluxes and keep their one-sided chi^2 at the grid model;
    only detections enter the sums.  ``phot`` (or None) = dict(data, model, sigma, mask, A,
    s, f_calib, f_data, jitter): photometry, A[b, j] the band response of fitted line j per
    unit flux, its lnL_diag the normalised Gaussian of eq. 6 with the noise floor of eq. G1
    at its model.  With r_k = d_k - mu_k - A_k alpha_0, b = sum_k A_k^T W_k
    r_k and P = sum_k A_k^T W_k A_k + diag(s^-2) over the Gaussian lines,

      ln Z = sum_k lnL_diag,k(r_k) + b^T P^-1 b / 2 - ln|P| / 2 - sum_G ln s_j + (m_flat / 2) ln 2 pi."""
    flat = np.asarray(flat, dtype=bool)
    alpha_bar = np.asarray(alpha_bar, dtype=np.float64)
    prior_sd = np.asarray(prior_sd, dtype=np.float64)
    alpha0 = np.where(flat, 0.0, alpha_bar)
    shift = np.where(flat, alpha_bar, 0.0)          # the grid flux of flat lines leaves mu + A alpha_0
    As = np.asarray(spec["A"], dtype=np.float64)
    ms = spec["mask"]
    d = np.where(ms, spec["data"], 0.0)
    sg = np.where(ms, spec["sigma"], 1.0)
    v = effective_variance(sg, spec["model"], d, spec.get("s", 1.0), spec.get("f_calib"), spec.get("f_data"),
                           spec.get("jitter"))
    iv = np.where(ms, 1.0 / v, 0.0)
    r = np.where(ms, d - (spec["model"] - As @ shift), 0.0)
    base = float(np.sum(np.where(ms, -0.5 * r * r * iv - 0.5 * np.log(2.0 * np.pi * np.where(ms, v, 1.0)), 0.0)))
    b = As.T @ (iv * r)
    P = As.T @ (iv[:, None] * As)
    if cat is not None:
        Ac = np.asarray(cat["A"], dtype=np.float64)
        mc = cat["mask"]
        up = np.asarray(cat["upper"], dtype=bool)
        det = mc & ~up
        dc = np.where(mc, cat["data"], 0.0)
        sc = np.where(mc, cat["sigma"], 1.0)
        rc = np.where(det, dc - (cat["model"] - Ac @ shift), 0.0)
        wc = np.where(det, 1.0 / sc ** 2, 0.0)
        base += float(-0.5 * np.sum(wc * rc * rc))
        ul = mc & up & (cat["model"] > dc)
        base += float(-0.5 * np.sum(np.where(ul, ((dc - cat["model"]) / sc) ** 2, 0.0)))
        b = b + Ac.T @ (wc * rc)
        P = P + Ac.T @ (wc[:, None] * Ac)
    if phot is not None:
        Ap = np.asarray(phot["A"], dtype=np.float64)
        mp = phot["mask"]
        dp = np.where(mp, phot["data"], 0.0)
        sgp = np.where(mp, phot["sigma"], 1.0)
        vp = effective_variance(sgp, phot["model"], dp, phot.get("s", 1.0), phot.get("f_calib"), phot.get("f_data"),
                                phot.get("jitter"))
        ivp = np.where(mp, 1.0 / vp, 0.0)
        rp = np.where(mp, dp - (phot["model"] - Ap @ shift), 0.0)
        base += float(np.sum(np.where(mp, -0.5 * rp * rp * ivp - 0.5 * np.log(2.0 * np.pi * np.where(mp, vp, 1.0)),
                                      0.0)))
        b = b + Ap.T @ (ivp * rp)
        P = P + Ap.T @ (ivp[:, None] * Ap)
    P = P + np.diag(np.where(flat, 0.0, 1.0 / np.where(flat, 1.0, prior_sd) ** 2))
    if len(flat) == 0:
        return (base, alpha0) if return_mean else base
    x = np.linalg.solve(P, b)
    _, logdet = np.linalg.slogdet(P)
    lnz = base + 0.5 * b @ x - 0.5 * logdet - np.sum(np.log(prior_sd[~flat])) \
        + 0.5 * np.count_nonzero(flat) * np.log(2.0 * np.pi)
    return (lnz, alpha0 + x) if return_mean else lnz
