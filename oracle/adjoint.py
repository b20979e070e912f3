"""Hand-written reverse pass of the oracle forward model: d logL / d theta in FP64.

The paper's forward model is differentiable end to end and its samplers use the
exact gradient (Sec. 4, Sec. 4.3); this module writes that gradient out step by
step, in the reverse order of ``model``:

  logL (eq. 6, G1) -> model observables -> projection (App. E / App. F, including
  the redshift dependence of the interpolation, the LSF shift and the line
  positions) -> observer-frame scale (Sec. 2.6: 10^logmass, (1+z), D_L(z)) ->
  attenuation (eq. D2) -> contraction (eq. 1; the young and old spectra) ->
  line luminosities (eq. C2) -> SSP weights (App. B: bin masses, bin
  metallicities, [alpha/Fe], and the SFH edges through t_univ(z)).

At kinks (a filter node on a model pixel, a bin edge on a cell edge, a value on
a grid node) the one-sided derivative of the branch taken by the forward pass is
returned; clamped values have zero derivative.
"""
from __future__ import annotations

import math

import numpy as np

from . import cosmology, dust, nebular, projection, sfh
from .constants import ANG_CM, C_CMS, C_KMS, FNU_AB, FWHM_PER_SIGMA, LAM_V, LSUN
from .likelihood import inclusion_mask
from .model import columns, noise_terms


def _split_deriv(x, nodes):
    """(j, t, dt/dx) of sfh.grid_split, dt/dx = 0 when x is clamped."""
    j, t = sfh.grid_split(x, nodes)
    inside = nodes[0] <= x <= nodes[-1]
    return j, t, (1.0 / (nodes[j + 1] - nodes[j]) if inside else 0.0)


def _dsigma_inst_dlam(obs, lam_obs):
    """sigma_inst(lambda_obs) and its derivative in lambda_obs (eq. F2 per mode)."""
    v = np.asarray(obs.lsf_value, dtype=np.float64)
    if v.ndim == 0:
        val, dval = float(v), 0.0
    else:
        pw = obs.pix_wave
        if lam_obs <= pw[0] or lam_obs >= pw[-1]:
            val, dval = float(np.interp(lam_obs, pw, v)), 0.0
        else:
            k = int(np.searchsorted(pw, lam_obs, side="right")) - 1
            dval = (v[k + 1] - v[k]) / (pw[k + 1] - pw[k])
            val = v[k] + dval * (lam_obs - pw[k])
    f, c, m = FWHM_PER_SIGMA, C_KMS, obs.lsf_mode
    if m == "R_fwhm":
        return c / (f * val), -c * dval / (f * val * val)
    if m == "R_sigma":
        return c / val, -c * dval / (val * val)
    if m == "fwhm_aa":
        return c * val / (f * lam_obs), c / f * (dval / lam_obs - val / lam_obs ** 2)
    if m == "sigma_aa":
        return c * val / lam_obs, c * (dval / lam_obs - val / lam_obs ** 2)
    if m == "sigma_kms":
        return val, dval
    if m == "fwhm_kms":
        return val / f, dval / f
    raise ValueError(m)


def grad_point(L, obs, th, trunc=5.0):
    """(logL, d logL/d theta) for one parameter vector.

    Covers the model with the step SFH scheme, without the nebular continuum, an escape
    geometry or the IGM, with nebular-covered ages starting at the youngest SSP age."""
    if getattr(obs, "calib", None) or obs.kind == "lines":
        raise NotImplementedError("the adjoint covers neither the calibration polynomial nor line catalogues")
    if L.cont is not None or L.escape != "none" or L.neb_a0 != 0 or L.sfh_scheme != "step" or L.igm:
        raise NotImplementedError("the adjoint covers the step SFH scheme without the nebular continuum, "
                                  "f_ob or the IGM")
    cols = columns(L.n_sfh, L.n_zh)
    P = cols["P"]
    g = np.zeros(P)
    spec = obs.kind == "spec"
    n = L.n_sfh
    z = th[cols["zred"]]
    mass10 = 10.0 ** th[cols["logmass"]]
    tau_bc, alpha_bc = th[cols["tau_bc"]], th[cols["alpha_bc"]]
    tau_diff, delta = th[cols["tau_diff"]], th[cols["delta"]]

    # ------------------------------------------------------------------ forward
    t_univ = float(cosmology.age_of_universe_yr(z, L.H0, L.Om))
    dt_dz = float(cosmology.d_age_dz_yr(z, L.H0, L.Om))
    dl = float(cosmology.luminosity_distance_cm(z, L.H0, L.Om))
    ddl = float(cosmology.d_luminosity_distance_dz_cm(z, L.H0, L.Om))
    edges = sfh.sfh_edges(t_univ, n, L.T1)
    # dT_i/dz: T_i = T1 (t_univ/T1)^{(i-1)/(n-1)} for i >= 1
    dT = np.zeros(n + 1)
    for i in range(2, n + 1):
        dT[i] = edges[i] * ((i - 1) / (n - 1)) * dt_dz / t_univ
    masses = th[cols["sfh"]:cols["sfh"] + n]
    lo, hi = L.lo, L.hi
    Ti, Tj = edges[:-1, None], edges[1:, None]
    upper = np.minimum(hi[None, :], Tj)
    lower = np.maximum(lo[None, :], Ti)
    ov_raw = upper - lower
    ov = np.maximum(ov_raw, 0.0)
    dT_bin = (Tj - Ti)
    w = masses[:, None] * ov / dT_bin

    if L.n_zh:
        zh = th[cols["zh"]:cols["zh"] + L.n_zh]
        zeta = sfh.bin_metallicity_hist(zh, edges, L.T1, t_univ)
        # d zeta_i / d zh_k: the interpolation weights in ln T (clamped ends)
        node_t = np.geomspace(L.T1, t_univ, L.n_zh)
        centres = np.empty(n)
        centres[0] = 0.5 * L.T1
        centres[1:] = np.sqrt(edges[1:-1] * edges[2:])
        Jz = np.zeros((n, L.n_zh))
        for k in range(L.n_zh):
            e = np.zeros(L.n_zh)
            e[k] = 1.0
            Jz[:, k] = np.interp(np.log(centres), np.log(node_t), e)
    else:
        zeta = np.full(n, th[cols["logzsol"]])
    nz, na, nf = len(L.logz), len(L.ages), len(L.afe)
    zs = [_split_deriv(zeta[i], L.logz) if nz > 1 else (0, 0.0, 0.0) for i in range(n)]
    if nf > 1:
        ja, ta, dta = _split_deriv(th[cols["afe"]], L.afe)
        asplit = ((ja, 1.0 - ta, -dta), (ja + 1, ta, dta))
    else:
        asplit = ((0, 1.0, 0.0),)
    W = sfh.ssp_weights(w, zeta, L.logz, th[cols["afe"]], L.afe)

    lines_on = L.lines is not None
    if lines_on:
        zg, un = L.lines["zg_nodes"], L.lines["u_nodes"]
        tab = L.lines["line_table"]
        jg, tg, dtg = _split_deriv(th[cols["gas_logz"]], zg)
        ju, tu, dtu = _split_deriv(th[cols["gas_logu"]], un)
        lhat = nebular.line_table_interp(tab, zg, un, th[cols["gas_logz"]], th[cols["gas_logu"]])
        dlhat_dzg = ((1 - tu) * (tab[:, :, jg + 1, ju] - tab[:, :, jg, ju])
                     + tu * (tab[:, :, jg + 1, ju + 1] - tab[:, :, jg, ju + 1])) * dtg
        dlhat_du = ((1 - tg) * (tab[:, :, jg, ju + 1] - tab[:, :, jg, ju])
                    + tg * (tab[:, :, jg + 1, ju + 1] - tab[:, :, jg + 1, ju])) * dtu
        nn = L.n_neb
        WQ = (W[:, :, :nn] * L.Q[:, :, :nn]).sum(axis=(0, 1))
        E = 10.0 ** lhat                     # [n_line, n_neb]
        Lline = E @ WQ
    young = L.young
    f = L.flux                               # [af, z, age, wave]
    Wy = W * young[None, None, :]
    Wo = W * (~young)[None, None, :]
    Y = np.einsum("zma,zmaw->w", Wy, f)
    O = np.einsum("zma,zmaw->w", Wo, f)
    if lines_on and not spec:
        Y = Y + (Lline / LSUN) @ L.G
    wave = L.wave
    lnlv = np.log(wave / LAM_V)
    p_bc = np.exp(alpha_bc * lnlv)
    T_bc = np.exp(-tau_bc * p_bc)
    Eb = 0.85 - 1.9 * delta
    q = np.exp(delta * lnlv)
    shape = L.dust_a + Eb * L.dust_d
    T_d = np.exp(-tau_diff * q * shape)
    F = T_d * (T_bc * Y + O)

    # ------------------------------------------------------------------ projection
    opz = 1.0 + z
    gF = np.zeros_like(F)          # d logL / d F (rest frame, per A)
    gz = 0.0                        # direct d logL / d z
    if not spec:
        scale = mass10 * opz / (4.0 * math.pi * dl * dl)
        A = scale * LSUN / (opz * opz * ANG_CM)            # f_lambda^obs = A * F
        dlnA = -1.0 / opz - 2.0 * ddl / dl
        m = np.empty(len(obs.filters))
        rows = []
        for b, (lam, R) in enumerate(obs.filters):
            c = R * lam * projection.local_spacing(lam) / projection.ab_zero_point(lam, R)
            lr = lam / opz
            inside = (lr >= wave[0]) & (lr <= wave[-1])
            k = np.clip(np.searchsorted(wave, lr, side="right") - 1, 0, len(wave) - 2)
            t = (lr - wave[k]) / (wave[k + 1] - wave[k])
            interp = np.where(inside, (1 - t) * F[k] + t * F[k + 1], 0.0)
            m[b] = A * np.sum(c * interp)
            rows.append((c, inside, k, t, interp, lam))
    else:
        S = mass10 * opz / (4.0 * math.pi * dl * dl) * LSUN * ANG_CM / C_CMS   # F_nu^obs = S F lambda^2
        dlnS = 1.0 / opz - 2.0 * ddl / dl
        fnu = S * F * wave ** 2
        sig_k = projection.kernel_sigma_kms(obs.pix_wave, obs.lsf_mode, obs.lsf_value, wave, obs.z_ref,
                                            obs.sigma_gal_kms)
        ln_rest = np.log(wave)
        cont = np.zeros(len(obs.pix_wave))
        dcont_dz = np.zeros(len(obs.pix_wave))
        lsf = []
        for i, (lam, sk) in enumerate(zip(obs.pix_wave, sig_k)):
            x = math.log(lam) - math.log1p(z)
            s = sk / C_KMS
            if x < ln_rest[0] or x > ln_rest[-1]:
                lsf.append(None)
                continue
            k = min(max(int(np.searchsorted(ln_rest, x, side="right")) - 1, 0), len(wave) - 2)
            dk = ln_rest[k + 1] - ln_rest[k]
            if s < 0.5 * dk:
                t = (x - ln_rest[k]) / dk
                idx = np.array([k, k + 1])
                wts = np.array([1 - t, t])
                cont[i] = wts @ fnu[idx]
                dcont_dz[i] = (fnu[k + 1] - fnu[k]) * (-1.0 / (opz * dk))
            else:
                idx = np.nonzero(np.abs(ln_rest - x) <= trunc * s)[0]
                u = (ln_rest[idx] - x) / s
                gg = np.exp(-0.5 * u * u)
                G = gg.sum()
                wts = gg / G
                cont[i] = wts @ fnu[idx]
                dg = -u * gg / (s * opz)                  # d g / d z
                dcont_dz[i] = np.sum(dg * (fnu[idx] - cont[i])) / G
            lsf.append((idx, wts))
        m = cont.copy()
        if lines_on:
            lw = L.lines["line_wave"]
            lnl = np.log(lw / LAM_V)
            a_l = np.interp(lw, wave, L.dust_a)
            d_l = np.interp(lw, wave, L.dust_d)
            p_l = np.exp(alpha_bc * lnl)
            q_l = np.exp(delta * lnl)
            T_l = np.exp(-tau_bc * p_l - tau_diff * q_l * (a_l + Eb * d_l))
            Kf = mass10 / (4.0 * math.pi * dl * dl)
            Fl = Lline * T_l * Kf
            lobs = opz * lw
            si = np.empty(len(lw))
            dsi = np.empty(len(lw))
            for l in range(len(lw)):
                si[l], dsi[l] = _dsigma_inst_dlam(obs, lobs[l])
            s_l = np.sqrt(obs.sigma_gas_kms ** 2 + si ** 2) / C_KMS
            ds_l_dz = si * dsi * lw / (C_KMS ** 2 * s_l)
            lnp = np.log(obs.pix_wave)[:, None]
            mu = np.log(lobs)[None, :]
            uu = (lnp - mu) / s_l[None, :]
            Nn = np.exp(-0.5 * uu * uu) / (math.sqrt(2 * math.pi) * s_l[None, :])
            pref = obs.pix_wave * ANG_CM / C_CMS
            m = m + pref * (Nn @ Fl)
        m = m / FNU_AB

    # ------------------------------------------------------------------ logL and dlogL/dm
    mask = inclusion_mask(obs.data, obs.sigma, obs.mask)
    s_, fc, fd, jt = noise_terms(obs, th, cols)
    d = np.where(mask, obs.data, 0.0)
    sg = np.where(mask, obs.sigma, 1.0)
    v = (s_ * sg) ** 2
    if fc is not None:
        v = v + (fc * m) ** 2
    if fd is not None:
        v = v + (fd * d) ** 2
    if jt is not None:
        v = v + jt ** 2
    r = d - m
    terms = -0.5 * r * r / v - 0.5 * np.log(2 * math.pi * v)
    logl = float(np.sum(np.where(mask, terms, 0.0)))
    dv = np.where(mask, 0.5 * r * r / v ** 2 - 0.5 / v, 0.0)
    gm = np.where(mask, r / v, 0.0)
    if fc is not None:
        gm = gm + dv * 2.0 * fc * fc * m
        g[cols["log_f_calib"]] = np.sum(dv * 2.0 * (fc * m) ** 2)
    if obs.noise and obs.noise.get("err_scale"):
        g[cols["log_err_scale"]] = np.sum(dv * 2.0 * (s_ * sg) ** 2)
    if fd is not None:
        g[cols["log_f_data"]] = np.sum(dv * 2.0 * (fd * d) ** 2)
    if jt is not None:
        g[cols["log_jitter"]] = np.sum(dv * 2.0 * jt * jt)
    # every model output is proportional to 10^logmass
    g[cols["logmass"]] = math.log(10.0) * np.sum(gm * m)

    # ------------------------------------------------------------------ projection adjoint
    gLline = np.zeros(0 if not lines_on else len(Lline))
    if not spec:
        for b, (c, inside, k, t, interp, lam) in enumerate(rows):
            gb = gm[b] * A
            np.add.at(gF, k[inside], gb * c[inside] * (1 - t[inside]))
            np.add.at(gF, k[inside] + 1, gb * c[inside] * t[inside])
            slope = np.where(inside, (F[k + 1] - F[k]) / (wave[k + 1] - wave[k]), 0.0)
            gz += gm[b] * (dlnA * m[b] + A * np.sum(c * slope * (-lam / opz ** 2)))
    else:
        gc = gm / FNU_AB                       # d logL / d cont_i
        gfnu = np.zeros_like(fnu)
        for i, row in enumerate(lsf):
            if row is None:
                continue
            idx, wts = row
            gfnu[idx] += gc[i] * wts
        gF += gfnu * S * wave ** 2
        gz += np.sum(gc * (dlnS * cont + dcont_dz))
        if lines_on:
            gl_pix = gc * pref                          # d logL / d (sum_l F_l N_il)
            gFl = Nn.T @ gl_pix                         # d logL / d F_l
            dN_dmu = Nn * uu / s_l[None, :]
            dN_ds = Nn * (uu * uu - 1.0) / s_l[None, :]
            gz += np.sum(gl_pix[:, None] * Fl[None, :] * (dN_dmu / opz + dN_ds * ds_l_dz[None, :]))
            gz += np.sum(gFl * Fl) * (-2.0 * ddl / dl)
            gLline = gFl * T_l * Kf
            g[cols["tau_bc"]] += np.sum(gFl * Fl * (-p_l))
            g[cols["alpha_bc"]] += np.sum(gFl * Fl * (-tau_bc * p_l * lnl))
            g[cols["tau_diff"]] += np.sum(gFl * Fl * (-q_l * (a_l + Eb * d_l)))
            g[cols["delta"]] += np.sum(gFl * Fl * (-tau_diff * (q_l * lnl * (a_l + Eb * d_l) - 1.9 * q_l * d_l)))

    # ------------------------------------------------------------------ attenuation adjoint
    gY = gF * T_d * T_bc
    gO = gF * T_d
    g[cols["tau_bc"]] += np.sum(gF * T_d * Y * T_bc * (-p_bc))
    g[cols["alpha_bc"]] += np.sum(gF * T_d * Y * T_bc * (-tau_bc * p_bc * lnlv))
    g[cols["tau_diff"]] += np.sum(gF * F * (-q * shape))
    g[cols["delta"]] += np.sum(gF * F * (-tau_diff * (q * lnlv * shape - 1.9 * q * L.dust_d)))

    # ------------------------------------------------------------------ contraction adjoint
    gW = (np.einsum("w,zmaw->zma", gY, f) * young[None, None, :]
          + np.einsum("w,zmaw->zma", gO, f) * (~young)[None, None, :])
    if lines_on and not spec:
        gLline = gLline + (L.G @ gY) / LSUN

    # ------------------------------------------------------------------ line luminosities adjoint
    if lines_on:
        nn = L.n_neb
        gWQ = E.T @ gLline                                  # [n_neb]
        gW[:, :, :nn] += gWQ[None, None, :] * L.Q[:, :, :nn]
        gE = np.outer(gLline, WQ)                           # d/d E_la
        ln10 = math.log(10.0)
        g[cols["gas_logz"]] += np.sum(gE * E * ln10 * dlhat_dzg)
        g[cols["gas_logu"]] += np.sum(gE * E * ln10 * dlhat_du)

    # ------------------------------------------------------------------ weights adjoint
    gw = np.zeros((n, na))                  # d logL / d w_ia
    gzeta = np.zeros(n)
    for i in range(n):
        j, t, dtz = zs[i]
        for ia, fa, dfa in asplit:
            if nz > 1:
                gw[i] += fa * ((1 - t) * gW[ia, j] + t * gW[ia, j + 1])
                gzeta[i] += fa * dtz * np.sum(w[i] * (gW[ia, j + 1] - gW[ia, j]))
                if nf > 1:
                    g[cols["afe"]] += dfa * np.sum(w[i] * ((1 - t) * gW[ia, j] + t * gW[ia, j + 1]))
            else:
                gw[i] += fa * gW[ia, 0]
                if nf > 1:
                    g[cols["afe"]] += dfa * np.sum(w[i] * gW[ia, 0])
    # bin masses
    g[cols["sfh"]:cols["sfh"] + n] = np.sum(gw * ov / dT_bin, axis=1)
    # metallicity parameters
    if L.n_zh:
        g[cols["zh"]:cols["zh"] + L.n_zh] = gzeta @ Jz
    else:
        g[cols["logzsol"]] = np.sum(gzeta)
    # edges -> z: d w_ia / d T_i and d T_{i+1}
    pos = ov_raw > 0
    dov_dTi = np.where(pos & (Ti > lo[None, :]), -1.0, 0.0)
    dov_dTj = np.where(pos & (Tj < hi[None, :]), 1.0, 0.0)
    dw_dTi = masses[:, None] * (dov_dTi / dT_bin + ov / dT_bin ** 2)
    dw_dTj = masses[:, None] * (dov_dTj / dT_bin - ov / dT_bin ** 2)
    gz += np.sum(gw * (dw_dTi * dT[:-1, None] + dw_dTj * dT[1:, None]))
    g[cols["zred"]] += gz
    return logl, g


def logl_grad(L, obs, theta, trunc=5.0):
    """logL [B] and d logL / d theta [B, P]."""
    theta = np.atleast_2d(theta)
    out_l = np.empty(theta.shape[0])
    out_g = np.empty_like(theta)
    for b in range(theta.shape[0]):
        out_l[b], out_g[b] = grad_point(L, obs, theta[b], trunc)
    return out_l, out_g
