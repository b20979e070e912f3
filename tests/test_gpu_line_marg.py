"""GPU parity for the analytic marginalisation of a spectrum's line fluxes (Sec. 4.1,
App. I.3, eq. app_line_marg), against the FP64 oracle on the same seeded inputs, through the
C ABI:

  - a 300-pixel spectrum whose data carry the lines at fluxes off the grid's (scaled by
    U(0.5, 1.8) per line) plus noise, fitted with Gaussian priors around the grid fluxes
    (two lines flagged flat) or with every line flat, with and without the noise-floor
    terms, at redshifts that move lines in and out of the pixel range;
  - a batch over several M tiles with a ragged tail at FP64, FP32 and FP16 (three passes);
  - the gradient, the allocation-free call and a calibration polynomial at the same time
    are refused; more than 128 lines within the pixel range is SPS_E_SHAPE;
  - the joint marginalisation over the spectrum, a line catalogue and 20-band photometry of
    the same object (sps_logl_lines_joint): single lines and blends, lines inside and
    outside the pixel range (fitted through the catalogue alone), two upper limits and a
    masked entry, a masked band, with Gaussian priors (two lines flat) and with every line
    flat (single-line entries: a flat line seen only in a blend is not identified and its
    marginal diverges); spectrum + catalogue, spectrum + photometry, and all three.

Tolerances: logL FP64 1e-10, FP32 and FP16 1e-4, relative to the larger of the marginal
and the grid-model likelihood (the marginal likelihood is a difference of terms of that
size), and FP16 |dlogL| <= 0.05 within reach of the data.
"""
import dataclasses
import sys

import numpy as np
import pytest

from helpers import gpu_objects, make_case, near_truth
from oracle import model as om
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402

CFG = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=16, n_zh=5,
                 n_lines=24, n_pix=300)
PRECS = ("fp64", "fp32", "fp16")
LOGL_TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16": 1e-4}
B = 200


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    c = make_case(CFG, B=B, kind="spec", noise=("err_scale", "jitter"))
    obs = c["obs"]
    olib = c["olib"]
    cols = om.lib_columns(olib)
    # the data: the grid model at theta_true with every line's flux scaled, plus noise
    th_t = c["theta_true"]
    m_true = om.predict(olib, obs, th_t)[0]
    rf = om.rest_frame(olib, th_t, lines_on_grid=False)
    probe = dataclasses.replace(obs, line_marg="flat")
    t = om.line_marg_terms(olib, probe, th_t[0], cols, rf["Lline"][0])
    scale = np.random.default_rng(41).uniform(0.5, 1.8, len(t["idx"]))
    rng = np.random.default_rng(43)
    obs.data = m_true + t["A"] @ ((scale - 1.0) * t["alpha_bar"]) + obs.sigma * rng.normal(size=m_true.size)
    L, _ = gpu_objects(c, precisions=("fp64", "fp32", "fp16"), max_batch=256)
    theta = np.concatenate([c["theta"][:B - 24], near_truth(c["cfg"], th_t, 24, 61)])
    theta[:4, 1] = [0.8, 2.0, 4.5, 7.0]
    return c, L, theta


def spec_obs(L, obs, max_batch, noise=(), **kw):
    return sps.Observation(L, "spec", max_batch, pix_wave=obs.pix_wave, lsf_mode=obs.lsf_mode,
                           lsf_value=obs.lsf_value, z_ref=obs.z_ref, sigma_gal_kms=obs.sigma_gal_kms,
                           sigma_gas_kms=obs.sigma_gas_kms, data=obs.data, sigma=obs.sigma, mask=obs.mask,
                           noise=noise, **kw)


MODES = [("gauss", 0.3, True, ()), ("gauss", 1.0, False, ("err_scale", "jitter")), ("flat", 0.0, False, ())]


@pytest.mark.parametrize("mode,frac,some_flat,noise", MODES)
def test_line_marginal_likelihood(case, mode, frac, some_flat, noise):
    c, L, theta = case
    obs = c["obs"]
    th = theta.copy()
    cols = om.lib_columns(c["olib"])
    if noise:
        th[:, cols["log_err_scale"]] = np.log(1.2)
        th[:, cols["log_jitter"]] = np.log(0.3 * np.median(obs.sigma))
    flat = np.zeros(CFG.n_lines, dtype=bool)
    if some_flat:
        flat[[5, 17]] = True
    oobs = dataclasses.replace(obs, noise={n: True for n in noise}, line_marg=mode, line_prior_frac=frac,
                               line_flat=flat if some_flat else None)
    ref_m = om.predict(c["olib"], oobs, th)
    ref_ll = om.logl(c["olib"], oobs, th, model=ref_m)
    plain = om.logl(c["olib"], dataclasses.replace(oobs, line_marg=None), th, model=ref_m)
    assert np.max(np.abs(ref_ll - plain)) > 1.0
    near = np.mean(((obs.data - ref_m) / obs.sigma) ** 2, axis=1) <= 100
    O = spec_obs(L, obs, 256, noise=noise, line_marg=mode, line_prior_frac=frac,
                 line_flat=flat if some_flat else None)
    for prec in PRECS:
        say(f"  line marginalisation {mode} frac {frac} flat {some_flat} noise {noise} {prec}")
        tt = torch.tensor(th, dtype=torch.float64, device="cuda")
        ll, m = sps.logl(L, O, tt, prec, return_model=True)
        torch.cuda.synchronize()
        ll = ll.cpu().numpy()
        scale = np.maximum(1.0, np.maximum(np.abs(ref_ll), np.abs(plain)))
        lle = np.abs(ll - ref_ll) / scale
        dnear = np.abs(ll - ref_ll)[near].max() if near.any() else 0.0
        say(f"    logL rel err {lle.max():.3e}; |dlogL| ({near.sum()} rows) {dnear:.3e}")
        assert np.all(np.isfinite(ll))
        assert lle.max() < LOGL_TOL[prec]
        if prec == "fp16":
            assert dnear <= 0.05


def test_refusals_and_size_limit(case):
    c, L, theta = case
    obs = c["obs"]
    O = spec_obs(L, obs, 16, line_marg="gauss", line_prior_frac=0.3)
    th = torch.tensor(theta[:8], dtype=torch.float64, device="cuda")
    for fn in (sps.logl_grad, sps.logl_static):
        with pytest.raises(sps.SpsError) as ei:
            fn(L, O, th, "fp32")
        assert ei.value.code == -1
    with pytest.raises(sps.SpsError) as ei:
        spec_obs(L, obs, 16, line_marg="gauss", line_prior_frac=0.3, calib="marginal", calib_order=1,
                 calib_prior=np.full(2, 0.1))
    assert ei.value.code == -1
    with pytest.raises(sps.SpsError) as ei:
        spec_obs(L, obs, 16, line_marg="gauss", line_prior_frac=0.0)
    assert ei.value.code == -1
    # 160 library lines drawn log-uniform over 1000 A - 2 um: a pixel range of 0.3 - 5.3 um
    # holds up to 157 of them at some redshift (more than 128), 1.0 - 5.3 um up to 96
    cfg = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=(-2.0, -1.0, 0.0), n_wave=1500, n_sfh=8, n_zh=0,
                     n_lines=160, n_pix=300)
    c2 = make_case(cfg, B=4, kind="spec")
    L2, _ = gpu_objects(c2, precisions=("fp32",), max_batch=8)
    pw = np.geomspace(3000.0, 53000.0, 300)
    with pytest.raises(sps.SpsError) as ei:
        sps.Observation(L2, "spec", 8, pix_wave=pw, lsf_mode="R_fwhm", lsf_value=100.0, line_marg="flat")
    assert ei.value.code == -2
    sps.Observation(L2, "spec", 8, pix_wave=np.geomspace(10000.0, 53000.0, 300), lsf_mode="R_fwhm",
                    lsf_value=100.0, line_marg="flat")


# catalogue entries over the 24 library lines: single lines, blends, lines that the
# spectrum's pixel range holds at some redshifts and not at others
JOINT_BLENDS = [[0], [3], [5, 6], [8], [10, 11, 12], [14], [17], [19, 20], [22], [23]]
# with every line flat, lines that only a blend sees are not identified one by one (the
# marginal likelihood of a flat prior diverges): single lines only
JOINT_SINGLES = [[0], [3], [5], [8], [10], [14], [17], [19], [22], [23]]


def cat_obs(case, blends, seed=29):
    olib = case["olib"]
    upper = np.zeros(len(blends), dtype=bool)
    upper[[3, 8]] = True
    lobs = om.Lines(blends=blends, upper=upper)
    f_true = om.predict(olib, lobs, case["theta_true"])[0]
    rng = np.random.default_rng(seed)
    lobs.sigma = 0.1 * f_true + 1e-25
    lobs.data = f_true * rng.uniform(0.6, 1.5, f_true.size) + lobs.sigma * rng.normal(size=f_true.size)
    lobs.data[upper] = 2.0 * lobs.sigma[upper]
    lobs.mask = np.ones(len(blends), dtype=bool)
    lobs.mask[6] = False
    return lobs


def phot_obs(case, seed=31):
    pobs = om.Photometry(filters=wl.make_filters("gauss20"))
    m_true = om.predict(case["olib"], pobs, case["theta_true"])[0]
    pobs.data, pobs.sigma = wl.noisy_photometry(m_true, seed)
    pobs.mask = np.ones(m_true.size, dtype=bool)
    pobs.mask[4] = False
    return pobs


@pytest.mark.parametrize("mode,frac,some_flat,with_cat,with_phot", [
    ("gauss", 0.3, True, True, False), ("flat", 0.0, False, True, False),
    ("gauss", 0.3, True, True, True), ("gauss", 0.3, False, False, True), ("flat", 0.0, False, True, True)])
def test_joint_with_a_line_catalogue(case, mode, frac, some_flat, with_cat, with_phot):
    c, L, theta = case
    obs = c["obs"]
    blends = JOINT_BLENDS if mode == "gauss" else JOINT_SINGLES
    lobs = cat_obs(c, blends) if with_cat else None
    pobs = phot_obs(c) if with_phot else None
    flat = np.zeros(CFG.n_lines, dtype=bool)
    if some_flat:
        flat[[5, 17]] = True
    sobs = dataclasses.replace(obs, noise={}, line_marg=mode, line_prior_frac=frac,
                               line_flat=flat if some_flat else None)
    ref = om.logl_lines_joint(c["olib"], sobs, lobs, theta, phot=pobs)
    alone = om.logl(c["olib"], sobs, theta)
    if lobs is not None:
        alone = alone + om.logl(c["olib"], lobs, theta)
    if pobs is not None:
        alone = alone + om.logl(c["olib"], pobs, theta)
    assert np.all(np.isfinite(ref)) and np.max(np.abs(ref - alone)) > 1.0
    O = spec_obs(L, obs, 256, line_marg=mode, line_prior_frac=frac, line_flat=flat if some_flat else None)
    Oc = sps.Observation(L, "lines", 256, blends=blends, upper=lobs.upper, data=lobs.data, sigma=lobs.sigma,
                         mask=lobs.mask) if lobs is not None else None
    Op = sps.Observation(L, "phot", 256, filters=pobs.filters, data=pobs.data, sigma=pobs.sigma,
                         mask=pobs.mask) if pobs is not None else None
    tt = torch.tensor(theta, dtype=torch.float64, device="cuda")
    scale = np.maximum(1.0, np.maximum(np.abs(ref), np.abs(alone)))
    for prec in PRECS:
        say(f"  joint {mode} flat {some_flat} catalogue {with_cat} photometry {with_phot} {prec}")
        ll = sps.logl_lines_joint(L, O, tt, cat=Oc, phot=Op, precision=prec)
        torch.cuda.synchronize()
        ll = ll.cpu().numpy()
        lle = np.abs(ll - ref) / scale
        say(f"    logL rel err {lle.max():.3e}")
        assert np.all(np.isfinite(ll))
        assert lle.max() < LOGL_TOL[prec]
    with pytest.raises(sps.SpsError) as ei:   # the observations in the wrong places
        sps.logl_lines_joint(L, Oc if Oc is not None else Op, tt, cat=O, precision="fp32")
    assert ei.value.code == -1
