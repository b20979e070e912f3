"""GPU parity for observation paths beyond the default configurations, each against the
FP64 oracle on the same seeded inputs:

  - the inclusion mask: a user mask, non-finite data and sigma <= 0 entries, on photometry
    and on a spectrum (eq. 6 summed over the mask, App. H.1), forward and gradient;
  - a fixed stellar dispersion sigma_gal = 200 km/s folded into the continuum kernel (eq. 5);
  - the LSF conventions of eq. F2 other than R_fwhm: FWHM in Angstrom, sigma in km/s, and an
    R_fwhm curve tabulated on the pixels;
  - all four noise-floor terms of eq. G1 on a spectrum, forward and gradient;
  - constant metallicity and [alpha/Fe] outside the grid (clamped, App. B);
  - a redshift that is not a number in one row of a batch after a larger batch: its own
    row is non-finite, every other row is unchanged and nothing is written past B.

Tolerances (per-output relative error, floored at 1e-6 of the datum's sigma): FP64 1e-12
(spectra 1e-11); FP32 1e-5; FP16 hi + residual (3 passes) 2e-3.  logL: FP64 1e-10
relative; FP32 and FP16 1e-4 relative, and FP16 |dlogL| <= 0.05 where chi^2 per datum
<= 100.  Gradients: per component |dg| <= tol |g| + 1e-2 tol S_p + 10 n_p, S_p from
helpers.grad_scale and n_p the rounding-noise estimate of helpers.grad_noise (x 2^-29 for
FP64); tol 1e-9 (FP64), 1e-4 (FP32).
"""
import ctypes as C
import sys

import numpy as np
import pytest

from helpers import gpu_objects, grad_noise, grad_ratio, grad_scale, make_case, model_err, near_truth, rel_err, worst_entries
from oracle import adjoint
from oracle import model as om
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402

CFG_PHOT = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=30,
                      n_zh=6, n_lines=24)
CFG_SPEC = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=16,
                      n_zh=5, n_lines=24, n_pix=300)
MODEL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 2e-3}
LOGL_TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16": 1e-4}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def batch(case, n_prior=24, n_near=24, seed=61):
    th_near = near_truth(case["cfg"], case["theta_true"], n_near, seed)
    return np.concatenate([case["theta"][:n_prior], th_near])


def check_forward(tag, case, L, O, theta, precs, spec=False):
    ref_m = om.predict(case["olib"], case["obs"], theta)
    ref_ll = om.logl(case["olib"], case["obs"], theta, model=ref_m)
    mask = np.isfinite(case["obs"].data) & np.isfinite(case["obs"].sigma) & (case["obs"].sigma > 0)
    if case["obs"].mask is not None:
        mask &= np.asarray(case["obs"].mask, dtype=bool)
    chi2 = np.sum(np.where(mask, ((case["obs"].data - ref_m) / np.where(mask, case["obs"].sigma, 1.0)) ** 2, 0.0),
                  axis=1) / max(1, mask.sum())
    for prec in precs:
        th = torch.tensor(theta, dtype=torch.float64, device="cuda")
        ll, m = sps.logl(L, O, th, prec, return_model=True)
        torch.cuda.synchronize()
        ll, m = ll.cpu().numpy(), m.cpu().numpy()
        e = model_err(m, ref_m, case["obs"].sigma)
        lle = np.abs(ll - ref_ll) / np.maximum(1.0, np.abs(ref_ll))
        near = chi2 <= 100
        dnear = np.abs(ll - ref_ll)[near].max() if near.any() else 0.0
        say(f"  {tag} {prec}: model max rel err {e.max():.3e}; logL rel err {lle.max():.3e}; "
            f"|dlogL| near data ({near.sum()} rows) {dnear:.3e}")
        mt = MODEL_TOL[prec] * (10 if (spec and prec == "fp64") else 1)
        if e.max() >= mt:
            say("    worst: " + worst_entries(m, ref_m, case["obs"].sigma))
        assert e.max() < mt
        assert np.all(np.isfinite(ll))
        assert lle.max() < LOGL_TOL[prec]
        if prec == "fp16":
            assert dnear <= 0.05


def check_grad(tag, case, L, O, theta):
    ll_ref, g_ref = adjoint.logl_grad(case["olib"], case["obs"], theta)
    S = grad_scale(case["olib"], case["obs"], theta)
    nz = grad_noise(case, theta)
    for prec, tol in (("fp64", 1e-9), ("fp32", 1e-4)):
        th = torch.tensor(theta, dtype=torch.float64, device="cuda")
        ll, g = sps.logl_grad(L, O, th, prec)
        torch.cuda.synchronize()
        ll, g = ll.cpu().numpy(), g.cpu().numpy()
        e = grad_ratio(g, g_ref, S, nz * (2.0 ** -29 if prec == "fp64" else 1.0), tol)
        pl = rel_err(g, g_ref)
        lle = np.max(np.abs(ll - ll_ref) / np.maximum(1.0, np.abs(ll_ref)))
        worst = np.argsort(e.max(axis=0))[::-1][:3]
        say(f"  {tag} grad {prec}: max ratio to the bar {e.max():.3e} (plain rel p99 {np.percentile(pl, 99):.3e}); "
            f"logL rel {lle:.3e}; worst columns {worst.tolist()}")
        assert e.max() <= 1.0
        assert lle < (1e-10 if prec == "fp64" else 1e-4)


# ------------------------------------------------------------------ inclusion mask
@pytest.fixture(scope="module")
def phot_masked():
    case = make_case(CFG_PHOT, B=48, kind="phot")
    obs = case["obs"]
    obs.data = obs.data.copy()
    obs.sigma = obs.sigma.copy()
    obs.data[3] = np.nan
    obs.sigma[5] = 0.0
    obs.sigma[7] = -obs.sigma[7]
    obs.data[9] = np.inf
    obs.mask = np.ones(obs.data.size, dtype=np.uint8)
    obs.mask[[10, 11, 16]] = 0
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    return case, L, O


def test_mask_photometry_forward(phot_masked):
    case, L, O = phot_masked
    say("masked photometry: NaN and inf data, sigma = 0 and < 0, user mask")
    check_forward("phot-mask", case, L, O, batch(case), ("fp64", "fp32", "fp16"))


def test_mask_photometry_gradient(phot_masked):
    case, L, O = phot_masked
    check_grad("phot-mask", case, L, O, near_truth(case["cfg"], case["theta_true"], 12, 62))


@pytest.fixture(scope="module")
def spec_masked():
    case = make_case(CFG_SPEC, B=48, kind="spec")
    obs = case["obs"]
    obs.data = obs.data.copy()
    obs.sigma = obs.sigma.copy()
    obs.data[[4, 150]] = np.nan
    obs.sigma[[20, 21]] = 0.0
    obs.sigma[200] = -1.0
    obs.mask = np.ones(obs.data.size, dtype=np.uint8)
    obs.mask[100:140] = 0
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    return case, L, O


def test_mask_spectrum_forward(spec_masked):
    case, L, O = spec_masked
    say("masked spectrum: NaN data, sigma = 0 and < 0, a masked range")
    check_forward("spec-mask", case, L, O, batch(case), ("fp64", "fp32", "fp16"), spec=True)


def test_mask_spectrum_gradient(spec_masked):
    case, L, O = spec_masked
    check_grad("spec-mask", case, L, O, near_truth(case["cfg"], case["theta_true"], 12, 63))


# ------------------------------------------------------------------ kernel widths and LSF modes
SPEC_VARIANTS = {
    "sigma_gal_200": dict(sigma_gal_kms=200.0),
    "fwhm_aa": dict(lsf_mode="fwhm_aa", lsf_value=350.0),
    "sigma_kms": dict(lsf_mode="sigma_kms", lsf_value=1100.0),
    # a prism-like resolving power rising from ~40 to ~300 over the range
    "R_curve": dict(lsf_mode="R_fwhm", lsf_value=lambda w: 40.0 + 260.0 * ((w - w[0]) / (w[-1] - w[0])) ** 1.5),
}


@pytest.fixture(scope="module", params=list(SPEC_VARIANTS))
def spec_variant(request):
    case = make_case(CFG_SPEC, B=48, kind="spec", spec=SPEC_VARIANTS[request.param])
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    return request.param, case, L, O


def test_spectrum_variant_forward(spec_variant):
    name, case, L, O = spec_variant
    say(f"spectrum {name}")
    check_forward(name, case, L, O, batch(case), ("fp64", "fp32", "fp16"), spec=True)


def test_spectrum_variant_gradient(spec_variant):
    name, case, L, O = spec_variant
    check_grad(name, case, L, O, near_truth(case["cfg"], case["theta_true"], 12, 64))


# ------------------------------------------------------------------ noise floor on a spectrum
@pytest.fixture(scope="module")
def spec_noise():
    case = make_case(CFG_SPEC, B=48, kind="spec", noise=("err_scale", "f_calib", "f_data", "jitter"))
    cols = om.columns(CFG_SPEC.n_sfh, CFG_SPEC.n_zh)
    th = batch(case, 16, 16)
    rng = np.random.default_rng(65)
    med = np.median(np.abs(case["obs"].data))
    th[:, cols["log_err_scale"]] = np.log(rng.uniform(0.8, 1.5, th.shape[0]))
    th[:, cols["log_f_calib"]] = np.log(rng.uniform(0.01, 0.05, th.shape[0]))
    th[:, cols["log_f_data"]] = np.log(rng.uniform(0.01, 0.05, th.shape[0]))
    th[:, cols["log_jitter"]] = np.log(rng.uniform(0.01, 0.05, th.shape[0]) * med)
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    return case, L, O, th


def test_noise_floor_spectrum_forward(spec_noise):
    case, L, O, th = spec_noise
    say("spectrum with s, f_calib, f_data and jitter")
    check_forward("spec-noise", case, L, O, th, ("fp64", "fp32", "fp16"), spec=True)


def test_noise_floor_spectrum_gradient(spec_noise):
    case, L, O, th = spec_noise
    check_grad("spec-noise", case, L, O, th[16:28])


# ------------------------------------------------------------------ constant Z and [alpha/Fe] beyond the grid
def test_constant_metallicity_outside_grid():
    case = make_case(wl.CONFIGS["c0"], B=64)
    cols = om.columns(case["cfg"].n_sfh, case["cfg"].n_zh)
    th = case["theta"].copy()
    th[:, cols["logzsol"]] = np.linspace(-3.5, 1.2, th.shape[0])   # grid is [-2, 0]
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    say("c0: logzsol from -3.5 to 1.2 over a [-2, 0] grid")
    check_forward("c0-Zclamp", case, L, O, th, ("fp64", "fp32", "fp16"))


def test_alpha_and_metallicity_outside_grid():
    cfg = wl.reduced(wl.CONFIGS["c4"], n_age=30, logz=(-2.0, -1.0, 0.0), afe=(0.0, 0.2, 0.4), n_wave=1000, n_sfh=10)
    case = make_case(cfg, B=64, kind="phot")
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    th = case["theta"].copy()
    th[:, cols["afe"]] = np.linspace(-0.4, 0.9, th.shape[0])
    th[:, cols["logzsol"]] = np.linspace(0.8, -2.9, th.shape[0])
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=64)
    say("alpha library: afe from -0.4 to 0.9 over [0, 0.4], logzsol from 0.8 to -2.9 over [-2, 0]")
    check_forward("afe-clamp", case, L, O, th, ("fp64", "fp32", "fp16"))


# ------------------------------------------------------------------ a redshift that is not a number
def _raw_logl(L, O, theta, B, prec, logl_buf, model_buf):
    lib = sps.lib()
    st = lib.sps_logl(L.handle, O.handle, C.c_void_p(theta.data_ptr()), B, sps.PRECISIONS[prec],
                      C.c_void_p(logl_buf.data_ptr()), C.c_void_p(model_buf.data_ptr()),
                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.sps_last_error().decode()


@pytest.mark.parametrize("kind", ["phot", "spec"])
def test_nan_redshift_row_after_larger_batch(kind):
    """A larger batch first leaves its per-point rows in the workspace; then one row of a
    smaller batch has z = NaN.  That row's logL is not finite, every other row is bitwise
    equal to the same batch with a finite z in that row, and nothing is written past B."""
    cfg = CFG_PHOT if kind == "phot" else CFG_SPEC
    case = make_case(cfg, B=320, kind=kind)
    L, O = gpu_objects(case, precisions=("fp64", "fp32", "fp16"), max_batch=384)
    cols = om.columns(cfg.n_sfh, cfg.n_zh)
    n = O.n_data
    for prec in ("fp64", "fp32", "fp16"):
        say(f"NaN z row, {kind} {prec}: B=320 then B=200 with row 17 at z = NaN")
        big = torch.tensor(case["theta"], dtype=torch.float64, device="cuda")
        sps.logl(L, O, big, prec)
        th_ok = case["theta"][:200].copy()
        th_nan = th_ok.copy()
        th_nan[17, cols["zred"]] = np.nan
        ll_ok, m_ok = sps.logl(L, O, torch.tensor(th_ok, device="cuda"), prec, return_model=True)
        sps.logl(L, O, big, prec)
        lbuf = torch.full((320,), 12345.0, dtype=torch.float64, device="cuda")
        mbuf = torch.full((320, n), 777.0, dtype=torch.float64, device="cuda")
        _raw_logl(L, O, torch.tensor(th_nan, device="cuda"), 200, prec, lbuf, mbuf)
        torch.cuda.synchronize()
        lb, mb = lbuf.cpu().numpy(), mbuf.cpu().numpy()
        ll_ok, m_ok = ll_ok.cpu().numpy(), m_ok.cpu().numpy()
        assert np.all(lb[200:] == 12345.0) and np.all(mb[200:] == 777.0)
        assert not np.isfinite(lb[17])
        others = np.r_[0:17, 18:200]
        assert np.array_equal(lb[others], ll_ok[others])
        assert np.array_equal(mb[others], m_ok[others])
    # the gradient pass: the other rows' logL and gradient agree with the finite batch
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        th_ok = case["theta"][:200].copy()
        th_nan = th_ok.copy()
        th_nan[17, cols["zred"]] = np.nan
        ll_a, g_a = sps.logl_grad(L, O, torch.tensor(th_ok, device="cuda"), prec)
        ll_b, g_b = sps.logl_grad(L, O, torch.tensor(th_nan, device="cuda"), prec)
        torch.cuda.synchronize()
        ll_a, g_a, ll_b, g_b = (x.cpu().numpy() for x in (ll_a, g_a, ll_b, g_b))
        others = np.r_[0:17, 18:200]
        assert not np.isfinite(ll_b[17])
        assert np.array_equal(ll_a[others], ll_b[others])
        assert np.all(np.abs(g_a[others] - g_b[others]) <= tol * np.maximum(np.abs(g_a[others]), 1e-300)
                      + 1e-12 * np.abs(g_a[others]).max(axis=1, keepdims=True))
