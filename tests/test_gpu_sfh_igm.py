"""GPU parity for the linear (tent-integral) SFH scheme (App. B, eq. tent_integral) and the
IGM transmission (Sec. 2.6, Madau 1995), each against the FP64 oracle on the same seeded
inputs, through the C ABI:

  - the linear scheme with a time-varying enrichment history and at constant metallicity
    on an [alpha/Fe] library (photometry);
  - the IGM on photometry (redshifts 0.5-12, so that the bluest bands cross the Lyman
    alpha forest and the Lyman limit) and on a spectrum with lines;
  - the Madau IGM with the damping wing of a partly neutral IGM and a damped Lyman-alpha
    absorber (Sec. 2.6), on photometry and on a spectrum, with sources on both sides of
    z = 6, x_HI of 0 and 1, absorbers at the source, far in front of it, of negligible and
    of saturating column;
  - everything at once: linear SFH, IGM, nebular continuum and the runaway_bc escape;
  - a batch over several M tiles with a ragged tail at FP64, FP32, FP16 hi + residual
    (three passes) and, on photometry, FP16 hi + weight residual;
  - the gradient call refuses these libraries.

Tolerances: per-output relative error floored at 1e-6 of the datum's sigma, FP64 1e-12
(spectra 1e-11), FP32 1e-5, 16-bit 2e-3; logL FP64 1e-10, FP32 and FP16 three-pass 1e-4,
FP16 weight residual 1e-3 relative; 16-bit |dlogL| <= 0.05 within reach of the data.
"""
import sys

import numpy as np
import pytest

from helpers import gpu_objects, make_case, model_err, near_truth, worst_entries
from oracle import model as om
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402

CFG_PHOT = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=30,
                      n_zh=6, n_lines=24)
CFG_ALPHA = wl.reduced(wl.CONFIGS["c4"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 6)), n_wave=1500, n_sfh=24)
CFG_SPEC = wl.reduced(wl.CONFIGS["c3"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=16,
                      n_zh=5, n_lines=24, n_pix=300)
MODEL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 2e-3, "fp16_wl": 2e-3}
LOGL_TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16": 1e-4, "fp16_wl": 1e-3}
PRECS = ("fp64", "fp32", "fp16", "fp16_wl")
B = 200


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check(tag, case, L, O, theta, spec):
    ref_m = om.predict(case["olib"], case["obs"], theta)
    ref_ll = om.logl(case["olib"], case["obs"], theta, model=ref_m)
    obs = case["obs"]
    near = np.mean(((obs.data - ref_m) / obs.sigma) ** 2, axis=1) <= 100
    for prec in PRECS:
        if spec and prec == "fp16_wl":
            continue
        th = torch.tensor(theta, dtype=torch.float64, device="cuda")
        say(f"  {tag} {prec}: B={theta.shape[0]} P={theta.shape[1]}")
        ll, m = sps.logl(L, O, th, prec, return_model=True)
        torch.cuda.synchronize()
        ll, m = ll.cpu().numpy(), m.cpu().numpy()
        e = model_err(m, ref_m, obs.sigma)
        lle = np.abs(ll - ref_ll) / np.maximum(1.0, np.abs(ref_ll))
        dnear = np.abs(ll - ref_ll)[near].max() if near.any() else 0.0
        say(f"    model max rel err {e.max():.3e}; logL rel err {lle.max():.3e}; "
            f"|dlogL| near data ({near.sum()} rows) {dnear:.3e}")
        mt = MODEL_TOL[prec] * (10 if (spec and prec == "fp64") else 1)
        if e.max() >= mt:
            say("    worst: " + worst_entries(m, ref_m, obs.sigma))
        assert e.max() < mt
        assert np.all(np.isfinite(ll))
        assert lle.max() < LOGL_TOL[prec]
        if prec.startswith("fp16"):
            assert dnear <= 0.05


def theta_of(case, seed=91):
    th = np.concatenate([case["theta"][:B - 24], near_truth(case["cfg"], case["theta_true"], 24, seed)])
    cols = om.lib_columns(case["olib"])
    if case["igm"]:
        th[:4, cols["igm_factor"]] = [0.0, 1.0, 2.0, 0.3]   # off, nominal, doubled, weak
    if "x_hi" in cols:   # the damping wing: sources on both sides of z = 6, fully neutral, none
        th[4:12, 1] = [5.9, 6.0, 6.05, 6.5, 7.5, 9.0, 11.0, 11.9]
        th[4:8, cols["x_hi"]] = [1.0, 0.0, 1.0, 0.5]
    if "log_nhi" in cols:   # the absorber: at the source, far in front, negligible, saturated
        th[12:16, 1] = [3.0, 7.0, 9.5, 11.0]
        th[12:16, cols["z_dla"]] = [3.0, 5.0, 9.4, 10.999]
        th[12:16, cols["log_nhi"]] = [22.0, 20.3, 0.0, 21.7]
    return th


CASES = {
    "linear_zh": (CFG_PHOT, "phot", dict(sfh_scheme="linear")),
    "linear_alpha": (CFG_ALPHA, "phot", dict(sfh_scheme="linear")),
    "igm_phot": (CFG_PHOT, "phot", dict(igm=True)),
    "igm_spec": (CFG_SPEC, "spec", dict(igm=True)),
    "igm_wing_dla_phot": (CFG_PHOT, "phot", dict(igm=7)),
    "igm_wing_dla_spec": (CFG_SPEC, "spec", dict(igm=7)),
    "all_phot": (CFG_PHOT, "phot", dict(sfh_scheme="linear", igm=True, cont=True, escape="runaway_bc")),
    "all_spec": (CFG_SPEC, "spec", dict(sfh_scheme="linear", igm=True, cont=True, escape="runaway_bc")),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    cfg, kind, kw = CASES[request.param]
    c = make_case(cfg, B=B, kind=kind, **kw)
    L, O = gpu_objects(c, precisions=("fp64", "fp32", "fp16"), max_batch=256)
    return request.param, c, L, O


def test_forward_parity(case):
    name, c, L, O = case
    check(name, c, L, O, theta_of(c), spec=c["kind"] == "spec")


def test_layout_and_gradient_refusal(case):
    name, c, L, O = case
    cols = om.lib_columns(c["olib"])
    assert L.layout["P"] == cols["P"]
    for k in ("igm_factor", "x_hi", "log_nhi", "z_dla", "sigma_gal"):
        assert L.layout[k] == cols.get(k, -1)
    th = torch.tensor(theta_of(c)[:8], dtype=torch.float64, device="cuda")
    with pytest.raises(sps.SpsError) as ei:
        sps.logl_grad(L, O, th, "fp32")
    assert ei.value.code == -1   # SPS_E_INVAL
