"""Full-size serving library against the FP64 oracle: the alpha-enhanced grid of
107 ages x 22 [Fe/H] x 3 [alpha/Fe] x 5994 wavelengths (K = 7062, constant metallicity,
no nebular emission), stored as FP16 hi + residual and contracted in three MFMA passes,
the precision the request server runs (Sec. 5.4).

Two observations of the serving stream's extremes: 25-band photometry and a 3000-pixel
prism spectrum.  Batches of 1024 points and of 4096 points (the size of a busy serving
tick); half of each batch are prior draws, half perturbations of the data-generating
vector.  Bars: 2e-3 per band or pixel (relative error floored at 1e-6 of the datum's sigma), logL within 1e-4
relative, and |dlogL| <= 0.05 where chi^2 per datum <= 100.
"""
import sys

import numpy as np
import pytest

from helpers import gpu_observation, model_err, near_truth, worst_entries
from oracle import model as om
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402

CFG = wl.CONFIGS["c4"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c4lib():
    lib = wl.make_library(CFG, 0)
    dust = wl.make_dust_tables(CFG, lib["wave"])
    olib = om.build_library(CFG, lib, None, dust)
    L = sps.Library(lib, n_sfh=CFG.n_sfh, T1=CFG.T1, n_zh=CFG.n_zh, cosmo=CFG.cosmo, dust=dust,
                    precisions=("fp16",))
    say(f"c4 library: K = {L.info['K']}, K_pad = {L.info['K_pad']}, N = {L.info['N']}")
    return lib, dust, olib, L


def _case(c4lib, kind, B):
    lib, dust, olib, L = c4lib
    theta_true = wl.make_theta(CFG, 1, seed=4100)
    if kind == "phot":
        obs = om.Photometry(filters=wl.make_filters("gaussN", 25))
        m_true = om.predict(olib, obs, theta_true)[0]
        obs.data, obs.sigma = wl.noisy_photometry(m_true, 4101)
    else:
        g = wl.make_spectrum_grid(3000)
        obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"], g["sigma_gal_kms"],
                          z_ref=float(theta_true[0, 1]))
        m_true = om.predict(olib, obs, theta_true)[0]
        obs.data, obs.sigma = wl.noisy_spectrum(m_true, 4101)
    theta = np.concatenate([wl.make_theta(CFG, B // 2, seed=4102 + B),
                            near_truth(CFG, theta_true, B - B // 2, 4103 + B)])
    case = dict(cfg=CFG, lib=lib, lines=None, dust=dust, olib=olib, theta=theta, theta_true=theta_true, obs=obs,
                kind=kind)
    return case


@pytest.mark.parametrize("kind,B,n_check", [("phot", 1024, 1024), ("phot", 4096, 4096), ("spec", 1024, 96),
                                            ("spec", 4096, 64)])
def test_c4_full_size_fp16_three_pass(c4lib, kind, B, n_check):
    lib, dust, olib, L = c4lib
    case = _case(c4lib, kind, B)
    O = gpu_observation(L, case, max_batch=B)
    say(f"c4 full size {kind} B={B}: fp16 3-pass, {n_check} rows against the oracle")
    th = torch.tensor(case["theta"], dtype=torch.float64, device="cuda")
    ll, m = sps.logl(L, O, th, "fp16", return_model=True)
    torch.cuda.synchronize()
    ll, m = ll.cpu().numpy(), m.cpu().numpy()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(m))
    idx = np.linspace(0, B - 1, n_check).astype(int)
    m_ref = om.predict(olib, case["obs"], case["theta"][idx])
    ll_ref = om.logl(olib, case["obs"], case["theta"][idx], model=m_ref)
    e = model_err(m[idx], m_ref, case["obs"].sigma)
    lle = np.abs(ll[idx] - ll_ref) / np.abs(ll_ref)
    chi2 = np.mean(((case["obs"].data - m_ref) / case["obs"].sigma) ** 2, axis=1)
    near = chi2 <= 100
    dnear = np.abs(ll[idx] - ll_ref)[near].max() if near.any() else 0.0
    say(f"  max rel err {e.max():.3e} (p99 {np.percentile(e, 99):.3e}); logL rel err {lle.max():.3e}; "
        f"|dlogL| near data ({near.sum()} rows) {dnear:.3e}")
    if e.max() >= 2e-3:
        say("  worst: " + worst_entries(m[idx], m_ref, case["obs"].sigma))
    assert e.max() < 2e-3
    assert lle.max() < 1e-4
    assert dnear <= 0.05
    O.close()
