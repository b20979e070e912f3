"""GPU request server: continuous batching of photometry and spectra requests on one
library; each request's result is the same alone and in the mix, its final logL agrees
with a direct sps_logl evaluation of its final live points, and with the FP64 oracle's
logL of those points (relative 1e-4 for FP32 and FP16 hi + residual, which also holds each
band or pixel of the forward model within 1e-5 and 2e-3 of the oracle)."""
import sys
import time

import numpy as np
import pytest

from helpers import model_err
from oracle import model as om
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402

CFG = wl.reduced(wl.CONFIGS["c4"], n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), afe=(0.0, 0.2, 0.4),
                 n_wave=1500, n_sfh=24)


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def glib():
    lib = wl.make_library(CFG, 0)
    dust = wl.make_dust_tables(CFG, lib["wave"])
    G = sps.Library(lib, n_sfh=CFG.n_sfh, T1=CFG.T1, n_zh=CFG.n_zh, cosmo=CFG.cosmo, dust=dust,
                    precisions=("fp32", "fp16"))
    G.oracle = om.build_library(CFG, lib, None, dust)
    return G


def _oracle_obs(kind, o):
    if kind == "phot":
        return om.Photometry(filters=o["filters"], data=o["data"], sigma=o["sigma"])
    return om.Spectrum(o["pix_wave"], "R_fwhm", 100.0, 100.0, 0.0, z_ref=3.0, data=o["data"], sigma=o["sigma"])


def _obs(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "phot":
        d = 1e-9 * np.exp(rng.normal(0, 0.3, n))
        return dict(filters=wl.make_filters("gaussN", n), data=d, sigma=0.05 * d)
    g = wl.make_spectrum_grid(n)
    d = 1e-9 * np.exp(rng.normal(0, 0.3, n))
    return dict(pix_wave=g["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0, z_ref=3.0, sigma_gas_kms=100.0,
                data=d, sigma=0.05 * d)


JOBS = [("phot", 12, 64), ("spec", 500, 192), ("phot", 25, 256), ("spec", 1200, 128)]


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_alone_equals_mixed_and_matches_direct_logl(glib, precision):
    say(f"server {precision}: {len(JOBS)} requests alone, then mixed")
    alone = {}
    for k, (kind, n, B) in enumerate(JOBS):
        S = sps.Server(glib, precision=precision, max_points=2048, max_active=16, hbm_budget_bytes=1 << 30)
        t = S.submit(kind, wl.make_theta(CFG, B, seed=50 + k), n_iter=6, seed=7 + k, **_obs(kind, n, k))
        alone[k] = S.wait(t, timeout_s=60)
        S.close()
        assert alone[k]["state"] == "done"
    S = sps.Server(glib, precision=precision, max_points=2048, max_active=16, hbm_budget_bytes=1 << 30)
    ts = []
    for k, (kind, n, B) in enumerate(JOBS):
        ts.append(S.submit(kind, wl.make_theta(CFG, B, seed=50 + k), n_iter=6, seed=7 + k, **_obs(kind, n, k)))
        time.sleep(0.001)
    for k, t in enumerate(ts):
        r = S.wait(t, timeout_s=60)
        assert r["state"] == "done"
        assert np.array_equal(r["logl"], alone[k]["logl"]), k
        assert np.array_equal(r["theta"], alone[k]["theta"]), k
    st = S.stats()
    say(f"  stats: ticks {st['ticks']} points/tick {st['mean_points_per_tick']:.0f} evals/s {st['evals_per_s']:.3g}")
    assert st["completed"] == len(JOBS)
    S.close()
    # the final live points' logL equals a direct evaluation
    for k, (kind, n, B) in enumerate(JOBS[:2]):
        o = _obs(kind, n, k)
        if kind == "phot":
            O = sps.Observation(glib, "phot", B, filters=o["filters"], data=o["data"], sigma=o["sigma"])
        else:
            O = sps.Observation(glib, "spec", B, pix_wave=o["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0,
                                z_ref=3.0, sigma_gas_kms=100.0, data=o["data"], sigma=o["sigma"])
        th = torch.tensor(alone[k]["theta"], device="cuda")
        ll = sps.logl(glib, O, th, precision).cpu().numpy()
        assert np.array_equal(ll, alone[k]["logl"]), k
    # every request's final live points against the FP64 oracle
    mtol = 1e-5 if precision == "fp32" else 2e-3
    for k, (kind, n, B) in enumerate(JOBS):
        o = _obs(kind, n, k)
        oo = _oracle_obs(kind, o)
        th = alone[k]["theta"]
        m_ref = om.predict(glib.oracle, oo, th)
        ll_ref = om.logl(glib.oracle, oo, th, model=m_ref)
        lle = np.abs(alone[k]["logl"] - ll_ref) / np.abs(ll_ref)
        if kind == "phot":
            O = sps.Observation(glib, "phot", B, filters=o["filters"], data=o["data"], sigma=o["sigma"])
        else:
            O = sps.Observation(glib, "spec", B, pix_wave=o["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0,
                                z_ref=3.0, sigma_gas_kms=100.0, data=o["data"], sigma=o["sigma"])
        m = sps.forward(glib, O, torch.tensor(th, device="cuda"), precision).cpu().numpy()
        e = model_err(m, m_ref, o["sigma"])
        say(f"  request {k} ({kind}, {n}, B={B}) vs oracle: logL rel err {lle.max():.3e}, model rel err {e.max():.3e}")
        assert lle.max() < 1e-4, k
        assert e.max() < mtol, k
