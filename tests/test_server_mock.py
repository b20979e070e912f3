"""Scheduler tests on a host-only library with the mock executor (no GPU needed):
FIFO admission under an HBM budget and a point capacity, continuous batching,
results independent of co-scheduled requests, rejection, cancellation, shutdown."""
import time

import numpy as np
import pytest

import paper_2609_30145_amd as sps
from synth import workloads as wl

CFG = wl.reduced(wl.CONFIGS["c4"], n_age=20, logz=(-2.0, -1.0, 0.0), afe=(0.0, 0.2, 0.4), n_wave=300, n_sfh=8)


@pytest.fixture(scope="module")
def hostlib():
    lib = wl.make_library(CFG, 0)
    return sps.Library(lib, n_sfh=CFG.n_sfh, T1=CFG.T1, n_zh=CFG.n_zh, device=-1)


def _obs(kind, n):
    if kind == "phot":
        filt = wl.make_filters("gaussN", n)
        return dict(filters=filt, data=np.full(n, 1e-9), sigma=np.full(n, 5e-11))
    g = wl.make_spectrum_grid(n)
    return dict(pix_wave=g["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0, z_ref=2.0,
                data=np.full(n, 1e-9), sigma=np.full(n, 5e-11))


def _theta(B, seed):
    return wl.make_theta(CFG, B, seed=seed)


def test_requests_complete_and_match_alone_vs_mixed(hostlib):
    alone = {}
    for k, (kind, n, B) in enumerate([("phot", 12, 64), ("spec", 400, 128), ("phot", 20, 192)]):
        S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=4096)
        t = S.submit(kind, _theta(B, 10 + k), n_iter=5, seed=100 + k, **_obs(kind, n))
        alone[k] = S.wait(t, timeout_s=30)
        S.close()
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=4096)
    tickets = {}
    for k, (kind, n, B) in enumerate([("phot", 12, 64), ("spec", 400, 128), ("phot", 20, 192)]):
        tickets[k] = S.submit(kind, _theta(B, 10 + k), n_iter=5, seed=100 + k, **_obs(kind, n))
        time.sleep(0.002)
    for k, t in tickets.items():
        r = S.wait(t, timeout_s=30)
        assert r["state"] == "done"
        assert np.array_equal(r["theta"], alone[k]["theta"])
        assert np.array_equal(r["logl"], alone[k]["logl"])
        assert r["evals"] == 6 * r["B"]
    st = S.stats()
    assert st["completed"] == 3 and st["completed_by_kind"] == [2, 1]
    assert st["p99_latency_s"][0] >= st["p50_latency_s"][0] > 0
    # logL only improves: the sampler accepts proposals above the worst quartile
    r = S.wait(tickets[0])
    assert np.all(np.isfinite(r["logl"]))
    S.close()


def test_budget_rejects_requests_that_can_never_fit(hostlib):
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=200_000, max_points=4096)
    with pytest.raises(sps.SpsError) as ei:
        S.submit("phot", _theta(1024, 1), n_iter=1, seed=1, **_obs("phot", 10))
    assert ei.value.code == -4
    with pytest.raises(sps.SpsError) as ei:
        S.submit("phot", _theta(8192, 1), n_iter=1, seed=1, **_obs("phot", 10))
    assert ei.value.code == -2
    with pytest.raises(sps.SpsError) as ei:
        S.submit("spec", _theta(8, 1), n_iter=1, seed=1, **dict(_obs("spec", 100), lsf_mode="R"))
    assert ei.value.code == -1
    assert S.stats()["rejected"] == 3
    S.close()


def test_admission_waits_for_budget_and_peak_stays_within(hostlib):
    one = 64 * (14 + CFG.n_sfh) * 8 + 64 * 8
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=int(2.3 * (one + 40_000)), max_points=4096,
                   mock_eval_ns=20_000.0)
    ts = [S.submit("phot", _theta(64, k), n_iter=10, seed=k, **_obs("phot", 10)) for k in range(6)]
    res = [S.wait(t, timeout_s=60) for t in ts]
    assert all(r["state"] == "done" for r in res)
    st = S.stats()
    assert st["hbm_peak"] <= st["hbm_budget"]
    assert st["max_queue_s"] > 0.0          # later requests waited for memory
    assert max(r["queue_s"] for r in res) > min(r["queue_s"] for r in res)
    S.close()


def test_point_capacity_limits_concurrency(hostlib):
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=256, mock_eval_ns=10_000.0)
    ts = [S.submit("phot", _theta(192, k), n_iter=4, seed=k, **_obs("phot", 8)) for k in range(3)]
    res = [S.wait(t, timeout_s=60) for t in ts]
    assert all(r["state"] == "done" for r in res)
    assert S.stats()["mean_points_per_tick"] <= 256
    S.close()


def test_cancel_pending_and_active(hostlib):
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=128, mock_eval_ns=200_000.0)
    t1 = S.submit("phot", _theta(128, 1), n_iter=200, seed=1, **_obs("phot", 8))
    t2 = S.submit("phot", _theta(128, 2), n_iter=200, seed=2, **_obs("phot", 8))
    time.sleep(0.2)
    S.cancel(t2)                                   # still queued behind t1
    assert S.wait(t2, timeout_s=5)["state"] == "cancelled"
    S.cancel(t1)                                   # running
    assert S.wait(t1, timeout_s=30)["state"] == "cancelled"
    with pytest.raises(sps.SpsError):
        S.release(12345)
    S.release(t1)
    with pytest.raises(sps.SpsError):
        S.poll(t1)
    S.close()


def test_shutdown_with_pending_work_returns(hostlib):
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=128, mock_eval_ns=100_000.0)
    for k in range(5):
        S.submit("phot", _theta(128, k), n_iter=1000, seed=k, **_obs("phot", 8))
    time.sleep(0.05)
    t0 = time.time()
    S.close()
    assert time.time() - t0 < 10


def test_wait_timeout(hostlib):
    S = sps.Server(hostlib, device=-1, hbm_budget_bytes=1 << 30, max_points=128, mock_eval_ns=200_000.0)
    t = S.submit("phot", _theta(128, 1), n_iter=500, seed=1, **_obs("phot", 8))
    with pytest.raises(sps.SpsError) as ei:
        S.wait(t, timeout_s=0.05)
    assert ei.value.code == -7
    S.cancel(t)
    S.close()
