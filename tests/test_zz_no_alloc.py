"""The allocation-free entry point sps_logl_static against sps_logl, through the C ABI.

Two calls in a row on one observation, the second with a smaller batch, at FP64, FP32
and FP16 (hi + residual): logL and the model must equal sps_logl's bit for bit (the same
kernels on the same inputs; only the scratch memory differs), which is inside every
parity bar.  The device's free memory must not change across the calls, and a batch
whose scratch exceeds the static array is rejected with SPS_E_SHAPE.  The observation is
created with max_batch = 1, so its own workspace could not hold the batches.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from helpers import make_case
from synth import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2609_30145_amd as sps  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _call(fn, L, O, th, prec, ll, m):
    lib = sps.lib()
    st = fn(L.handle, O.handle, C.c_void_p(th.data_ptr()), th.shape[0], sps.PRECISIONS[prec],
            C.c_void_p(ll.data_ptr()), C.c_void_p(m.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, lib.sps_last_error().decode()


@pytest.mark.parametrize("kind", ["phot", "spec"])
def test_static_entry_matches_logl_on_two_calls(kind):
    base = wl.CONFIGS["c1"] if kind == "phot" else wl.CONFIGS["c3"]
    cfg = wl.reduced(base, n_age=40, logz=tuple(np.linspace(-2.5, 0.5, 8)), n_wave=1500, n_sfh=20, n_zh=5,
                     n_lines=24, n_pix=400)
    case = make_case(cfg, B=300, kind=kind)
    obs = case["obs"]
    L = sps.Library(case["lib"], n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=case["dust"],
                    lines=case["lines"], precisions=("fp64", "fp32", "fp16"))
    if kind == "phot":
        O_small = sps.Observation(L, "phot", 1, filters=obs.filters, data=obs.data, sigma=obs.sigma)
        O_ref = sps.Observation(L, "phot", 300, filters=obs.filters, data=obs.data, sigma=obs.sigma)
    else:
        kw = dict(pix_wave=obs.pix_wave, lsf_mode=obs.lsf_mode, lsf_value=obs.lsf_value, z_ref=obs.z_ref,
                  sigma_gal_kms=obs.sigma_gal_kms, sigma_gas_kms=obs.sigma_gas_kms, data=obs.data, sigma=obs.sigma)
        O_small = sps.Observation(L, "spec", 1, **kw)
        O_ref = sps.Observation(L, "spec", 300, **kw)
    lib = sps.lib()
    n = O_ref.n_data
    for prec in ("fp64", "fp32", "fp16"):
        outs = {}
        for B in (300, 70):   # two calls in a row, the second smaller
            th = torch.tensor(case["theta"][:B], dtype=torch.float64, device="cuda")
            ll_a = torch.empty(B, dtype=torch.float64, device="cuda")
            m_a = torch.empty((B, n), dtype=torch.float64, device="cuda")
            ll_b = torch.empty_like(ll_a)
            m_b = torch.empty_like(m_a)
            # the reference call first: the runtime loads each kernel's code on its first
            # launch in the process, which takes device memory that is not the entry point's
            st, msg = _call(lib.sps_logl, L, O_ref, th, prec, ll_b, m_b)
            assert st == 0, msg
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            st, msg = _call(lib.sps_logl_static, L, O_small, th, prec, ll_a, m_a)
            assert st == 0, msg
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            say(f"static entry {kind} {prec} B={B}: free device memory {free0} -> {free1}")
            assert free1 == free0
            outs[B] = (ll_a.cpu().numpy(), m_a.cpu().numpy(), ll_b.cpu().numpy(), m_b.cpu().numpy())
            assert np.all(np.isfinite(outs[B][0]))
            assert np.array_equal(outs[B][0], outs[B][2]), (prec, B)
            assert np.array_equal(outs[B][1], outs[B][3]), (prec, B)
        # the smaller batch's rows equal the larger batch's first rows (no stale scratch)
        assert np.array_equal(outs[70][0], outs[300][0][:70])
    # a batch whose scratch exceeds the static array is rejected before any launch
    B = 16384
    th = torch.zeros((B, L.P), dtype=torch.float64, device="cuda")
    ll = torch.empty(B, dtype=torch.float64, device="cuda")
    m = torch.empty((B, n), dtype=torch.float64, device="cuda")
    st, msg = _call(lib.sps_logl_static, L, O_small, th, "fp64", ll, m)
    say(f"B={B} fp64: status {st} ({msg})")
    assert st == -2
