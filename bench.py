#!/usr/bin/env python3
"""Benchmark of the batched SPS forward model + logL on one MI355X.

A step is one sps_logl call over a batch of 1024 live points of the full-size
photometric workload (library 107 ages x 22 metallicities x 5994 wavelengths,
120-bin SFH with a 24-node enrichment history, two-component dust, 128 nebular
lines, 20 filters): sort + weights + K-tile lists + library contraction (fused
attenuation) + projection + FP64 chi-squared.  Inputs are resident in HBM.

The timed variant is FP16 storage with FP32 accumulation and one weight-residual
MFMA pass (W_h L_h + W_l L_h), the cheapest variant that meets 2e-3 per band and
|dlogL| <= 0.05 on this workload; the three-pass variant (library residual as well),
which spectra need, FP32 and BF16 are timed beside it.

Prints one JSON line.  The roofline entry is for the library contraction, timed
live during the timed steps with HIP events that the kernel's own dispatch stamps
(start and end) on the stream it runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0, "bf16_hr": 2500.0,
               "fp16_hr": 2500.0, "bf16_1pass": 2500.0, "fp16_1pass": 2500.0, "bf16_wl": 2500.0,
               "fp16_wl": 2500.0}
MFMA_PASSES = {"fp32": 1, "fp64": 1, "bf16": 3, "fp16": 3, "bf16_hr": 2, "fp16_hr": 2, "bf16_1pass": 1,
               "fp16_1pass": 1, "bf16_wl": 2, "fp16_wl": 2}
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16": "bf16 (f32 accumulate, residual pass)",
         "fp16": "f16 (f32 accumulate, residual pass)", "bf16_hr": "bf16", "fp16_hr": "f16",
         "bf16_1pass": "bf16", "fp16_1pass": "f16", "bf16_wl": "bf16 (f32 accumulate, weight residual pass)",
         "fp16_wl": "f16 (f32 accumulate, weight residual pass)"}


def traffic_record(precision):
    """HBM bytes per launch of the contraction from the committed counter summary, or
    None when there is none for this precision or the kernel sources changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))):
        text = open(path).read()
        for line in text.splitlines():
            line = line.strip()
            if not (line.startswith("{") and '"traffic_bytes_per_launch"' in line):
                continue
            rec = json.loads(line)
            if rec.get("precision") != precision:
                continue
            h = hashlib.sha256()
            for f in rec["sources"]:
                h.update(open(os.path.join(ROOT, "paper_2609_30145_amd", "csrc", f), "rb").read())
            if h.hexdigest() != rec["sources_sha256"]:
                return None
            return dict(bytes=rec["traffic_bytes_per_launch"], source=os.path.relpath(path, ROOT))
    return None


def build_workload(cfg_name, precisions, seed=0):
    import torch

    import paper_2609_30145_amd as sps
    from synth import workloads as wl
    cfg = wl.CONFIGS[cfg_name]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=precisions)
    filters = wl.make_filters(cfg.filters)
    O = sps.Observation(L, "phot", cfg.batch, filters=filters)
    # data: the GPU model at a reference point plus 5 % noise
    th_true = torch.tensor(wl.make_theta(cfg, 1, seed=seed + 1002), device="cuda")
    m_true = sps.forward(L, O, th_true, "fp32")[0].cpu().numpy()
    d, s = wl.noisy_photometry(m_true, seed + 5)
    O.set_data(d, s)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2), device="cuda")
    return cfg, lib, lines, dust, L, O, theta


def time_precision(L, O, theta, prec, steps, warmup):
    import torch

    import paper_2609_30145_amd as sps
    for _ in range(warmup):
        sps.logl(L, O, theta, prec)
    torch.cuda.synchronize()
    O.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sps.logl(L, O, theta, prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = O.contract_timing()
    O.enable_timing(False)
    return (t1 - t0), tim


def cpu_baseline(cfg_name, budget_s=12.0, seed=0):
    """The FP64 oracle (as it stands) on the host cores over a bounded sample."""
    from oracle import model as om
    from synth import workloads as wl
    cfg = wl.CONFIGS[cfg_name]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    olib = om.build_library(cfg, lib, lines, dust)
    obs = om.Photometry(filters=wl.make_filters(cfg.filters))
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002)
    obs.data, obs.sigma = wl.noisy_photometry(om.predict(olib, obs, th_true)[0], seed + 5)
    theta = wl.make_theta(cfg, cfg.batch, seed=seed + 2)
    sample = 256
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        th = theta[(n % cfg.batch):(n % cfg.batch) + sample]
        om.logl(olib, obs, th)
        n += len(th)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    out = dict(value=n / dt, unit="evals/s", cores=int(cores), kind="oracle",
               sample=f"{n} parameter vectors of the same workload in batches of {sample} "
                      f"(FP64 NumPy, BLAS dgemm contraction), {dt:.1f} s")
    # the same oracle on one BLAS thread, over a shorter sample
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            n1 = 0
            t1 = time.perf_counter()
            while time.perf_counter() - t1 < budget_s / 3:
                om.logl(olib, obs, theta[(n1 % cfg.batch):(n1 % cfg.batch) + sample])
                n1 += sample
            out["value_1_thread"] = n1 / (time.perf_counter() - t1)
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            out["cpu_model"] = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        pass
    out["legs"] = cpu_baseline_legs(seed)
    return out


def cpu_baseline_legs(seed=0):
    """The oracle on the other workloads, each over one bounded sample: forward + logL of the
    small photometric workload (B = 64), of the headline photometric workload at B = 64 and
    in one batch of 1024, of the 3000-pixel spectrum at B = 64 (its projection is a loop over
    points, so the rate does not depend on the batch), and the spectrum's adjoint on 16
    points.  Medians over repeats where a call is short."""
    from oracle import adjoint as oa
    from oracle import model as om
    from synth import workloads as wl
    legs = []

    def case(name):
        cfg = wl.CONFIGS[name]
        lib = wl.make_library(cfg, seed)
        lines = wl.make_lines(cfg, lib, seed + 1)
        dust = wl.make_dust_tables(cfg, lib["wave"])
        olib = om.build_library(cfg, lib, lines, dust)
        th_true = wl.make_theta(cfg, 1, seed=seed + 1002)
        if cfg.n_pix:
            g = wl.make_spectrum_grid(cfg.n_pix)
            obs = om.Spectrum(g["pix_wave"], g["lsf_mode"], g["lsf_value"], g["sigma_gas_kms"], 0.0,
                              z_ref=float(th_true[0, 1]))
            obs.data, obs.sigma = wl.noisy_spectrum(om.predict(olib, obs, th_true)[0], seed + 5)
        else:
            obs = om.Photometry(filters=wl.make_filters(cfg.filters))
            obs.data, obs.sigma = wl.noisy_photometry(om.predict(olib, obs, th_true)[0], seed + 5)
        return cfg, olib, obs, wl.make_theta(cfg, max(cfg.batch, 64), seed=seed + 2)

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    for name, Bs, reps in (("c0", (64,), 5), ("c1", (64, 1024), 3), ("c3", (64,), 1)):
        cfg, olib, obs, theta = case(name)
        what = (f"{cfg.n_pix}-pixel spectrum" if cfg.n_pix else f"{cfg.filters} photometry") + \
               f", library {cfg.n_age} x {len(cfg.logz)} x {cfg.n_wave}"
        for B in Bs:
            r = reps if B < 1024 else 1
            if r > 1:
                om.logl(olib, obs, theta[:B])       # warm-up
            dt = timed(lambda: om.logl(olib, obs, theta[:B]), r)
            legs.append(dict(workload=f"{name}: {what}", path="forward + logL (FP64)", B=B,
                             value=round(B / dt, 2), unit="evals/s",
                             sample=(f"median of {r} calls" if r > 1 else "one call") +
                                    f" on {B} vectors, {dt:.2f} s per call"))
        if name == "c3":
            n = 16
            t0 = time.perf_counter()
            oa.logl_grad(olib, obs, theta[:n])
            dt = time.perf_counter() - t0
            legs.append(dict(workload=f"{name}: {what}", path="forward + logL + gradient (FP64 adjoint)", B=n,
                             value=round(n / dt, 2), unit="evals/s", sample=f"one call on {n} vectors, {dt:.2f} s"))
    return legs


def spectrum_leg(steps=20, warmup=3, seed=0):
    """The spectroscopic workload at full size: 1024 live points, 3000-pixel prism
    spectrum (R_fwhm = 100, 5-sigma LSF rows, 128 lines on the pixels); forward + logL
    in FP16 hi + residual and FP32, and the FP32 gradient (P = 158) for the record."""
    import torch

    import paper_2609_30145_amd as sps
    from synth import workloads as wl
    cfg = wl.CONFIGS["c3"]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=("fp32", "fp16"))
    g = wl.make_spectrum_grid(cfg.n_pix)
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002)
    O = sps.Observation(L, "spec", cfg.batch, pix_wave=g["pix_wave"], lsf_mode=g["lsf_mode"],
                        lsf_value=g["lsf_value"], z_ref=float(th_true[0, 1]), sigma_gas_kms=g["sigma_gas_kms"])
    m_true = sps.forward(L, O, torch.tensor(th_true, device="cuda"), "fp32")[0].cpu().numpy()
    d, sg = wl.noisy_spectrum(m_true, seed + 5)
    O.set_data(d, sg)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2), device="cuda")
    out = {"workload": f"{cfg.batch} live points, {cfg.n_pix}-pixel prism spectrum (R_fwhm 100), library "
                       f"{cfg.n_age} x {len(cfg.logz)} x {cfg.n_wave}, {cfg.n_lines} lines"}
    for p in ("fp16", "fp32"):
        dt, tim = time_precision(L, O, theta, p, steps, warmup)
        out[f"forward_{p}_evals_per_s"] = round(cfg.batch * steps / dt, 1)
        out[f"forward_{p}_ms"] = round(1e3 * dt / steps, 4)
    for _ in range(warmup):
        sps.logl_grad(L, O, theta, "fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sps.logl_grad(L, O, theta, "fp32")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["gradient_fp32_evals_per_s"] = round(cfg.batch * steps / dt, 1)
    out["gradient_fp32_ms"] = round(1e3 * dt / steps, 4)
    out["P"] = int(theta.shape[1])
    return out


def nebular_leg(base, steps=20, warmup=3, seed=0):
    """The photometric workload at full size with the nebular continuum cube (7 ages x 5
    Z_gas x 4 log U on the 5994 wavelengths; 26 nebular SSP ages) and the runaway_bc escape
    geometry (f_ob ~ U(0, 1): the ionising rows active): forward + logL throughput at the
    headline precision and FP32, and the time it adds per step to the plain workload."""
    import torch

    import paper_2609_30145_amd as sps
    from synth import workloads as wl
    cfg = wl.CONFIGS["c1"]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    cont = wl.make_nebular_continuum(lib["wave"], seed + 3)
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=("fp32", "fp16"), cont=cont, escape="runaway_bc")
    filters = wl.make_filters(cfg.filters)
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002, escape=True)
    O = sps.Observation(L, "phot", cfg.batch, filters=filters)
    m_true = sps.forward(L, O, torch.tensor(th_true, device="cuda"), "fp32")[0].cpu().numpy()
    d, sg = wl.noisy_photometry(m_true, seed + 5)
    O.set_data(d, sg)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2, escape=True), device="cuda")
    out = {"workload": f"c1 photometry, {cfg.batch} live points, with a nebular continuum cube (7 ages x 5 Z_gas x "
                       f"4 log U, 26 nebular SSP ages) and the runaway_bc escape geometry (f_ob ~ U(0, 1))"}
    for p in ("fp16_wl", "fp32"):
        dt, tim = time_precision(L, O, theta, p, steps, warmup)
        ms = 1e3 * dt / steps
        out[f"{p}_evals_per_s"] = round(cfg.batch * steps / dt, 1)
        out[f"{p}_ms_per_step"] = round(ms, 4)
        if p in base:
            out[f"{p}_added_ms_per_step"] = round(ms - base[p]["ms_per_step"], 4)
    return out


def features_leg(base_spec, base_phot, steps=20, warmup=3, seed=0):
    """The paper's optional stages at full size, each timed as forward + logL on 1024 live
    points, with the time it adds to the plain workload's step:
      - the 3000-pixel prism spectrum with a free stellar velocity dispersion (sigma_gal ~
        U(0, 500) km/s, the Fourier stage), and also with a calibration polynomial of order
        5, marginalised, or with the line fluxes marginalised (FP16 hi + residual, the
        spectroscopic default);
      - the photometric workload under the linear (tent-integral) SFH scheme with the IGM
        (FP16 weight residual, the photometric default);
      - a catalogue of 16 entries (single lines and blends, three upper limits) of the 128
        library lines (no contraction)."""
    import torch

    import paper_2609_30145_amd as sps
    from synth import workloads as wl
    out = {}
    cfg = wl.CONFIGS["c3"]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=("fp16",), sigma_gal_max=500.0)
    g = wl.make_spectrum_grid(cfg.n_pix)
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002, vdisp=500.0)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2, vdisp=500.0), device="cuda")
    for tag, calib in (("spectrum_vdisp", {}),
                       ("spectrum_vdisp_calib", dict(calib="marginal", calib_order=5, calib_prior=np.full(6, 0.1))),
                       ("spectrum_vdisp_linemarg", dict(line_marg="gauss", line_prior_frac=0.3))):
        O = sps.Observation(L, "spec", cfg.batch, pix_wave=g["pix_wave"], lsf_mode=g["lsf_mode"],
                            lsf_value=g["lsf_value"], z_ref=float(th_true[0, 1]), sigma_gas_kms=g["sigma_gas_kms"],
                            **calib)
        m_true = sps.forward(L, O, torch.tensor(th_true, device="cuda"), "fp16")[0].cpu().numpy()
        d, sg = wl.noisy_spectrum(m_true, seed + 5)
        O.set_data(d, sg)
        dt, _ = time_precision(L, O, theta, "fp16", steps, warmup)
        ms = 1e3 * dt / steps
        out[tag] = {"precision": "fp16", "evals_per_s": round(cfg.batch * steps / dt, 1), "ms_per_step": round(ms, 4),
                    "added_ms_per_step": round(ms - base_spec["forward_fp16_ms"], 4) if base_spec else None}
    out["spectrum_vdisp"]["workload"] = (f"{cfg.batch} live points, {cfg.n_pix}-pixel prism spectrum, free sigma_gal "
                                         f"~ U(0, 500) km/s (Fourier stage)")
    out["spectrum_vdisp_calib"]["workload"] = "the same with a marginalised calibration polynomial of order 5"
    out["spectrum_vdisp_linemarg"]["workload"] = ("the same with the line fluxes marginalised (Gaussian priors of 30 "
                                                  "per cent around the grid fluxes)")
    del L, lib
    cfg = wl.CONFIGS["c1"]
    lib = wl.make_library(cfg, seed)
    lines = wl.make_lines(cfg, lib, seed + 1)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=("fp16",), sfh_scheme="linear", igm=True)
    filters = wl.make_filters(cfg.filters)
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002, igm=True, sfh_scheme="linear")
    O = sps.Observation(L, "phot", cfg.batch, filters=filters)
    m_true = sps.forward(L, O, torch.tensor(th_true, device="cuda"), "fp16")[0].cpu().numpy()
    d, sg = wl.noisy_photometry(m_true, seed + 5)
    O.set_data(d, sg)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2, igm=True, sfh_scheme="linear"), device="cuda")
    dt, _ = time_precision(L, O, theta, "fp16_wl", steps, warmup)
    ms = 1e3 * dt / steps
    out["linear_sfh_igm"] = {"workload": f"c1 photometry, {cfg.batch} live points, linear (tent-integral) SFH scheme "
                                         f"and Madau IGM (igm_factor ~ U(0.5, 1.5))",
                             "precision": "fp16_wl", "evals_per_s": round(cfg.batch * steps / dt, 1),
                             "ms_per_step": round(ms, 4),
                             "added_ms_per_step": round(ms - base_phot["ms_per_step"], 4) if base_phot else None}
    del L
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust, lines=lines,
                    precisions=("fp16",))
    blends = [[i] for i in range(0, 120, 12)] + [[3, 4], [20, 21, 22], [40, 41], [60, 61], [80, 81, 82], [100, 101]]
    upper = np.zeros(len(blends), dtype=bool)
    upper[[2, 7, 11]] = True
    O = sps.Observation(L, "lines", cfg.batch, blends=blends, upper=upper)
    th_true = wl.make_theta(cfg, 1, seed=seed + 1002)
    f_true = sps.forward(L, O, torch.tensor(th_true, device="cuda"), "fp16")[0].cpu().numpy()
    O.set_data(f_true * (1.0 + 0.1 * np.random.default_rng(seed + 5).normal(size=f_true.size)), 0.1 * f_true)
    theta = torch.tensor(wl.make_theta(cfg, cfg.batch, seed=seed + 2), device="cuda")
    dt, _ = time_precision(L, O, theta, "fp16_wl", steps, warmup)
    out["lines"] = {"workload": f"{cfg.batch} live points, catalogue of {len(blends)} entries (single lines and "
                                f"blends of the 128 library lines, 3 upper limits)",
                    "precision": "fp16_wl", "evals_per_s": round(cfg.batch * steps / dt, 1),
                    "ms_per_step": round(1e3 * dt / steps, 4)}
    return out


def serve_leg(seconds, rate_hz=50.0, target_load=0.5, seed=0, log=None):
    """Poisson stream of photometry / prism-spectrum fit requests served by sps_server on
    the alpha-enhanced library in FP16.  Capacity is measured first with a saturating
    burst; n_iter is then chosen so that the offered load is ``target_load`` of it."""
    import paper_2609_30145_amd as sps
    from synth import workloads as wl
    log = log or (lambda m: None)
    cfg = wl.CONFIGS["c4"]
    lib = wl.make_library(cfg, seed + 40)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L = sps.Library(lib, n_sfh=cfg.n_sfh, T1=cfg.T1, n_zh=cfg.n_zh, cosmo=cfg.cosmo, dust=dust,
                    precisions=("fp16",))
    del lib
    pool = [wl.make_theta(cfg, 1024, seed=seed + 300 + i) for i in range(8)]
    rng = np.random.default_rng(seed + 9)

    def obs_of(q):
        d = 1e-9 * np.exp(rng.normal(0.0, 0.3, q["size"]))
        if q["kind"] == "phot":
            return dict(filters=wl.make_filters("gaussN", q["size"]), data=d, sigma=0.05 * d)
        g = wl.make_spectrum_grid(q["size"])
        return dict(pix_wave=g["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0, z_ref=float(rng.uniform(0.5, 12)),
                    sigma_gas_kms=100.0, data=d, sigma=0.05 * d)

    def run(reqs, n_iter, paced):
        S = sps.Server(L, precision="fp16", max_points=16384, max_active=256, hbm_budget_bytes=8 << 30)
        tickets, t0, last = [], time.perf_counter(), time.perf_counter()
        for q in reqs:
            if paced:
                dt = q["arrival_s"] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            th = pool[q["id"] % len(pool)][:q["B"]]
            tickets.append(S.submit(q["kind"], th, n_iter=n_iter, seed=q["seed"], **obs_of(q)))
            if time.perf_counter() - last > 5.0:
                last = time.perf_counter()
                log(f"serve: submitted {len(tickets)}/{len(reqs)}")
        states = []
        for t in tickets:
            states.append(S.wait(t, timeout_s=600)["state"])
            S.release(t)
        st = S.stats()
        S.close()
        st["wall_s"] = time.perf_counter() - t0
        st["failed"] = sum(s != "done" for s in states)
        return st

    burst = wl.make_requests(48, rate_hz=1e6, seed=seed + 11)
    cap = run(burst, 8, False)
    log(f"serve: capacity {cap['evals_per_s']:.3g} evals/s ({cap['mean_points_per_tick']:.0f} points/tick)")
    n_req = max(1, int(round(seconds * rate_hz)))
    reqs = wl.make_requests(n_req, rate_hz=rate_hz, seed=seed + 12)
    mean_B = float(np.mean([q["B"] for q in reqs]))
    n_iter = int(max(1, round(target_load * cap["evals_per_s"] / (rate_hz * mean_B) - 1)))
    st = run(reqs, n_iter, True)
    offered = rate_hz * mean_B * (n_iter + 1)
    log(f"serve: {n_req} requests, n_iter {n_iter}, p50/p99 phot {st['p50_latency_s'][0]:.3f}/"
        f"{st['p99_latency_s'][0]:.3f} s spec {st['p50_latency_s'][1]:.3f}/{st['p99_latency_s'][1]:.3f} s")
    r = lambda v: round(float(v), 4)
    return {"workload": f"c4: library {cfg.n_age} ages x {len(cfg.logz)} Z x {len(cfg.afe)} afe x {cfg.n_wave} "
                        f"wavelengths in fp16 (+residual); Poisson {rate_hz:g} req/s for {seconds:g} s; 50/50 "
                        f"photometry (8-25 bands) / prism (400-3000 px); B_r in 64..1024",
            "requests": n_req, "n_iter": n_iter, "evals_per_request_mean": r(mean_B * (n_iter + 1)),
            "capacity_evals_per_s": r(cap["evals_per_s"]), "offered_evals_per_s": r(offered),
            "offered_load": r(offered / cap["evals_per_s"]),
            "evals_per_s_busy": r(st["evals_per_s"]), "evals_per_s_wall": r(st["evals"] / st["wall_s"]),
            "p50_latency_s": {"phot": r(st["p50_latency_s"][0]), "spec": r(st["p50_latency_s"][1])},
            "p99_latency_s": {"phot": r(st["p99_latency_s"][0]), "spec": r(st["p99_latency_s"][1])},
            "completed": {"phot": st["completed_by_kind"][0], "spec": st["completed_by_kind"][1]},
            "failed": st["failed"], "rejected": st["rejected"], "mean_points_per_tick": r(st["mean_points_per_tick"]),
            "mean_admission_wait_s": r(st["mean_queue_s"]), "max_admission_wait_s": r(st["max_queue_s"]),
            "hbm_peak_bytes": st["hbm_peak"], "hbm_budget_bytes": st["hbm_budget"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp16_wl",
                    help="contraction variant of the timed step (default: FP16 with one weight-residual pass, "
                         "the cheapest variant that meets the photometric bounds)")
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--also", default="fp16,fp32,bf16", help="other precisions timed for the record")
    ap.add_argument("--no-spectrum", action="store_true", help="skip the spectroscopic leg")
    ap.add_argument("--no-small-batch", action="store_true", help="skip the 64-point leg")
    ap.add_argument("--no-nebular", action="store_true", help="skip the nebular-continuum / escape leg")
    ap.add_argument("--no-features", action="store_true",
                    help="skip the leg of optional stages (sigma_gal, calibration, linear SFH + IGM, lines)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB 5 times (HBM counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the Poisson request stream of the serving leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 18
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}))
        return
    precs = [args.precision] + [p for p in args.also.split(",") if p and p != args.precision]
    cfg, lib, lines, dust, L, O, theta = build_workload(args.workload, tuple(precs))
    B = theta.shape[0]
    K_dense = cfg.n_age * len(cfg.logz) * len(cfg.afe)
    N = cfg.n_wave
    flop_per_eval = 2.0 * K_dense * N          # dense sum over the SSP grid (eq. 1)
    results = {}
    for p in precs:
        steps = args.steps if p == args.precision else max(10, args.steps // 5)
        dt, tim = time_precision(L, O, theta, p, steps, args.warmup)
        avg_ms = tim["ms_total"] / max(1, tim["launches"])
        frac_exec = tim["executed_k_tiles"] / max(1, tim["dense_k_tiles"])
        K_pad = L.info["K_pad"]
        exec_flops = 2.0 * B_pad(B) * K_pad * L.info["N_pad"] * frac_exec * MFMA_PASSES[p]
        results[p] = dict(ms_per_step=1e3 * dt / steps, evals_per_s=B * steps / dt, contract_ms=avg_ms,
                          contract_alg_tflops=flop_per_eval * B / (avg_ms * 1e-3) / 1e12,
                          contract_exec_tflops=exec_flops / (avg_ms * 1e-3) / 1e12,
                          active_k_tile_frac=frac_exec, steps=steps)
    main_r = results[args.precision]
    peak = PEAK_TFLOPS[args.precision]
    tr = traffic_record(args.precision)
    roof = {"bound": "mfma", "achieved": round(main_r["contract_alg_tflops"], 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(main_r["contract_alg_tflops"] / peak, 4),
            "traffic": tr["bytes"] if tr else None,
            "traffic_unit": "bytes per launch (HBM-side counters scaled by a copy probe)",
            "traffic_source": tr["source"] if tr else None,
            "alg_bytes_per_launch": alg_bytes(cfg, B, args.precision),
            "executed_mfma_tflops": round(main_r["contract_exec_tflops"], 3),
            "executed_frac": round(main_r["contract_exec_tflops"] / peak, 4),
            "kernel": "library contraction (k_contract)", "contract_ms": round(main_r["contract_ms"], 4),
            "alg_flop_per_eval": flop_per_eval, "active_k_tile_frac": round(main_r["active_k_tile_frac"], 4)}
    out = {
        "metric": "forward-model evals/s at 1024 live pts (low-prec vs FP32 plain); served p50/p99",
        "value": round(main_r["evals_per_s"], 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": main_r["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded SSP library, filters, line tables and parameter draws)",
        "config": {"workload": f"{args.workload}: {B} live points, library {cfg.n_age} ages x {len(cfg.logz)} Z x "
                               f"{len(cfg.afe)} afe x {N} wavelengths, {cfg.n_sfh}-bin SFH, {cfg.n_zh}-node ZH, "
                               f"two-component dust, {cfg.n_lines} lines, photometry ({cfg.filters})",
                   "batch": B, "precision": args.precision},
        "roofline": roof,
        "by_precision": {p: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                         for p, r in results.items()},
    }
    # the HBM-bound regime: a batch of 64 points streams the whole library for few flops
    if not args.no_small_batch:
        nb, st64 = 64, max(20, args.steps // 2)
        dt64, tim64 = time_precision(L, O, theta[:nb], args.precision, st64, args.warmup)
        ms64 = tim64["ms_total"] / max(1, tim64["launches"])
        b64 = alg_bytes(cfg, nb, args.precision)
        out["small_batch"] = {"batch": nb, "precision": args.precision,
                              "ms_per_step": round(1e3 * dt64 / st64, 4),
                              "evals_per_s": round(nb * st64 / dt64, 1),
                              "contract_ms": round(ms64, 4), "alg_bytes_per_launch": b64,
                              "contract_achieved_GBps": round(b64 / (ms64 * 1e-3) / 1e9, 1),
                              "hbm_peak_GBps": 8000.0,
                              "hbm_frac": round(b64 / (ms64 * 1e-3) / 8e12, 4)}
    if not args.no_spectrum:
        out["spectrum"] = spectrum_leg()
    if not args.no_nebular and args.workload == "c1":
        out["nebular"] = nebular_leg(results)
    if not args.no_features and args.workload == "c1":
        out["features"] = features_leg(out.get("spectrum"), results.get("fp16_wl"))
    if args.serve_seconds > 0:
        out["serving"] = serve_leg(args.serve_seconds, log=lambda m: print(m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


def alg_bytes(cfg, B, precision):
    """Minimum bytes of one contraction launch: the library once (both 16-bit planes, or
    the FP32/FP64 copy), the weight rows and the rest-frame output."""
    K = cfg.n_age * len(cfg.logz) * len(cfg.afe) + cfg.n_lines
    N = cfg.n_wave
    suffix = precision.split("_")[1] if "_" in precision else ""
    # bytes per library element and per weight: both 16-bit planes where a pass reads them
    lib = {"fp64": 8, "fp32": 4}.get(precision, 4 if suffix in ("", "hr") else 2)
    w = {"fp64": 8, "fp32": 4}.get(precision, 4 if suffix in ("", "wl") else 2)
    out = 8 if precision == "fp64" else 4
    return int(K * N * lib + B * K * w + B * N * out)


def B_pad(B):
    return (B + 127) // 128 * 128


if __name__ == "__main__":
    main()
