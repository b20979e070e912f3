"""ctypes binding of libsps.so (include/sps.h).  Argument marshalling only: every step
of the forward model, likelihood and gradient runs in the gfx950 kernels.

PyTorch provides device memory and streams: theta/outputs are CUDA (HIP) tensors
whose data pointers are passed to the C ABI, and calls are enqueued on the
current torch stream unless another stream is given.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsps.so")

SPS_OK, SPS_PENDING = 0, 1
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "bf16_1pass": 4, "fp16_1pass": 5,
              "bf16_hr": 6, "fp16_hr": 7, "bf16_wl": 8, "fp16_wl": 9}
LSF_MODES = {"R_fwhm": 0, "R_sigma": 1, "fwhm_aa": 2, "sigma_aa": 3, "sigma_kms": 4, "fwhm_kms": 5, "R": 6}
NOISE = {"err_scale": 1, "f_calib": 2, "f_data": 4, "jitter": 8}
OBS_PHOT, OBS_SPEC, OBS_LINES = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class LibraryDesc(C.Structure):
    _fields_ = [("n_age", C.c_int32), ("n_z", C.c_int32), ("n_afe", C.c_int32), ("n_wave", C.c_int32),
                ("ages", _dp), ("logz", _dp), ("afe", _dp), ("wave", _dp), ("flux", _dp),
                ("t_young", C.c_double), ("n_sfh", C.c_int32), ("T1", C.c_double), ("n_zh", C.c_int32),
                ("H0", C.c_double), ("Om", C.c_double), ("dust_a", _dp), ("dust_d", _dp),
                ("n_line", C.c_int32), ("n_zg", C.c_int32), ("n_u", C.c_int32),
                ("line_wave", _dp), ("line_table", _dp), ("zg_nodes", _dp), ("u_nodes", _dp),
                ("precisions", C.c_uint32), ("device", C.c_int32),
                ("n_line_tau", C.c_int32), ("line_tau", _dp),
                ("n_cont_tau", C.c_int32), ("n_cont_zg", C.c_int32), ("n_cont_u", C.c_int32),
                ("cont_tau", _dp), ("cont_zg", _dp), ("cont_u", _dp), ("cont_table", _dp),
                ("escape", C.c_int32), ("sfh_scheme", C.c_int32), ("igm", C.c_int32),
                ("sigma_gal_max", C.c_double)]

ESCAPE = {"none": 0, "runaway_bc": 1, "picket": 2}
SFH_SCHEMES = {"step": 0, "linear": 1}


class LibraryInfo(C.Structure):
    _fields_ = [("K", C.c_int32), ("K_pad", C.c_int32), ("K_young_pad", C.c_int32), ("N", C.c_int32),
                ("N_pad", C.c_int32), ("n_young", C.c_int32), ("n_line", C.c_int32),
                ("device_bytes", C.c_int64)]


class Layout(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "P", "n_scalar", "sfh", "n_sfh", "zh", "n_zh", "logmass", "zred", "tau_bc", "alpha_bc", "tau_diff",
        "delta", "logzsol", "gas_logz", "gas_logu", "afe", "log_err_scale", "log_f_calib", "log_f_data",
        "log_jitter", "frac_obrun", "igm_factor", "sigma_gal", "x_hi", "log_nhi", "z_dla")]


class ObsDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_band", C.c_int32), ("filter_len", _ip), ("filter_wave", _dp),
                ("filter_trans", _dp), ("n_pix", C.c_int32), ("pix_wave", _dp), ("lsf_mode", C.c_int32),
                ("lsf_value", C.c_double), ("lsf_curve", _dp), ("z_ref", C.c_double),
                ("sigma_gal_kms", C.c_double), ("sigma_gas_kms", C.c_double), ("data", _dp), ("sigma", _dp),
                ("mask", _u8p), ("noise_flags", C.c_uint32), ("max_batch", C.c_int32),
                ("calib_mode", C.c_int32), ("calib_order", C.c_int32), ("calib_prior", _dp),
                ("line_len", _ip), ("line_index", _ip), ("upper", _u8p),
                ("line_marg", C.c_int32), ("line_prior_frac", C.c_double), ("line_flat", _u8p)]

CALIB = {None: 0, "marginal": 1, "optimise": 2}
LINEMARG = {None: 0, "gauss": 1, "flat": 2}


class SpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sps error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libsps.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_30145_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sps_library_load.argtypes = [C.POINTER(LibraryDesc), C.POINTER(vp)]
        L.sps_library_info_get.argtypes = [vp, C.POINTER(LibraryInfo)]
        L.sps_library_destroy.argtypes = [vp]
        L.sps_library_destroy.restype = None
        L.sps_theta_layout.argtypes = [vp, C.POINTER(Layout)]
        L.sps_obs_create.argtypes = [vp, C.POINTER(ObsDesc), C.POINTER(vp), C.POINTER(C.c_uint32)]
        L.sps_obs_set_data.argtypes = [vp, _dp, _dp, _u8p]
        L.sps_obs_n_data.argtypes = [vp]
        L.sps_obs_destroy.argtypes = [vp]
        L.sps_obs_destroy.restype = None
        L.sps_forward.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp, vp]
        L.sps_logl.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
        L.sps_logl_grad.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
        L.sps_logl_static.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
        L.sps_logl_lines_joint.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_int32, vp, vp]
        L.sps_obs_enable_timing.argtypes = [vp, C.c_int32]
        L.sps_obs_contract_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                              C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sps_last_error.restype = C.c_char_p
        L.sps_version.restype = C.c_char_p
        for name in ("sps_library_load", "sps_library_info_get", "sps_theta_layout", "sps_obs_create",
                     "sps_obs_set_data", "sps_obs_n_data", "sps_forward", "sps_logl", "sps_logl_grad", "sps_logl_static",
                     "sps_logl_lines_joint", "sps_obs_enable_timing", "sps_obs_contract_timing"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def check(code):
    if code < 0:
        raise SpsError(code, lib().sps_last_error().decode())
    return code


def _arr(x, dtype=np.float64):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def _ptr(a, ctype=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Library:
    """Device-resident SSP library and model configuration (sps_library_load)."""

    def __init__(self, lib_arrays: dict, n_sfh: int, T1: float, n_zh: int, cosmo=(70.0, 0.3),
                 dust: dict | None = None, lines: dict | None = None, precisions=("fp32",), device: int = 0,
                 cont: dict | None = None, escape: str = "none", sfh_scheme: str = "step", igm: int = 0,
                 sigma_gal_max: float = 0.0):
        """``device=-1`` loads a host-only library (layout and observation operators; used by
        the mock server executor).  ``lines`` may carry ``line_tau`` (the table's own age axis);
        ``cont`` is a nebular continuum cube (cont_table [tau][zg][u][wave], tau_nodes,
        zg_nodes, u_nodes); ``escape`` is "none", "runaway_bc" or "picket"; ``sfh_scheme`` is
        "step" or "linear"; ``igm`` the IGM transmission: True or 1 (Madau), 3 (+ damping wing), 5
        (+ damped absorber) or 7 (both); ``sigma_gal_max`` > 0
        adds a free stellar velocity dispersion column (km/s, Fourier stage)."""
        L = lib()
        keep = []
        ages, logz, wave = _arr(lib_arrays["ages"]), _arr(lib_arrays["logz"]), _arr(lib_arrays["wave"])
        afe = _arr(lib_arrays.get("afe", [0.0]))
        flux = _arr(lib_arrays["flux"])
        keep += [ages, logz, wave, afe, flux]
        d = LibraryDesc()
        d.n_age, d.n_z, d.n_afe, d.n_wave = len(ages), len(logz), len(afe), len(wave)
        if flux.shape != (d.n_afe, d.n_z, d.n_age, d.n_wave):
            raise ValueError(f"flux shape {flux.shape} != {(d.n_afe, d.n_z, d.n_age, d.n_wave)}")
        d.ages, d.logz, d.wave, d.flux = _ptr(ages), _ptr(logz), _ptr(wave), _ptr(flux)
        d.afe = _ptr(afe) if d.n_afe > 1 else None
        d.t_young = float(lib_arrays.get("t_young", 1e7))
        d.n_sfh, d.T1, d.n_zh = int(n_sfh), float(T1), int(n_zh)
        d.H0, d.Om = float(cosmo[0]), float(cosmo[1])
        if dust is not None:
            da, dd = _arr(dust["dust_a"]), _arr(dust["dust_d"])
            keep += [da, dd]
            d.dust_a, d.dust_d = _ptr(da), _ptr(dd)
        if lines is not None:
            lw, lt = _arr(lines["line_wave"]), _arr(lines["line_table"])
            zg, un = _arr(lines["zg_nodes"]), _arr(lines["u_nodes"])
            keep += [lw, lt, zg, un]
            d.n_line, d.n_zg, d.n_u = len(lw), len(zg), len(un)
            d.line_wave, d.line_table, d.zg_nodes, d.u_nodes = _ptr(lw), _ptr(lt), _ptr(zg), _ptr(un)
            if lines.get("line_tau") is not None:
                ltau = _arr(lines["line_tau"])
                keep.append(ltau)
                d.n_line_tau, d.line_tau = len(ltau), _ptr(ltau)
        if cont is not None:
            ct, cz, cu = _arr(cont["tau_nodes"]), _arr(cont["zg_nodes"]), _arr(cont["u_nodes"])
            cc = _arr(cont["cont_table"])
            if cc.shape != (len(ct), len(cz), len(cu), d.n_wave):
                raise ValueError(f"cont_table shape {cc.shape} != {(len(ct), len(cz), len(cu), d.n_wave)}")
            keep += [ct, cz, cu, cc]
            d.n_cont_tau, d.n_cont_zg, d.n_cont_u = len(ct), len(cz), len(cu)
            d.cont_tau, d.cont_zg, d.cont_u, d.cont_table = _ptr(ct), _ptr(cz), _ptr(cu), _ptr(cc)
        d.escape = ESCAPE[escape]
        d.sfh_scheme = SFH_SCHEMES[sfh_scheme]
        d.igm = int(igm)
        d.sigma_gal_max = float(sigma_gal_max)
        mask = 0
        for p in precisions:
            mask |= 1 << PRECISIONS[p]
        d.precisions = mask
        d.device = device
        h = C.c_void_p()
        check(L.sps_library_load(C.byref(d), C.byref(h)))
        self.handle = h
        self.n_sfh, self.n_zh = n_sfh, n_zh
        lay = Layout()
        check(L.sps_theta_layout(h, C.byref(lay)))
        self.layout = {n: getattr(lay, n) for n, _ in Layout._fields_}
        info = LibraryInfo()
        check(L.sps_library_info_get(h, C.byref(info)))
        self.info = {n: getattr(info, n) for n, _ in LibraryInfo._fields_}

    @property
    def P(self):
        return self.layout["P"]

    def close(self):
        if getattr(self, "handle", None):
            lib().sps_library_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Observation:
    """Photometry, a spectrum or an emission-line catalogue bound to a library (sps_obs_create).

    Spectra take ``calib`` ("marginal" or "optimise"), ``calib_order`` and ``calib_prior``
    for the calibration polynomial, or ``line_marg`` ("gauss" or "flat"),
    ``line_prior_frac`` and ``line_flat`` to marginalise the line fluxes; a line catalogue ("lines") takes ``blends`` (per entry,
    the library line indices it sums) and ``upper`` (per entry, an upper-limit flag)."""

    def __init__(self, library: Library, kind: str, max_batch: int, filters=None, pix_wave=None,
                 lsf_mode="R_fwhm", lsf_value=100.0, lsf_curve=None, z_ref=0.0, sigma_gal_kms=0.0,
                 sigma_gas_kms=0.0, data=None, sigma=None, mask=None, noise=(), calib=None, calib_order=0,
                 calib_prior=None, blends=None, upper=None, line_marg=None, line_prior_frac=0.0, line_flat=None):
        L = lib()
        self.library = library
        keep = []
        d = ObsDesc()
        d.kind = {"phot": OBS_PHOT, "spec": OBS_SPEC, "lines": OBS_LINES}.get(kind, 99)
        if kind == "lines":
            ln = _arr([len(bl) for bl in blends], np.int32)
            li = _arr(np.concatenate([np.asarray(bl, dtype=np.int32) for bl in blends]), np.int32)
            keep += [ln, li]
            d.n_band, d.line_len, d.line_index = len(blends), _ptr(ln, C.c_int32), _ptr(li, C.c_int32)
            if upper is not None:
                up = _arr(upper, np.uint8)
                keep.append(up)
                d.upper = _ptr(up, C.c_uint8)
            self.n_data = len(blends)
        elif kind == "phot":
            lens = _arr([len(f[0]) for f in filters], np.int32)
            fw = _arr(np.concatenate([f[0] for f in filters]))
            ft = _arr(np.concatenate([f[1] for f in filters]))
            keep += [lens, fw, ft]
            d.n_band, d.filter_len, d.filter_wave, d.filter_trans = len(filters), _ptr(lens, C.c_int32), \
                _ptr(fw), _ptr(ft)
            self.n_data = len(filters)
        else:
            pw = _arr(pix_wave)
            keep.append(pw)
            d.n_pix, d.pix_wave = len(pw), _ptr(pw)
            d.lsf_mode = LSF_MODES[lsf_mode]
            d.lsf_value = float(lsf_value)
            if lsf_curve is not None:
                lc = _arr(lsf_curve)
                keep.append(lc)
                d.lsf_curve = _ptr(lc)
            d.z_ref, d.sigma_gal_kms, d.sigma_gas_kms = float(z_ref), float(sigma_gal_kms), float(sigma_gas_kms)
            d.calib_mode = CALIB[calib]
            if calib is not None:
                cp = _arr(calib_prior)
                keep.append(cp)
                d.calib_order, d.calib_prior = int(calib_order), _ptr(cp)
            d.line_marg = LINEMARG[line_marg]
            d.line_prior_frac = float(line_prior_frac)
            if line_flat is not None:
                lf = _arr(line_flat, np.uint8)
                keep.append(lf)
                d.line_flat = _ptr(lf, C.c_uint8)
            self.n_data = len(pw)
        if data is not None:
            da, sg = _arr(data), _arr(sigma)
            keep += [da, sg]
            d.data, d.sigma = _ptr(da), _ptr(sg)
            if mask is not None:
                mk = _arr(mask, np.uint8)
                keep.append(mk)
                d.mask = _ptr(mk, C.c_uint8)
        flags = 0
        for n in noise:
            flags |= NOISE[n]
        d.noise_flags = flags
        d.max_batch = int(max_batch)
        h = C.c_void_p()
        warn = C.c_uint32(0)
        check(L.sps_obs_create(library.handle, C.byref(d), C.byref(h), C.byref(warn)))
        self.handle = h
        self.warnings = warn.value
        self.max_batch = max_batch

    def set_data(self, data, sigma, mask=None):
        da, sg = _arr(data), _arr(sigma)
        mk = None if mask is None else _arr(mask, np.uint8)
        check(lib().sps_obs_set_data(self.handle, _ptr(da), _ptr(sg), _ptr(mk, C.c_uint8)))

    def enable_timing(self, on=True):
        check(lib().sps_obs_enable_timing(self.handle, 1 if on else 0))

    def contract_timing(self):
        ms, n, ex, de = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().sps_obs_contract_timing(self.handle, C.byref(ms), C.byref(n), C.byref(ex), C.byref(de)))
        return dict(ms_total=ms.value, launches=n.value, executed_k_tiles=ex.value, dense_k_tiles=de.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().sps_obs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_theta(library, theta):
    import torch
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.is_contiguous()):
        raise ValueError("theta must be a contiguous float64 CUDA tensor")
    if theta.dim() != 2 or theta.shape[1] != library.P:
        raise ValueError(f"theta must be [B, {library.P}]")


def forward(library, obs, theta, precision="fp32", stream=None):
    """Model observables [B, n_data] (float64, maggies) — sps_forward."""
    import torch
    _check_theta(library, theta)
    out = torch.empty((theta.shape[0], obs.n_data), dtype=torch.float64, device=theta.device)
    check(lib().sps_forward(library.handle, obs.handle, C.c_void_p(theta.data_ptr()), theta.shape[0],
                            PRECISIONS[precision], C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def logl(library, obs, theta, precision="fp32", stream=None, return_model=False):
    """logL [B] (float64) — sps_logl."""
    import torch
    _check_theta(library, theta)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    model = None
    if return_model:
        model = torch.empty((theta.shape[0], obs.n_data), dtype=torch.float64, device=theta.device)
    check(lib().sps_logl(library.handle, obs.handle, C.c_void_p(theta.data_ptr()), theta.shape[0],
                         PRECISIONS[precision], C.c_void_p(out.data_ptr()),
                         C.c_void_p(model.data_ptr()) if model is not None else None, _stream_ptr(stream)))
    return (out, model) if return_model else out


def logl_static(library, obs, theta, precision="fp32", stream=None, return_model=False):
    """logL [B] (float64) through the allocation-free entry point — sps_logl_static."""
    import torch
    _check_theta(library, theta)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    model = None
    if return_model:
        model = torch.empty((theta.shape[0], obs.n_data), dtype=torch.float64, device=theta.device)
    check(lib().sps_logl_static(library.handle, obs.handle, C.c_void_p(theta.data_ptr()), theta.shape[0],
                                PRECISIONS[precision], C.c_void_p(out.data_ptr()),
                                C.c_void_p(model.data_ptr()) if model is not None else None, _stream_ptr(stream)))
    return (out, model) if return_model else out


def logl_lines_joint(library, spec, theta, cat=None, phot=None, precision="fp32", stream=None):
    """logL [B] (float64) of a spectrum with a line catalogue and/or a photometric
    observation of the same object, the line fluxes marginalised jointly —
    sps_logl_lines_joint."""
    import torch
    _check_theta(library, theta)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    check(lib().sps_logl_lines_joint(library.handle, spec.handle, cat.handle if cat is not None else None,
                                     phot.handle if phot is not None else None, C.c_void_p(theta.data_ptr()),
                                     theta.shape[0], PRECISIONS[precision], C.c_void_p(out.data_ptr()),
                                     _stream_ptr(stream)))
    return out


def logl_grad(library, obs, theta, precision="fp32", stream=None):
    """(logL [B], dlogL/dtheta [B, P]) — sps_logl_grad."""
    import torch
    _check_theta(library, theta)
    out = torch.empty(theta.shape[0], dtype=torch.float64, device=theta.device)
    grad = torch.empty_like(theta)
    check(lib().sps_logl_grad(library.handle, obs.handle, C.c_void_p(theta.data_ptr()), theta.shape[0],
                              PRECISIONS[precision], C.c_void_p(out.data_ptr()), C.c_void_p(grad.data_ptr()),
                              _stream_ptr(stream)))
    return out, grad


# ---------------------------------------------------------------------------------
# Request server (include/sps_server.h)
# ---------------------------------------------------------------------------------
class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_points", C.c_int32), ("max_active", C.c_int32),
                ("precision", C.c_int32), ("device", C.c_int32), ("mock_eval_ns", C.c_double)]


class Request(C.Structure):
    _fields_ = [("obs", ObsDesc), ("B", C.c_int32), ("theta0", _dp), ("n_iter", C.c_int32), ("seed", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("B", C.c_int32), ("P", C.c_int32), ("kind", C.c_int32),
                ("theta", _dp), ("logl", _dp), ("queue_s", C.c_double), ("latency_s", C.c_double),
                ("evals", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("cancelled", C.c_int64), ("active", C.c_int64), ("pending", C.c_int64), ("ticks", C.c_int64),
                ("evals", C.c_int64), ("busy_s", C.c_double), ("evals_per_s", C.c_double),
                ("mean_points_per_tick", C.c_double), ("p50_latency_s", C.c_double * 2),
                ("p99_latency_s", C.c_double * 2), ("completed_by_kind", C.c_int64 * 2),
                ("mean_queue_s", C.c_double), ("max_queue_s", C.c_double), ("hbm_in_use", C.c_int64),
                ("hbm_peak", C.c_int64), ("hbm_budget", C.c_int64)]


REQ_STATES = {0: "pending", 1: "active", 2: "done", 3: "cancelled", 4: "failed"}


def _server_lib():
    L = lib()
    if not getattr(L, "_server_bound", False):
        vp = C.c_void_p
        L.sps_server_create.argtypes = [vp, C.POINTER(ServerDesc), C.POINTER(vp)]
        L.sps_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.sps_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result)]
        L.sps_wait.argtypes = [vp, C.c_uint64, C.c_int64, C.POINTER(Result)]
        L.sps_cancel.argtypes = [vp, C.c_uint64]
        L.sps_release.argtypes = [vp, C.c_uint64]
        L.sps_server_stats.argtypes = [vp, C.POINTER(Stats)]
        L.sps_server_destroy.argtypes = [vp]
        L.sps_server_destroy.restype = None
        for n in ("sps_server_create", "sps_submit", "sps_poll", "sps_wait", "sps_cancel", "sps_release",
                  "sps_server_stats"):
            getattr(L, n).restype = C.c_int32
        L._server_bound = True
    return L


def _obs_desc(kind, filters=None, pix_wave=None, lsf_mode="R_fwhm", lsf_value=100.0, z_ref=0.0,
              sigma_gal_kms=0.0, sigma_gas_kms=0.0, data=None, sigma=None, noise=(), keep=None):
    d = ObsDesc()
    d.kind = OBS_PHOT if kind == "phot" else OBS_SPEC
    if kind == "phot":
        lens = _arr([len(f[0]) for f in filters], np.int32)
        fw = _arr(np.concatenate([f[0] for f in filters]))
        ft = _arr(np.concatenate([f[1] for f in filters]))
        keep += [lens, fw, ft]
        d.n_band, d.filter_len, d.filter_wave, d.filter_trans = len(filters), _ptr(lens, C.c_int32), _ptr(fw), \
            _ptr(ft)
    else:
        pw = _arr(pix_wave)
        keep.append(pw)
        d.n_pix, d.pix_wave, d.lsf_mode, d.lsf_value = len(pw), _ptr(pw), LSF_MODES[lsf_mode], float(lsf_value)
        d.z_ref, d.sigma_gal_kms, d.sigma_gas_kms = float(z_ref), float(sigma_gal_kms), float(sigma_gas_kms)
    if data is not None:
        da, sg = _arr(data), _arr(sigma)
        keep += [da, sg]
        d.data, d.sigma = _ptr(da), _ptr(sg)
    flags = 0
    for n in noise:
        flags |= NOISE[n]
    d.noise_flags = flags
    return d


class Server:
    """Continuous-batching request server (sps_server_*).  ``device=-1`` selects the
    host-only mock executor, which needs no GPU (scheduler tests)."""

    def __init__(self, library, hbm_budget_bytes=8 << 30, max_points=16384, max_active=256, precision="fp16",
                 device=0, mock_eval_ns=0.0):
        L = _server_lib()
        d = ServerDesc(int(hbm_budget_bytes), int(max_points), int(max_active), PRECISIONS[precision], int(device),
                       float(mock_eval_ns))
        h = C.c_void_p()
        check(L.sps_server_create(library.handle, C.byref(d), C.byref(h)))
        self.handle = h
        self.library = library

    def submit(self, kind, theta0, n_iter, seed, **obs):
        keep = []
        th = _arr(theta0)
        keep.append(th)
        q = Request()
        q.obs = _obs_desc(kind, keep=keep, **obs)
        q.B = th.shape[0]
        q.theta0 = _ptr(th)
        q.n_iter = int(n_iter)
        q.seed = int(seed)
        t = C.c_uint64()
        check(_server_lib().sps_submit(self.handle, C.byref(q), C.byref(t)))
        return t.value

    @staticmethod
    def _result(r):
        out = dict(state=REQ_STATES[r.state], B=r.B, P=r.P, kind=("phot", "spec")[r.kind], queue_s=r.queue_s,
                   latency_s=r.latency_s, evals=r.evals)
        if r.state == 2:
            out["theta"] = np.ctypeslib.as_array(r.theta, shape=(r.B * r.P,)).reshape(r.B, r.P).copy()
            out["logl"] = np.ctypeslib.as_array(r.logl, shape=(r.B,)).copy()
        return out

    def poll(self, ticket):
        r = Result()
        code = check(_server_lib().sps_poll(self.handle, ticket, C.byref(r)))
        return None if code == SPS_PENDING else self._result(r)

    def wait(self, ticket, timeout_s=None):
        r = Result()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        check(_server_lib().sps_wait(self.handle, ticket, us, C.byref(r)))
        return self._result(r)

    def cancel(self, ticket):
        check(_server_lib().sps_cancel(self.handle, ticket))

    def release(self, ticket):
        check(_server_lib().sps_release(self.handle, ticket))

    def stats(self):
        s = Stats()
        check(_server_lib().sps_server_stats(self.handle, C.byref(s)))
        out = {n: getattr(s, n) for n, _ in Stats._fields_}
        for k in ("p50_latency_s", "p99_latency_s", "completed_by_kind"):
            out[k] = list(out[k])
        return out

    def close(self):
        if getattr(self, "handle", None):
            _server_lib().sps_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
