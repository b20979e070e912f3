"""Pins for the oracle's full nebular grid evaluation and ionising-photon escape
(Sec. 2.3.1-2.3.2, App. C, App. D.1): trilinear cubes, the nebular continuum
Q_ma 10^Chat, the nebular age range, and the runaway_bc / picket geometries of f_ob.

Each pin is fixed by something outside the code under test: functions that trilinear
interpolation reproduces exactly, brute-force sums over the raw SSP grid, the escape
fractions eq. fesc_runaway and the picket fence state, and limits (f_ob = 0, f_ob = 1)
that reduce to models without nebular emission.
"""
import math

import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import model as om
from oracle import nebular
from oracle.constants import ANG_CM, C_CMS, LSUN
from synth import workloads as wl

CFG = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.5, -1.5, -0.5, 0.5), n_wave=1500,
                 n_sfh=12, n_zh=4, n_lines=8)


def _multilinear(z, t, u):
    # every product of the three coordinates appears: trilinear interpolation on any grid
    # reproduces this function exactly inside the grid
    return -24.0 + 0.4 * z - 0.3 * t + 0.2 * u + 0.15 * z * t - 0.1 * t * u + 0.05 * z * u + 0.02 * z * t * u


@pytest.fixture(scope="module")
def parts():
    lib = wl.make_library(CFG, 0)
    lines = wl.make_lines(CFG, lib, 1, line_tau=wl.LINE_TAU)
    cont = wl.make_nebular_continuum(lib["wave"], 3)
    dust = wl.make_dust_tables(CFG, lib["wave"])
    return lib, lines, cont, dust


def _dark(cont, wave):
    # the cube with no nebular continuum at all below the Lyman limit (10^-300), so that the
    # emergent ionising flux is the stars' alone
    cube = cont["cont_table"].copy()
    cube[..., wave < 912.0] = -300.0
    return dict(cont, cont_table=cube)


def test_trilinear_reproduces_a_trilinear_function_and_clamps():
    zg = np.array([-2.0, -1.1, -0.2, 0.4])
    tau = np.array([5e5, 1e6, 2e6, 3.5e6, 1e7]) / 1e6     # unequal spacings on every axis
    uu = np.array([-4.0, -3.0, -1.5])
    cube = _multilinear(zg[:, None, None], tau[None, :, None], uu[None, None, :])
    rng = np.random.default_rng(0)
    for _ in range(50):
        z, t, u = rng.uniform(-2.0, 0.4), rng.uniform(0.5, 10.0), rng.uniform(-4.0, -1.5)
        got = nebular.trilinear(cube, zg, tau, uu, z, t, u)
        assert got == pytest.approx(_multilinear(z, t, u), rel=1e-13, abs=0.0)
    # outside the grid each coordinate is clamped to its end node
    got = nebular.trilinear(cube, zg, tau, uu, 3.0, 0.1, -9.0)
    assert got == pytest.approx(_multilinear(0.4, 0.5, -4.0), rel=1e-13, abs=0.0)


def test_line_cube_on_birth_cloud_ages_is_the_bilinear_table(parts):
    lib = parts[0]
    ny = int(np.sum(lib["ages"] < CFG.t_young))
    legacy = wl.make_lines(CFG, lib, 1)
    for gz, gu in ((-0.7, -2.2), (0.3, -1.0), (-1.3, -4.0)):
        ref = nebular.line_table_interp(legacy["line_table"], legacy["zg_nodes"], legacy["u_nodes"], gz, gu)
        got = nebular.line_table_at_ages(legacy["line_table"], legacy["zg_nodes"], lib["ages"][:ny],
                                         legacy["u_nodes"], gz, gu, lib["ages"][:ny])
        assert np.array_equal(got, ref)


def test_nebular_ages_are_the_overlap_of_the_cube_age_ranges(parts):
    lib, lines, cont, dust = parts
    c2 = dict(cont, tau_nodes=np.array([2e6, 3e6, 4e6, 6e6]), cont_table=cont["cont_table"][:4])
    l2 = dict(lines, line_tau=np.array([1.5e6, 3e6, 5e6, 8e6]), line_table=lines["line_table"][:, :4])
    L = om.build_library(CFG, lib, l2, dust, cont=c2)
    ages = lib["ages"]
    inside = [a for a in range(len(ages)) if 2e6 <= ages[a] <= 6e6]
    assert (L.neb_a0, L.n_neb) == (inside[0], inside[-1] + 1)
    assert inside[0] > 0
    ion = lib["wave"] < 912.0
    for a in range(len(ages)):
        if a in inside:
            assert np.all(L.flux[:, :, a][..., ion] == 0.0)
        else:
            assert np.array_equal(L.flux[:, :, a], lib["flux"][:, :, a])
    # a burst at an age outside the range has no nebular emission
    th = wl.make_theta(CFG, 1, seed=3)[0]
    cols = om.columns(CFG.n_sfh, CFG.n_zh)
    W = np.zeros_like(lib["flux"][..., 0])
    W[0, 1, inside[0] - 1] = 1.0
    assert np.all(om.point_continuum(L, th, cols, W) == 0.0)
    assert np.all(om.point_lines(L, th, cols, W)[0] == 0.0)
    # the cubes' ages must be birth-cloud ages
    c3 = dict(cont, tau_nodes=np.array([2e6, 3e6, 5e7]), cont_table=cont["cont_table"][:3])
    with pytest.raises(ValueError):
        om.build_library(CFG, lib, None, dust, cont=c3)


def test_continuum_of_a_single_burst_is_q_times_the_cube(parts):
    # one SSP node (alpha 0, Z m, age a) with unit weight: the continuum is
    # Q_ma 10^{C(Z_gas, tau_a, U, lambda)} converted from L_nu to L_lambda per Lsun, with C a
    # multilinear function of the three coordinates, which the trilinear cube reproduces
    lib, lines, cont, dust = parts
    wave = lib["wave"]
    zg, tau, uu = cont["zg_nodes"], cont["tau_nodes"], cont["u_nodes"]
    lam_term = -0.2 * np.log10(wave / 5000.0) ** 2
    cube = (_multilinear(zg[None, :, None, None], tau[:, None, None, None] / 1e6, uu[None, None, :, None])
            + lam_term[None, None, None, :])
    L = om.build_library(CFG, lib, None, dust, cont=dict(cont, cont_table=cube))
    cols = om.columns(CFG.n_sfh, CFG.n_zh)
    th = np.zeros(cols["P"])
    for (m, a, gz, gu) in ((1, L.neb_a0, -0.3, -2.0), (3, L.n_neb - 1, 0.1, -3.7), (0, L.neb_a0 + 2, -1.9, -1.2)):
        th[cols["gas_logz"]], th[cols["gas_logu"]] = gz, gu
        W = np.zeros_like(lib["flux"][..., 0])
        W[0, m, a] = 2.5
        # Q from its defining integral over the raw spectrum (eq. C1), by the trapezoid rule
        sel = wave <= 912.0
        q = LSUN * ANG_CM / (6.62607015e-27 * C_CMS) * np.trapezoid(lib["flux"][0, m, a, sel] * wave[sel], wave[sel])
        chat = _multilinear(gz, lib["ages"][a] / 1e6, gu) + lam_term
        expect = 2.5 * q * 10.0 ** chat * (C_CMS / ANG_CM) / wave ** 2 / LSUN
        got = om.point_continuum(L, th, cols, W)
        np.testing.assert_allclose(got, expect, rtol=1e-11, atol=0.0)


def test_constant_cube_continuum_ignores_the_gas_parameters(parts):
    lib, lines, cont, dust = parts
    c0 = np.where(lib["wave"] < 912.0, -38.0, -25.0 + 0.1 * np.sin(lib["wave"] / 700.0))
    cube = np.broadcast_to(c0, cont["cont_table"].shape).copy()
    L = om.build_library(CFG, lib, lines, dust, cont=dict(cont, cont_table=cube))
    cols = om.columns(CFG.n_sfh, CFG.n_zh)
    th = wl.make_theta(CFG, 2, seed=9)
    th[1] = th[0]
    th[1, cols["gas_logz"]], th[1, cols["gas_logu"]] = 0.35, -3.9
    rf = om.rest_frame(L, th)
    W = rf["per"][0]["W"]
    WQ = sum(W[ia, m, a] * L.Q[ia, m, a] for ia in range(W.shape[0]) for m in range(W.shape[1])
             for a in range(L.neb_a0, L.n_neb))
    expect = WQ * 10.0 ** c0 * (C_CMS / ANG_CM) / lib["wave"] ** 2 / LSUN
    np.testing.assert_allclose(rf["neb"][0], expect, rtol=1e-12, atol=0.0)
    np.testing.assert_allclose(rf["neb"][1], rf["neb"][0], rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("geometry", ["runaway_bc", "picket"])
def test_zero_fob_is_the_model_without_escape(parts, geometry):
    lib, lines, cont, dust = parts
    L0 = om.build_library(CFG, lib, lines, dust, cont=cont)
    L1 = om.build_library(CFG, lib, lines, dust, cont=cont, escape=geometry)
    th = wl.make_theta(CFG, 4, seed=11, escape=True)
    th[:, -1] = 0.0
    assert np.array_equal(om.rest_frame(L1, th)["F"], om.rest_frame(L0, th[:, :-1])["F"])
    filters = wl.make_filters("gauss20")
    ph = om.Photometry(filters=filters)
    assert np.array_equal(om.predict(L1, ph, th), om.predict(L0, ph, th[:, :-1]))
    g = wl.make_spectrum_grid(300)
    sp = om.Spectrum(pix_wave=g["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0, sigma_gas_kms=80.0,
                     sigma_gal_kms=0.0, z_ref=3.0)
    assert np.array_equal(om.predict(L1, sp, th), om.predict(L0, sp, th[:, :-1]))


def _young_burst_theta(L, f, tau_bc, tau_diff, seed=21):
    # all mass in the first SFH bin [0, T1]: SSP ages up to ~T1, every one nebular-covered
    cols = om.columns(CFG.n_sfh, CFG.n_zh, True)
    th = wl.make_theta(CFG, 1, seed=seed, escape=True)[0]
    th[cols["sfh"]:cols["sfh"] + CFG.n_sfh] = 0.0
    th[cols["sfh"]] = 1.0
    th[cols["tau_bc"]], th[cols["tau_diff"]], th[cols["frac_obrun"]] = tau_bc, tau_diff, f
    return th, cols


def _raw_ionising(L, W):
    # sum over every SSP node of W times the raw spectrum, kept below the Lyman limit
    ion = L.wave < 912.0
    out = np.zeros(len(L.wave))
    for ia in range(W.shape[0]):
        for m in range(W.shape[1]):
            for a in range(W.shape[2]):
                out += W[ia, m, a] * L.flux_raw[ia, m, a] * ion
    return out


def _photon_rate(wave, f_lam):
    sel = wave <= 912.0
    return np.trapezoid(f_lam[sel] * wave[sel], wave[sel])


@pytest.mark.parametrize("f", [0.0, 0.17, 0.6, 1.0])
def test_runaway_escape_fraction(parts, f):
    # eq. fesc_runaway: f_esc = f_ob e^{-tau_diff}; with no diffuse dust it equals f_ob
    # whatever the birth-cloud depth, and below 912 A the emergent spectrum is f_ob e^{-tau_d}
    # times the raw ionising continuum
    lib, lines, cont, dust = parts
    L = om.build_library(CFG, lib, lines, dust, cont=_dark(cont, lib["wave"]), escape="runaway_bc")
    th, cols = _young_burst_theta(L, f, 1.3, 0.0)
    rf = om.rest_frame(L, th[None])
    W = rf["per"][0]["W"]
    assert np.all(W[:, :, :L.neb_a0] == 0.0) and np.all(W[:, :, L.n_neb:] == 0.0)
    raw = _raw_ionising(L, W)
    n_int = _photon_rate(L.wave, raw)
    assert _photon_rate(L.wave, rf["F"][0]) / n_int == pytest.approx(f, rel=1e-9, abs=1e-200)
    th[cols["tau_diff"]] = 0.8
    rf = om.rest_frame(L, th[None])
    ion = L.wave < 912.0
    tau_d = 0.8 * (L.wave / 5500.0) ** th[cols["delta"]] * (L.dust_a + (0.85 - 1.9 * th[cols["delta"]]) * L.dust_d)
    np.testing.assert_allclose(rf["F"][0][ion], f * np.exp(-tau_d[ion]) * raw[ion], rtol=1e-9, atol=1e-200)


@pytest.mark.parametrize("f", [0.0, 0.3, 1.0])
def test_picket_escape_fraction_is_fob_through_any_dust(parts, f):
    # picket fence (Sec. 2.3.2): f_esc = f_ob, the escaping sightlines see no dust at all
    lib, lines, cont, dust = parts
    L = om.build_library(CFG, lib, lines, dust, cont=_dark(cont, lib["wave"]), escape="picket")
    th, cols = _young_burst_theta(L, f, 1.7, 0.9)
    rf = om.rest_frame(L, th[None])
    raw = _raw_ionising(L, rf["per"][0]["W"])
    ion = L.wave < 912.0
    np.testing.assert_allclose(rf["F"][0][ion], f * raw[ion], rtol=1e-9, atol=1e-200)


def test_fob_one_removes_nebular_emission_and_the_birth_cloud(parts):
    # f_ob = 1: no nebular emission, the young light crosses no birth cloud and keeps its
    # ionising continuum: runaway_bc is the plain model (no nebular grids) at tau_BC = 0;
    # picket is that model with no dust on the young light, i.e. at tau_BC = tau_diff = 0
    # when the SFH has no old stars
    lib, lines, cont, dust = parts
    plain = om.build_library(CFG, lib, None, dust)
    filters = wl.make_filters("gauss20")
    ph = om.Photometry(filters=filters)
    g = wl.make_spectrum_grid(300)
    sp = om.Spectrum(pix_wave=g["pix_wave"], lsf_mode="R_fwhm", lsf_value=100.0, sigma_gas_kms=80.0,
                     sigma_gal_kms=0.0, z_ref=3.0)
    L = om.build_library(CFG, lib, lines, dust, cont=cont, escape="runaway_bc")
    cols = om.columns(CFG.n_sfh, CFG.n_zh, True)
    th = wl.make_theta(CFG, 3, seed=13, escape=True)
    th[:, cols["frac_obrun"]] = 1.0
    th0 = th[:, :-1].copy()
    th0[:, cols["tau_bc"]] = 0.0
    for obs in (ph, sp):
        np.testing.assert_allclose(om.predict(L, obs, th), om.predict(plain, obs, th0), rtol=1e-12, atol=0.0)
    Lp = om.build_library(CFG, lib, lines, dust, cont=cont, escape="picket")
    thb, _ = _young_burst_theta(Lp, 1.0, 2.0, 1.1)
    thb0 = thb[:-1].copy()
    thb0[cols["tau_bc"]] = 0.0
    thb0[cols["tau_diff"]] = 0.0
    for obs in (ph, sp):
        np.testing.assert_allclose(om.predict(Lp, obs, thb[None]), om.predict(plain, obs, thb0[None]),
                                   rtol=1e-12, atol=0.0)


def test_covered_fraction_scales_nebular_emission(parts):
    # at tau_BC = tau_diff = 0 the young light is Y* + (1 - f) (continuum + lines) + f I in
    # both geometries (Sec. 2.3.2: only the covered fraction powers the nebula)
    lib, lines, cont, dust = parts
    L0 = om.build_library(CFG, lib, lines, dust, cont=cont)
    th, cols = _young_burst_theta(L0, 0.0, 0.0, 0.0)
    ref = om.rest_frame(L0, th[None, :-1])
    neb = ref["F"][0] - ref["Ystar"][0]           # nebular continuum + lines on the grid
    raw = _raw_ionising(L0, ref["per"][0]["W"])
    for geometry in ("runaway_bc", "picket"):
        L = om.build_library(CFG, lib, lines, dust, cont=cont, escape=geometry)
        th[cols["frac_obrun"]] = 0.35
        rf = om.rest_frame(L, th[None])
        np.testing.assert_allclose(rf["F"][0], ref["Ystar"][0] + 0.65 * neb + 0.35 * raw,
                                   rtol=1e-12, atol=1e-300)


def test_adjoint_refuses_what_it_does_not_cover(parts):
    lib, lines, cont, dust = parts
    L = om.build_library(CFG, lib, lines, dust, cont=cont)
    obs = om.Photometry(filters=wl.make_filters("gauss20"), data=np.ones(20), sigma=np.ones(20))
    with pytest.raises(NotImplementedError):
        oa.grad_point(L, obs, wl.make_theta(CFG, 1, seed=1)[0])
