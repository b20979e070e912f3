"""Pins for the oracle's emission-line catalogue arm (Sec. 3.3, App. I.1-I.2).

A single-line entry is checked against its definition written out by brute force (the
photon-weighted mass of every nebular SSP node times 10^Lhat, times 10^logmass / 4 pi D_L^2,
through the birth cloud and the diffuse screen at the line), a blend against the sum of its
members, and the likelihood against the detection and one-sided upper-limit forms.
"""
import math

import numpy as np
import pytest

from oracle import cosmology, dust
from oracle import likelihood as lk
from oracle import model as om
from oracle import nebular
from synth import workloads as wl

CFG = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.5, -1.5, -0.5, 0.5), n_wave=1500, n_sfh=12, n_zh=4,
                 n_lines=8)


@pytest.fixture(scope="module")
def parts():
    lib = wl.make_library(CFG, 0)
    lines = wl.make_lines(CFG, lib, 1)
    dust_tab = wl.make_dust_tables(CFG, lib["wave"])
    L = om.build_library(CFG, lib, lines, dust_tab)
    return lib, lines, dust_tab, L


def test_single_line_entry_is_its_definition(parts):
    lib, lines, dust_tab, L = parts
    cols = om.columns(CFG.n_sfh, CFG.n_zh)
    th = wl.make_theta(CFG, 3, seed=4)
    obs = om.Lines(blends=[[l] for l in range(CFG.n_lines)])
    got = om.predict(L, obs, th)
    ny = int(np.sum(lib["ages"] < CFG.t_young))
    for b in range(3):
        W = om.point_weights(L, th[b], cols)["W"]
        lhat = nebular.line_table_interp(lines["line_table"], lines["zg_nodes"], lines["u_nodes"],
                                         th[b, cols["gas_logz"]], th[b, cols["gas_logu"]])
        z = th[b, cols["zred"]]
        dl = cosmology.luminosity_distance_cm(z, 70.0, 0.3)
        for l in range(CFG.n_lines):
            Ll = 0.0
            for ia in range(W.shape[0]):
                for m in range(W.shape[1]):
                    for a in range(ny):
                        Ll += W[ia, m, a] * L.Q[ia, m, a] * 10.0 ** lhat[l, a]
            lw = lines["line_wave"][l]
            tau = (dust.birth_cloud_tau(lw, th[b, cols["tau_bc"]], th[b, cols["alpha_bc"]])
                   + dust.diffuse_tau(lw, th[b, cols["tau_diff"]], th[b, cols["delta"]],
                                      np.interp(lw, lib["wave"], dust_tab["dust_a"]),
                                      np.interp(lw, lib["wave"], dust_tab["dust_d"])))
            expect = Ll * math.exp(-tau) * 10.0 ** th[b, cols["logmass"]] / (4.0 * math.pi * dl * dl)
            assert got[b, l] == pytest.approx(expect, rel=1e-12, abs=0.0)


def test_blend_is_the_sum_of_its_lines(parts):
    _, _, _, L = parts
    th = wl.make_theta(CFG, 4, seed=6)
    single = om.predict(L, om.Lines(blends=[[l] for l in range(CFG.n_lines)]), th)
    blends = [[0, 1], [2, 5, 7], [3], [4, 6]]
    got = om.predict(L, om.Lines(blends=blends), th)
    for k, bl in enumerate(blends):
        np.testing.assert_allclose(got[:, k], single[:, bl].sum(axis=1), rtol=1e-15, atol=0.0)


def test_detection_and_upper_limit_likelihood():
    d = np.array([1.0, 2.0, 3.0, 4.0])
    s = np.array([0.5, 0.5, 1.0, 2.0])
    m = np.array([1.5, 1.0, 5.0, 3.0])
    mask = np.array([True, True, True, False])
    det = np.zeros(4, dtype=bool)
    assert lk.lines_lnlike(d, m, s, mask, det) == pytest.approx(-0.5 * (1.0 + 4.0 + 4.0), rel=1e-15, abs=0.0)
    up = np.array([False, True, True, True])
    # entry 1: model below its limit, no penalty; entry 2: above, the Gaussian residual
    assert lk.lines_lnlike(d, m, s, mask, up) == pytest.approx(-0.5 * (1.0 + 0.0 + 4.0), rel=1e-15, abs=0.0)
