"""Pins for the oracle's SFH/ZH -> SSP weights (Sec. 2.2, App. B).

Brute force (sub-sampled bins assigned to the nearest SSP age in linear time),
mass conservation, single-age-bin identity, exact interpolation of linear
functions, and the metallicity split reproducing the bin metallicity.
"""
import numpy as np
import pytest

from oracle import sfh
from synth import workloads as wl


def _ages(n=20):
    return np.geomspace(1e6, 1.3e10, n)


def test_brute_force_nearest_age_assignment():
    ages = _ages(20)
    lo, hi = sfh.age_cells(ages)
    edges = sfh.sfh_edges(2.2e9, 10, 1e7)
    rng = np.random.default_rng(0)
    masses = rng.dirichlet(np.ones(10))
    w = sfh.step_weights(edges, masses, lo, hi)
    n = 400_000
    ref = np.zeros_like(w)
    for i in range(10):
        # midpoint sub-sampling of a constant SFR over the bin, each sample given
        # to the SSP age closest to it in linear time
        t = edges[i] + (np.arange(n) + 0.5) / n * (edges[i + 1] - edges[i])
        nearest = np.argmin(np.abs(t[:, None] - ages[None, :]), axis=1)
        ref[i] = masses[i] * np.bincount(nearest, minlength=len(ages)) / n
    assert np.max(np.abs(w - ref)) < 1e-5


def test_mass_conservation_and_nonnegativity():
    cfg = wl.CONFIGS["c1"]
    ages = _ages(cfg.n_age)
    lo, hi = sfh.age_cells(ages)
    th = wl.make_theta(cfg, 16, seed=3)
    for t_univ in (3.6e8, 2e9, 8.6e9):
        edges = sfh.sfh_edges(t_univ, cfg.n_sfh, cfg.T1)
        for b in range(16):
            m = th[b, wl.N_SCALARS:wl.N_SCALARS + cfg.n_sfh]
            w = sfh.step_weights(edges, m, lo, hi)
            assert np.all(w >= 0)
            assert np.allclose(w.sum(axis=1), m, rtol=1e-14, atol=0)
            W = sfh.ssp_weights(w, np.full(cfg.n_sfh, -0.7), np.array(cfg.logz))
            assert abs(W.sum() - m.sum()) < 1e-14


def test_single_age_bin_goes_to_one_node():
    ages = _ages(20)
    lo, hi = sfh.age_cells(ages)
    for a in (0, 7, 19):
        top = hi[a] if np.isfinite(hi[a]) else 2 * ages[-1]
        w = sfh.step_weights(np.array([lo[a], top]), np.array([3.5]), lo, hi)
        expect = np.zeros(20)
        expect[a] = 3.5
        assert np.array_equal(w[0], expect)


def test_edges_rescale_to_age_of_universe():
    e = sfh.sfh_edges(5e9, 12, 3e6)
    assert e[0] == 0 and e[1] == 3e6 and e[-1] == pytest.approx(5e9, rel=1e-15, abs=0.0)
    r = e[2:] / e[1:-1]
    assert np.allclose(r, r[0], rtol=1e-12)


@pytest.mark.parametrize("t_univ", [3.6e8, 4e9])
def test_zh_interpolates_linear_in_lnT_exactly(t_univ):
    edges = sfh.sfh_edges(t_univ, 120, 3e6)
    node_t = np.geomspace(3e6, t_univ, 24)
    a, b = -1.1, 0.07
    zeta = sfh.bin_metallicity_hist(a + b * np.log(node_t), edges, 3e6, t_univ)
    centres = np.sqrt(edges[1:-1] * edges[2:])
    assert np.allclose(zeta[1:], a + b * np.log(centres), rtol=0, atol=1e-13)
    assert zeta[0] == pytest.approx(a + b * np.log(3e6), abs=1e-14)   # clamped at the first node


@pytest.mark.parametrize("zeta", [-2.5, -2.37, -1.0, 0.0, 0.123, 0.5, 0.9, -3.0])
def test_metallicity_split_reproduces_zeta(zeta):
    nodes = np.linspace(-2.5, 0.5, 22)
    w = np.array([[0.0, 0.4, 0.6]])
    W = sfh.ssp_weights(w, np.array([zeta]), nodes)[0]
    tot = W.sum(axis=0)
    mean = (W * nodes[:, None]).sum(axis=0)[1:] / tot[1:]
    assert np.allclose(mean, np.clip(zeta, -2.5, 0.5), atol=1e-14)
    assert np.count_nonzero(W[:, 1]) <= 2


def test_grid_split_ties_and_clamps():
    nodes = np.array([0.0, 1.0, 2.0, 4.0])
    assert sfh.grid_split(1.0, nodes) == (1, 0.0)
    assert sfh.grid_split(4.0, nodes) == (2, 1.0)
    assert sfh.grid_split(-5.0, nodes) == (0, 0.0)
    assert sfh.grid_split(9.0, nodes) == (2, 1.0)
    assert sfh.grid_split(3.0, nodes) == (2, 0.5)


def test_alpha_split():
    w = np.array([[1.0, 2.0]])
    W = sfh.ssp_weights(w, np.array([-1.0]), np.array([-2.0, 0.0]), afe=0.3, afe_nodes=(0.0, 0.2, 0.4))
    assert W.shape == (3, 2, 2)
    assert np.allclose(W[:, :, 1].sum(axis=1), [0.0, 1.0, 1.0])
    assert np.allclose(W.sum(), 3.0)
