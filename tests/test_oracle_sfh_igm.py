"""Pins for the oracle's linear (tent-integral) SFH scheme (App. B, eq. tent_integral) and
the IGM transmission (Sec. 2.6, final paragraph; Madau 1995).

The tent weights are checked against brute-force quadrature of eq. tent_integral, per-bin
mass conservation, and the narrow-burst limit (a burst between two age nodes is split by
the log-age interpolation weights).  The IGM coefficients are the published ones and are
not pinned by anything outside the formula (parity unpinned); the pins fix its structure:
identity redward of Lyman alpha and at zero scaling, the power law in the optical-depth
scaling, the Lyman alpha forest's lambda^3.46 law, continuity at the Lyman limit, and that
photometric bands redward of Lyman alpha are untouched.

The two optional additions are pinned from outside their formulas: the damping wing's
closed form against direct quadrature of the optical depth it integrates (the Lorentzian
wing of Lyman alpha through a neutral, matter-dominated IGM whose density is fixed by the
Gunn-Peterson depth), Tepper-Garcia's Voigt approximation against the Faddeeva function
(scipy) within the approximation's accuracy, the absorber's far wings against the pure
Lorentzian and its line centre against the Doppler core; and both vanish in their limits
(x_HI = 0, a source below the neutral region, a negligible column).
"""
import numpy as np
import pytest

from oracle import igm
from oracle import model as om
from oracle import sfh
from synth import workloads as wl

AGES = np.geomspace(1e6, 1.3e10, 40)


def _brute_tent(edges, psi_nodes, ages, nq=100000):
    """eq. tent_integral by the midpoint rule on every bin (no closed form)."""
    psi = np.concatenate([psi_nodes, [psi_nodes[-1]]])
    out = np.zeros((len(edges) - 1, len(ages)))
    for i in range(len(edges) - 1):
        T0, T1 = edges[i], edges[i + 1]
        tt = T0 + (np.arange(nq) + 0.5) / nq * (T1 - T0)
        ps = psi[i] + (psi[i + 1] - psi[i]) * (tt - T0) / (T1 - T0)
        j = np.searchsorted(ages, tt) - 1
        lo = j < 0
        hi = j >= len(ages) - 1
        mid = ~lo & ~hi
        jm = j[mid]
        a = np.log(ages[jm + 1] / tt[mid]) / np.log(ages[jm + 1] / ages[jm])
        np.add.at(out[i], jm, ps[mid] * a)
        np.add.at(out[i], jm + 1, ps[mid] * (1.0 - a))
        out[i, 0] += ps[lo].sum()
        out[i, -1] += ps[hi].sum()
        out[i] *= (T1 - T0) / nq
    return out


def test_tent_weights_hold_twelve_digits_on_sloped_bins_far_from_t0():
    # bins of a few per cent of their lookback time with SFRs changing tenfold across them:
    # the closed form in alpha + beta t (alpha = psi_i - beta T_i) cancels there; written
    # about each piece's own start it keeps its digits.  Reference: each piece between two
    # age nodes integrated by 24-point Gauss-Legendre in extended precision (the integrand
    # is analytic on a piece, so the rule is exact to rounding)
    ages = np.geomspace(1e6, 1.3e10, 107)
    edges = np.concatenate([[0.0], np.geomspace(3e6, 1.2e10, 121)])
    psi = np.where(np.arange(121) % 2 == 0, 1e-9, 1e-8)
    w = sfh.tent_weights(edges, psi, ages)
    ld = np.longdouble
    gx, gw = np.polynomial.legendre.leggauss(24)
    gx, gw = gx.astype(ld), gw.astype(ld)
    for i in (60, 90, 118):
        T0, T1 = ld(edges[i]), ld(edges[i + 1])
        p0, p1 = ld(psi[i]), ld(psi[i + 1] if i + 1 < len(psi) else psi[-1])
        ref = np.zeros(len(ages), dtype=ld)
        for j in range(len(ages) - 1):
            u, v = max(T0, ld(ages[j])), min(T1, ld(ages[j + 1]))
            if v <= u:
                continue
            tt = 0.5 * (u + v) + 0.5 * (v - u) * gx
            ps = p0 + (p1 - p0) * (tt - T0) / (T1 - T0)
            a = np.log(ld(ages[j + 1]) / tt) / np.log(ld(ages[j + 1]) / ld(ages[j]))
            ref[j] += 0.5 * (v - u) * np.sum(gw * ps * a)
            ref[j + 1] += 0.5 * (v - u) * np.sum(gw * ps * (1 - a))
        nz = ref > 0
        err = np.abs(w[i][nz] - ref[nz].astype(float)) / ref[nz].astype(float)
        assert err.max() < 1e-12
        # the bin's weights sum to its trapezoid mass to rounding
        assert w[i].sum() == pytest.approx(float(0.5 * (p0 + p1) * (T1 - T0)), rel=1e-14, abs=0.0)


def test_tent_weights_match_quadrature_of_the_tent_integral():
    rng = np.random.default_rng(3)
    edges = sfh.sfh_edges(1.1e10, 12, 3e6)
    psi = np.exp(rng.normal(0.0, 1.0, 12)) * 1e-9
    w = sfh.tent_weights(edges, psi, AGES)
    ref = _brute_tent(edges, psi, AGES)
    np.testing.assert_allclose(w, ref, rtol=0.0, atol=1e-7 * np.abs(ref).max())


def test_tent_weights_conserve_each_bins_trapezoid_mass():
    rng = np.random.default_rng(4)
    edges = sfh.sfh_edges(9e9, 30, 3e6)
    psi = np.exp(rng.normal(0.0, 2.0, 30)) * 1e-9
    w = sfh.tent_weights(edges, psi, AGES)
    p = np.concatenate([psi, [psi[-1]]])
    mass = 0.5 * (p[:-1] + p[1:]) * np.diff(edges)
    np.testing.assert_allclose(w.sum(axis=1), mass, rtol=1e-13, atol=0.0)
    assert np.all(w >= 0.0)


def test_narrow_burst_is_split_by_the_log_age_weights():
    # a constant-SFR burst of width 1e-6 of its age between nodes j and j+1 puts mass m at
    # t: (1 - b) m on node j and b m on node j+1, b = ln(t / t_j) / ln(t_{j+1} / t_j)
    j, frac = 17, 0.37
    t = AGES[j] * (AGES[j + 1] / AGES[j]) ** frac
    h = 1e-6 * t
    edges = np.array([0.0, t - h, t + h, t + 2 * h, 2e10])
    psi = np.array([0.0, 1.0, 1.0, 0.0])
    w = sfh.tent_weights(edges, psi, AGES)
    # bin 1 holds the burst at constant SFR; the others ramp up to and down from it
    m = w[1].sum()
    assert m == pytest.approx(edges[2] - edges[1], rel=1e-12, abs=0.0)   # its trapezoid mass
    assert w[1, j] / m == pytest.approx(1.0 - frac, rel=1e-11, abs=0.0)
    assert w[1, j + 1] / m == pytest.approx(frac, rel=1e-11, abs=0.0)
    assert np.count_nonzero(w[1]) == 2


def test_model_linear_scheme_forms_the_trapezoid_masses():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.0, -1.0, 0.0), n_wave=600, n_sfh=10, n_zh=0, n_lines=0)
    lib = wl.make_library(cfg, 0)
    L = om.build_library(cfg, lib, None, wl.make_dust_tables(cfg, lib["wave"]), sfh_scheme="linear")
    th = wl.make_theta(cfg, 3, seed=5, sfh_scheme="linear")
    cols = om.lib_columns(L)
    for b in range(3):
        p = om.point_weights(L, th[b], cols)
        psi = np.concatenate([th[b, cols["sfh"]:cols["sfh"] + cfg.n_sfh], [th[b, cols["sfh"] + cfg.n_sfh - 1]]])
        mass = np.sum(0.5 * (psi[:-1] + psi[1:]) * np.diff(p["edges"]))
        assert p["W"].sum() == pytest.approx(mass, rel=1e-12, abs=0.0)


def test_igm_is_identity_redward_of_lyman_alpha_and_at_zero_scaling():
    for z in (0.5, 3.0, 7.2):
        lam = np.geomspace(1215.67 * (1 + z), 6e4, 200)
        assert np.all(igm.transmission(lam, z, 1.3) == 1.0)
        lam = np.geomspace(912.0 * (1 + z) * 0.5, 1215.6 * (1 + z), 300)
        assert np.all(igm.transmission(lam, z, 0.0) == 1.0)
        T1 = igm.transmission(lam, z, 1.0)
        # absorbers between z = 0 and the source: the Ly alpha forest covers (1216 A, 1216 (1 + z))
        forest = lam > 1215.67
        assert np.all(T1[forest] < 1.0) and np.all(T1 > 0.0) and np.all(T1 <= 1.0)
        np.testing.assert_allclose(igm.transmission(lam, z, 0.6), T1 ** 0.6, rtol=1e-13, atol=0.0)


def test_igm_lyman_alpha_forest_follows_its_power_law_and_the_limit_is_continuous():
    z = 4.0
    # between Ly beta and Ly alpha (observed) only the Ly alpha forest absorbs: tau ~ lambda^3.46
    l1, l2 = 1030.0 * (1 + z), 1200.0 * (1 + z)
    t1, t2 = igm.madau_tau(np.array([l1, l2]), z)
    assert np.log(t2 / t1) / np.log(l2 / l1) == pytest.approx(3.46, rel=1e-12, abs=0.0)
    # the Lyman-limit term starts from zero at the source's limit
    ll = 911.75 * (1 + z)
    tau = igm.madau_tau(np.array([ll * (1 - 1e-9), ll * (1 + 1e-9)]), z)
    assert tau[0] == pytest.approx(tau[1], rel=1e-6, abs=0.0)
    # and absorbs more at shorter wavelengths below it
    lam = np.linspace(0.7, 0.999, 50) * ll
    assert np.all(np.diff(igm.madau_tau(lam, z)) < 0.0)


def test_model_bands_redward_of_lyman_alpha_are_untouched_by_the_igm():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.0, -1.0, 0.0), n_wave=1500, n_sfh=10, n_zh=0, n_lines=0)
    lib = wl.make_library(cfg, 0)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L0 = om.build_library(cfg, lib, None, dust)
    L1 = om.build_library(cfg, lib, None, dust, igm=True)
    filters = wl.make_filters("gauss20")
    obs = om.Photometry(filters=filters)
    th = wl.make_theta(cfg, 4, seed=8, igm=True)
    th[:, 1] = [0.6, 1.0, 1.5, 2.0]                  # Ly alpha below every filter's nodes
    reddest_blue_edge = min(f[0].min() for f in filters)
    assert np.all(1215.67 * (1 + th[:, 1]) < reddest_blue_edge)
    assert np.array_equal(om.predict(L1, obs, th), om.predict(L0, obs, th[:, :-1]))
    th[:, 1] = 9.0                                   # now the bluest bands see the forest
    m0, m1 = om.predict(L0, obs, th[:, :-1]), om.predict(L1, obs, th)
    assert np.all(m1 <= m0) and np.any(m1 < 0.9 * m0)


# the damping wing and the damped absorber (Sec. 2.6): constants of Lyman alpha in cgs
_K_LYA = np.pi * igm.E_ESU ** 2 / (igm.ME_G * igm.C_CMS) * igm.LYA_F     # integrated cross-section [cm^2 Hz]
_NU_A = igm.C_CMS / igm.LYA_CM


def test_damping_wing_is_the_lorentzian_wing_integrated_through_the_neutral_igm():
    from scipy.integrate import quad
    z, x_hi = 8.3, 0.7
    for lam in (1215.67 * (1 + z) * np.array([1.0005, 1.003, 1.02, 1.1, 1.5])):
        # optical depth from z_l = 6 to the source: n_HI sigma c dt, with n_HI / H(z) fixed by
        # tau_GP(z) = K lambda_alpha n_HI(z) / H(z) and dt = dz / ((1 + z) H(z)); the wing of
        # the cross-section, K Gamma / (4 pi^2 (nu - nu_alpha)^2) with the Rayleigh factor
        # (nu / nu_alpha)^4 of the scattering wing, at nu = c (1 + z') / lambda_obs
        def dtau(zp):
            nu = igm.C_CMS * (1.0 + zp) / (lam * 1e-8)
            return (x_hi * float(igm.tau_gp(zp)) / (_K_LYA * igm.LYA_CM) * _K_LYA * igm.LYA_GAMMA
                    * (nu / _NU_A) ** 4 / (4.0 * np.pi ** 2 * (nu - _NU_A) ** 2) * igm.C_CMS / (1.0 + zp))
        direct = quad(dtau, igm.Z_NEUTRAL_END, z, epsabs=0.0, epsrel=1e-12, limit=200)[0]
        assert float(igm.damping_wing_tau(np.array([lam]), z, x_hi)[0]) == pytest.approx(direct, rel=1e-9, abs=0.0)


def test_damping_wing_limits_and_the_trough():
    lam = np.geomspace(7000.0, 30000.0, 400)
    assert np.all(igm.damping_wing_tau(lam, 5.5, 0.8) == 0.0)          # source below the neutral region
    assert np.all(igm.damping_wing_tau(lam, 9.0, 0.0) == 0.0)
    tau = igm.damping_wing_tau(lam, 9.0, 0.5)
    red = lam > 1215.67 * 10.0
    assert np.all(np.diff(tau[red]) < 0.0) and tau[red][-1] < 1e-2       # the wing decays redward
    trough = (lam > 1215.67 * 7.0) & (lam < 1215.67 * 10.0)
    assert np.all(tau[trough] > 1e4)                                       # Gunn-Peterson: no flux
    assert np.all(tau[lam < 1215.67 * 7.0] == 0.0)
    np.testing.assert_allclose(igm.damping_wing_tau(lam, 9.0, 0.25), 0.5 * tau, rtol=1e-14, atol=0.0)


def test_voigt_approximation_against_the_faddeeva_function():
    from scipy.special import wofz
    dnu_d = igm.DLA_B_KMS * 1e5 / igm.LYA_CM
    a = igm.LYA_GAMMA / (4.0 * np.pi * dnu_d)
    x = np.concatenate([[0.0, 1e-4, 9e-3, 1.1e-2], np.linspace(0.02, 12.0, 3000), np.geomspace(12.0, 1e5, 300)])
    exact = wofz(x + 1j * a).real
    got = igm.voigt_tepper_garcia(a, x)
    # the approximation's own accuracy at this damping parameter: a few per cent where the
    # Doppler core gives way to the wings, far better in the core and the wings
    assert np.max(np.abs(got - exact) / exact) < 0.035
    core, near, wing = x < 1.0, x > 6.0, x > 12.0
    assert np.max(np.abs(got - exact)[core] / exact[core]) < 1e-3
    assert np.max(np.abs(got - exact)[near] / exact[near]) < 5e-3
    assert np.max(np.abs(got - exact)[wing] / exact[wing]) < 1e-3


def test_damped_absorber_wing_centre_and_column():
    z_dla, lnh = 6.2, 21.3
    N = 10.0 ** lnh
    dnu_d = igm.DLA_B_KMS * 1e5 / igm.LYA_CM
    a = igm.LYA_GAMMA / (4.0 * np.pi * dnu_d)
    # line centre: the Doppler core, H(a, 0) = 1 - 2 a / sqrt(pi) to first order in a
    lam_c = 1215.67 * (1 + z_dla)
    t0 = float(igm.dla_tau(np.array([lam_c]), z_dla, lnh)[0])
    assert t0 == pytest.approx(N * _K_LYA / (np.sqrt(np.pi) * dnu_d) * (1.0 - 2.0 * a / np.sqrt(np.pi)),
                               rel=1e-6, abs=0.0)
    # far wings: the Lorentzian N K Gamma / (4 pi^2 (nu - nu_alpha)^2)
    lam = lam_c * np.array([0.97, 0.99, 1.01, 1.05])
    nu = igm.C_CMS * (1 + z_dla) / (lam * 1e-8)
    lor = N * _K_LYA * igm.LYA_GAMMA / (4.0 * np.pi ** 2 * (nu - _NU_A) ** 2)
    np.testing.assert_allclose(igm.dla_tau(lam, z_dla, lnh), lor, rtol=2e-3, atol=0.0)
    # linear in the column
    np.testing.assert_allclose(igm.dla_tau(lam, z_dla, lnh - 1.0), 0.1 * igm.dla_tau(lam, z_dla, lnh), rtol=1e-13)


def test_model_with_negligible_additions_is_the_madau_model():
    cfg = wl.reduced(wl.CONFIGS["c1"], n_age=40, logz=(-2.0, -1.0, 0.0), n_wave=1500, n_sfh=10, n_zh=0, n_lines=0)
    lib = wl.make_library(cfg, 0)
    dust = wl.make_dust_tables(cfg, lib["wave"])
    L1 = om.build_library(cfg, lib, None, dust, igm=om.IGM_MADAU)
    L7 = om.build_library(cfg, lib, None, dust, igm=om.IGM_MADAU | om.IGM_DAMPING | om.IGM_DLA)
    c1, c7 = om.lib_columns(L1), om.lib_columns(L7)
    assert c7["P"] == c1["P"] + 3 and c7["x_hi"] == c1["igm_factor"] + 1 and c7["z_dla"] == c7["log_nhi"] + 1
    obs = om.Photometry(filters=wl.make_filters("gauss20"))
    th1 = wl.make_theta(cfg, 6, seed=8, igm=1)
    th1[:, 1] = [6.5, 7.5, 8.5, 9.5, 10.5, 11.5]
    th7 = np.concatenate([th1, np.zeros((6, 3))], axis=1)
    th7[:, c7["x_hi"]] = 0.0
    th7[:, c7["log_nhi"]] = -30.0
    th7[:, c7["z_dla"]] = th1[:, 1] - 0.2
    np.testing.assert_allclose(om.predict(L7, obs, th7), om.predict(L1, obs, th1), rtol=1e-14, atol=0.0)
    th7[:, c7["x_hi"]] = 0.9
    th7[:, c7["log_nhi"]] = 21.5
    m1, m7 = om.predict(L1, obs, th1), om.predict(L7, obs, th7)
    assert np.all(m7 <= m1 * (1 + 1e-14)) and np.any(m7 < 0.95 * m1)
    with pytest.raises(ValueError):
        om.build_library(cfg, lib, None, dust, igm=om.IGM_DAMPING)
