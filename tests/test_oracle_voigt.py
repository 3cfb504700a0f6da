"""Pins of the oracle's Voigt line profile (Eq. (MC): the thermal profile
convolved with the natural width of the 2p level) and of its far damping wing
against the mathematics (CPU only)."""
import math

import numpy as np
import pytest
from scipy import special, stats

from oracle import walker, physics as P

W0 = 1 << 32


def homog(n=4, n_packets=20000, seed=7, kappa=5.0, delta=0.05, x_eff=6.0, vel=None, damping=0.0,
          kappa_far=None, x_blue=None):
    nc = n ** 3
    return walker.Prepared.custom((n, n, n), np.full(nc, kappa), np.ones(nc), n_packets, seed,
                                  delta, x_eff, vel=vel, damping=damping, kappa_far=kappa_far,
                                  x_blue=x_blue)


def test_damping_parameter_value():
    """a = A lambda / (4 pi v_th): 8.61e-4 at 3000 K (the natural half width
    6.27e8 / 2 s^-1 over the Doppler width nu_alpha v_th / c, times 1/2 pi)."""
    a = P.damping(3000.0)
    nu_d = P.C_LIGHT / P.LAMBDA_ALPHA * P.thermal_velocity(3000.0) / P.C_LIGHT
    assert a == pytest.approx(P.A_2P1S / (4.0 * math.pi * nu_d), rel=1e-12)
    assert 8.55e-4 < a < 8.7e-4


@pytest.mark.parametrize("x", [-1e4, -300.0, -40.0, -6.0, -3.0, -0.924, -0.2, 1e-3, 0.5, 1.5,
                               2.7, 5.0, 12.0, 1e3])
def test_dawson_series_matches_library(x):
    """Rybicki's series in the C oracle equals the library's Dawson integral."""
    assert walker.dawson(x) == pytest.approx(float(special.dawsn(x)), rel=1e-12, abs=1e-16)


def test_dawson_closed_properties():
    """F is odd, F'(x) = 1 - 2 x F(x) (its differential equation), and
    F(x) -> 1/(2x) far out."""
    for x in (0.3, 1.0, 2.0, 4.0):
        h = 1e-5
        deriv = (walker.dawson(x + h) - walker.dawson(x - h)) / (2 * h)
        assert deriv == pytest.approx(1.0 - 2.0 * x * walker.dawson(x), abs=1e-9)
        assert walker.dawson(-x) == pytest.approx(-walker.dawson(x), rel=1e-15)
    assert walker.dawson(5e3) * 2 * 5e3 == pytest.approx(1.0, rel=1e-7)


@pytest.mark.parametrize("a", [P.damping(3000.0), 0.003])
def test_first_order_cdf_against_exact_voigt(a):
    """The first-order cumulative profile is within a^2 / 2 of the exact
    Voigt CDF (quadrature of the thermal density times the Cauchy CDF), at
    every frequency from the far red wing to the far blue one; the oracle's C
    and numpy versions agree."""
    for x in (-200.0, -30.0, -8.0, -6.0, -4.0, -2.5, -1.5, -0.7, -0.1, 0.0, 0.4, 1.1, 2.0,
              3.5, 6.0, 20.0):
        exact = P.voigt_cdf_exact(x, a)
        first = float(P.Phi_voigt(x, a))
        assert abs(first - exact) <= 0.5 * a * a, (x, first, exact)
        assert walker.profile_cdf(x, a) == pytest.approx(first, rel=1e-13, abs=1e-18)


def test_wing_tail_is_lorentzian():
    """Far in the red wing the cumulative profile is the Cauchy tail
    a / (pi |x|) (the thermal part is negligible there)."""
    a = P.damping(3000.0)
    for x in (-20.0, -100.0, -1e3):
        assert walker.profile_cdf(x, a) == pytest.approx(a / (math.pi * abs(x)), rel=2.0 / x ** 2)


def test_doppler_limit():
    """a = 0 is the thermal profile."""
    for x in (-3.0, -0.5, 0.0, 1.0):
        assert walker.profile_cdf(x, 0.0) == pytest.approx(float(P.Phi(x)), rel=1e-15)


def test_voigt_emission_law():
    """Emission frequencies follow the Voigt law (thermal plus Cauchy
    deviate): Kolmogorov-Smirnov against the library's Voigt density
    integrated exactly, with a damping large enough to make the tails
    count. The Doppler-only emission fails the same test."""
    a = 0.05
    grid = np.linspace(-60, 60, 240001)
    pdf = P.voigt_density(grid, a)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf += (a / math.pi) / 60.0          # the Cauchy mass below -60
    law = lambda x: np.interp(x, grid, cdf)
    prep = homog(n_packets=100000, seed=5, damping=a, kappa=1e-6, x_eff=80.0, delta=200.0)
    x0 = prep.transport(records=True)["records"]["x0"]
    inside = x0[np.abs(x0) < 60]
    assert stats.kstest(inside, lambda x: (law(x) - law(-60)) / (law(60) - law(-60))).pvalue > 1e-3
    tail = np.mean(x0 < -10.0)
    expect = P.voigt_cdf_exact(-10.0, a)
    assert abs(tail - expect) <= 4 * math.sqrt(expect / x0.size)
    plain = homog(n_packets=100000, seed=5, damping=0.0, kappa=1e-6, x_eff=80.0, delta=200.0)
    xd = plain.transport(records=True)["records"]["x0"]
    assert stats.kstest(xd[np.abs(xd) < 60], lambda x: (law(x) - law(-60)) / (law(60) - law(-60))).pvalue < 1e-6


@pytest.mark.parametrize("tau,a,delta", [(20.0, 0.01, 0.1), (190.0, P.damping(3000.0), 0.0192),
                                         (2.0, 0.02, 0.3)])
def test_homogeneous_walk_wing_and_escape(tau, a, delta):
    """Homogeneous static box with the Voigt profile: the walked absorption,
    the far-wing absorption and the true escape agree with the 1-D quadrature
    of their definitions over the Voigt emission law; the true escape is the
    Sobolev form (1 - exp(-tau)) / tau for any profile (its CDF maps the
    emission law to a uniform one); the wing part is a share of the escaped
    weight; the integers are conserved."""
    X = 6.0
    prep = homog(kappa=tau, delta=delta, n_packets=60000, seed=13, damping=a, x_eff=X)
    r = prep.transport(records=True)
    rec = r["records"]
    n = rec.size
    walked = rec["absorbed"] / W0
    wing = rec["wing"] / W0
    esc = np.where(rec["fate"] == 1, rec["escaped"] - rec["wing"], 0) / W0
    assert np.all(rec["wing"] <= np.where(rec["fate"] == 1, rec["escaped"], 0))
    assert r["A"].sum() + r["escaped"] + r["capped_weight"] == W0 * n
    assert r["wing"] == int(rec["wing"].sum())
    ew, eg, ee = P.wing_homogeneous(tau, X, X, a)
    for got, want in ((walked, ew), (wing, eg), (esc, ee)):
        sig = got.std() / math.sqrt(n)
        assert abs(got.mean() - want) <= 4 * sig + 1e-7, (got.mean(), want, sig)
    sob = -math.expm1(-tau) / tau
    assert abs(esc.mean() - sob) <= 4 * esc.std() / math.sqrt(n) + 2 * a * a * tau


def test_wing_absent_for_doppler():
    """With the thermal profile the wing is zero and the walk is unchanged."""
    r = homog(kappa=20.0, n_packets=5000).transport(records=True)
    assert r["wing"] == 0 and np.all(r["records"]["wing"] == 0)


def test_voigt_galilean_invariance():
    """T6 with the Voigt profile: a uniform bulk flow changes no integer
    (no face jumps, no velocity margin)."""
    n = 6
    nc = n ** 3
    kap = np.random.default_rng(3).uniform(1.0, 30.0, nc)
    rest = walker.Prepared.custom((n, n, n), kap, np.ones(nc), 8000, 9, 0.05, 6.0, damping=0.01)
    vel = np.zeros((3, nc))
    vel[0] += 0.7
    vel[2] -= 0.4
    moving = walker.Prepared.custom((n, n, n), kap, np.ones(nc), 8000, 9, 0.05, 6.0, vel=vel,
                                    damping=0.01)
    a, b = rest.transport(), moving.transport()
    assert np.array_equal(a["A"], b["A"])
    assert (a["escaped"], a["wing"], a["crossings"]) == (b["escaped"], b["wing"], b["crossings"])


def test_blue_packets_beyond_window_go_to_the_wing():
    """A packet emitted above x_blue is not walked: no crossing, and the
    wing takes 1 - exp(-kbar Phi(x0)) of it, nearly all."""
    a = 0.05
    prep = homog(kappa=30.0, n_packets=40000, seed=17, damping=a, x_eff=6.0)
    rec = prep.transport(records=True)["records"]
    blue = rec["x0"] > 6.0
    assert blue.sum() > 50
    assert np.all(rec["crossings"][blue] == 0) and np.all(rec["fate"][blue] == 1)
    want = -np.expm1(-30.0 * np.array([walker.profile_cdf(x, a) for x in rec["x0"][blue]])) * W0
    assert np.all(np.abs(rec["wing"][blue] - want) <= 1.0)


def test_feed_counts_wing_as_fully_mixed():
    """The far-wing weight joins the absorption spread like n_1s (full
    mixing): the per-cell absorption still sums to the full-mixing total, and
    C_MC counts only the weight that truly escapes."""
    import workloads as W
    spec = W.make_box("c1", n=8, n_packets=20000, profile="voigt")
    r = walker.run_box(spec)
    assert r["wing"] > 0
    f = P.feed(spec, r["A"], r["escaped"], spec.n_packets, wing=r["wing"])
    f0 = P.feed(spec, r["A"], r["escaped"], spec.n_packets)
    wtot = spec.w0 * spec.n_packets
    assert f["c_mc"] < f0["c_mc"]
    sc = P.box_scalars(spec)
    lam = P.LAMBDA_2G
    assert f["c_mc"] == pytest.approx(((r["escaped"] - r["wing"]) + (r["A"].sum() + r["wing"]) * lam
                                       / (sc["beta"] + lam)) / wtot, rel=1e-12)
    n1s = P.n1s_field(spec)
    a_tot = r["A"] + r["wing"] * n1s / n1s.sum()
    assert np.allclose(f["mix_corr"] * (a_tot.sum() * n1s / n1s.sum()), a_tot, rtol=1e-12)
