"""Pins of the oracle's recombination histories (Sec. III.A.1 Eq. (rec),
Sec. IV.B Eq. (dotne-mix), the 2-zone toy model of Sec. IV.C) against
identities and the paper's statements (CPU only)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import recombination as R, physics as P

COSMO = W.CosmoParams()


def test_saha_start():
    """Hydrogen Saha: x^2 / (1 - x) equals the Saha factor, and x -> 1 at high z."""
    for z in (1300.0, 1500.0, 1600.0):
        x = R.saha_xe(z, COSMO)
        T = COSMO.t_cmb0 * (1 + z)
        nH = P.n_h0(COSMO) * (1 + z) ** 3
        s = (2 * math.pi * P.M_E * P.K_B * T / P.H_PLANCK ** 2) ** 1.5 * math.exp(-P.E_ION / (P.K_B * T)) / nH
        assert x * x / (1 - x) == pytest.approx(s, rel=1e-8)
    assert R.saha_xe(2000.0, COSMO) > 0.999


def test_mixing_term_averages_to_zero():
    """The new term of Eq. (dotne-mix) vanishes on average, and with equal
    regions the full-mixing rate is Eq. (rec) itself."""
    rng = np.random.default_rng(1)
    for _ in range(5):
        delta = rng.uniform(0.2, 2.0, 6)
        w = rng.uniform(0.1, 1.0, 6)
        w /= w.sum()
        xe = rng.uniform(0.01, 0.9, 6)
        z = rng.uniform(800, 1500)
        total, mixing = R.rate_full_mixing(z, xe, delta, w, COSMO)
        assert abs((w * mixing).sum()) <= 1e-12 * (w * np.abs(mixing)).sum()
        same = R.rate_full_mixing(z, np.full(3, xe[0]), np.ones(3), np.ones(3) / 3, COSMO)[0]
        assert np.allclose(same, R.rate_no_mixing(z, np.full(3, xe[0]), np.ones(3), COSMO), rtol=1e-12)


def test_no_clumping_limit():
    """b -> 0: both limits follow the homogeneous history."""
    d, w = R.two_zone(1e-10)
    zs, yh = R.history("homogeneous", d, w, COSMO, z1=800.0)
    for mode in ("no_mixing", "full_mixing"):
        _, y = R.history(mode, d, w, COSMO, z1=800.0)
        assert np.allclose(R.global_xe(y, d, w), yh[:, 0], rtol=1e-6)


def test_fixed_step_rk4_matches_radau():
    """The fixed-step fourth-order Runge-Kutta used by the Monte-Carlo driven
    integration reproduces the implicit integration below z = 1300."""
    d, w = R.two_zone(0.5)
    for mode in ("no_mixing", "full_mixing"):
        zs, y = R.history(mode, d, w, COSMO, z0=1600.0, z1=900.0, z_eval=np.linspace(1600, 900, 701))
        i0 = 300                                            # z = 1300
        f = R.rhs(mode, d, w, COSMO)
        _, yk = R.rk4(f, 1300.0, 900.0, 800, y[i0])
        assert np.allclose(yk[-1], y[-1], rtol=1e-6)


def test_two_zone_model_statements():
    """Sec. IV.C, Fig. rec-2zone (b = 0.5): the global X_e deviates from the
    standard history much less than the zones' own x_e, and the no-mixing
    and full-mixing X_e are very similar."""
    d, w = R.two_zone(0.5)
    zs, yh = R.history("homogeneous", d, w, COSMO)
    xs = yh[:, 0]
    out = {}
    for mode in ("no_mixing", "full_mixing"):
        _, y = R.history(mode, d, w, COSMO)
        X = R.global_xe(y, d, w)
        zone_dev = np.abs(y / xs[:, None] - 1).max()
        glob_dev = np.abs(X / xs - 1).max()
        assert glob_dev < 0.5 * zone_dev
        out[mode] = X
    rel = np.abs(out["no_mixing"] / out["full_mixing"] - 1).max()
    assert rel < 0.05
    # the homogeneous Peebles history: mostly ionised at z = 1300, frozen out near 1e-3 by z = 700
    assert 0.4 < xs[300] < 0.7 and 5e-4 < xs[-1] < 3e-3
