"""Pins of the oracle's physics scalars, closed forms and recombination feed
against printed values, textbook numbers and exact identities (CPU only)."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import physics as P, walker

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
COSMO = W.CosmoParams()


def _printed():
    out = {}
    with open(os.path.join(GOLDEN, "paper_printed_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            out[t[0]] = (float(t[1]), float(t[2]))
    return out


def _z1100():
    spec = W.BoxSpec(n=(4, 4, 4), overdensity=W.uniform_box(4))
    sc = P.box_scalars(spec)
    n1s = (1.0 - 0.1) * sc["n_H"]
    tau = sc["kappa_per_n1s"] * n1s
    f_z = P.escape_homogeneous(tau, 6.0)
    f_2g = (1.0 - f_z) * P.LAMBDA_2G / (sc["beta"] + P.LAMBDA_2G)
    return dict(f_z_v0=f_z, f_2gamma=f_2g, peebles_C=P.peebles_c(3000.0, sc["H"], n1s),
                p_destroy=sc["p_ab"], A_2p1s=P.A_2P1S, Lambda_2gamma=P.LAMBDA_2G,
                E_alpha_eV=P.E_ALPHA / P.EV)


@pytest.mark.parametrize("name", list(_printed()))
def test_paper_printed_values(name):
    """T3: the constants chain reproduces the numbers the paper prints at z~1100
    (Sec. III.A.1, Sec. III.B, App. A) to their printed precision."""
    value, tol = _printed()[name]
    got = _z1100()[name]
    assert abs(got - value) <= tol * value, (name, got, value)


def test_hubble_today_and_equality():
    # H0 = 100 h km/s/Mpc = 3.2408e-18 h s^-1 (textbook)
    assert abs(P.hubble0(0.67) / 0.67 - 3.2408e-18) < 1e-4 * 3.2408e-18
    # matter-radiation equality near z ~ 3400 for Omega_m h^2 ~ 0.14 (textbook
    # estimate z_eq ~ 2.4e4 Omega_m h^2 for T0 = 2.7255 K, N_eff = 3.046)
    z_eq = P.omega_m(COSMO) / P.omega_r(COSMO) - 1.0
    assert abs(z_eq - 2.4e4 * (COSMO.omega_b_h2 + COSMO.omega_c_h2)) < 60.0
    # flatness, and H scales as (1+z)^1.5 deep in matter domination
    h1 = P.hubble(100.0, COSMO)
    h2 = P.hubble(200.0, COSMO)
    assert 1.45 < math.log(h2 / h1) / math.log(201.0 / 101.0) < 1.55
    assert P.hubble(1100.0, COSMO, zeta=7.0) == pytest.approx(7.0 * P.hubble(1100.0, COSMO), rel=1e-15)


def test_hydrogen_density():
    # n_b today = Omega_b rho_c / m_p ~ 2.5e-7 cm^-3 for Omega_b h^2 = 0.0224;
    # 76 % of the baryon mass is hydrogen
    nb = COSMO.omega_b_h2 / COSMO.h ** 2 * P.rho_crit0(COSMO.h) / 1.67262e-24
    assert abs(nb - 2.52e-7) < 0.02e-7
    assert P.n_h0(COSMO) == pytest.approx(0.76 * nb * 1.67262e-24 / P.M_H, rel=1e-12)


def _case_b_table():
    rows = []
    with open(os.path.join(GOLDEN, "case_b_recombination.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            T, a = line.split()[:2]
            rows.append((float(T), float(a)))
    return rows


# the fit reproduces the tabulated coefficients to better than 1 %; the table
# is printed to three figures
CASE_B_REL = 0.01


def _case_b_misses():
    return [abs(P.alpha_e(T) / 1.14 - a) / a for T, a in _case_b_table()]


def test_case_b_coefficient_textbook():
    """alpha_e / 1.14 against the textbook case-B coefficients at 5000, 10^4
    and 2 x 10^4 K (tests/golden/case_b_recombination.txt): the amplitude and
    both temperature exponents of the fit are pinned, and with them alpha_e,
    beta_e, p_ab and kappa_c at the paper's 3000 K."""
    misses = _case_b_misses()
    assert max(misses) < CASE_B_REL, misses


@pytest.mark.parametrize("which,delta", [(1, 0.05), (1, -0.05), (3, 0.05), (3, -0.05),
                                         (2, 0.05), (2, -0.05), (0, 0.1)])
def test_case_b_pin_catches_a_perturbed_coefficient(monkeypatch, which, delta):
    """A fit coefficient mistyped by a few hundredths (the exponent b or d, the
    denominator's c, the amplitude a) moves the fit off the table by more than
    the tolerance at one of the three temperatures."""
    fit = list(P.CASE_B_FIT)
    fit[which] += delta
    monkeypatch.setattr(P, "CASE_B_FIT", tuple(fit))
    assert max(_case_b_misses()) > CASE_B_REL


def test_detailed_balance_saha():
    """In Saha equilibrium the net rate of Eq. (rec) vanishes: beta_e is the
    detailed-balance partner of alpha_e and E_2 + E_alpha = E_I."""
    for T in (2500.0, 3000.0, 4000.0):
        nH = 300.0
        saha = (2 * math.pi * P.M_E * P.K_B * T / P.H_PLANCK ** 2) ** 1.5 \
            * math.exp(-P.E_ION / (P.K_B * T)) / nH
        xe = (-saha + math.sqrt(saha * saha + 4 * saha)) / 2  # x^2/(1-x) = saha
        ne, n1s = xe * nH, (1 - xe) * nH
        rec = P.alpha_e(T) * ne * ne
        ion = P.beta_e(T) * n1s * math.exp(-P.E_ALPHA / (P.K_B * T))
        assert abs(rec - ion) <= 1e-10 * rec


def test_sobolev_identities():
    """R_alpha = 3 P_esc A (Eq. R-alpha) and tau_ab P_esc = p_ab (Eq. <fnu>):
    the mean absorption depth is the destruction probability over the escape
    probability."""
    H = P.hubble(1100.0, COSMO)
    n1s = 229.5
    assert P.r_alpha(H, n1s) == pytest.approx(3 * P.sobolev_p_esc(H, n1s) * P.A_2P1S, rel=1e-13)
    tau = P.tau_ab_per_n1s(3000.0, H) * n1s
    assert tau * P.sobolev_p_esc(H, n1s) == pytest.approx(P.p_ab(3000.0), rel=1e-13)


def test_thermal_velocity_and_line():
    # hydrogen thermal speed sqrt(2kT/m_H) = 12.85 km/s at 1e4 K
    assert abs(P.thermal_velocity(1.0e4) - 12.85e5) < 0.01e5
    # the wavelength is the 1s-2p energy: lambda = h c / E_alpha
    assert P.H_PLANCK * P.C_LIGHT / P.E_ALPHA == pytest.approx(P.LAMBDA_ALPHA, rel=2e-5)


def test_escape_closed_form_limits():
    # tau -> 0: everything escapes; tau -> inf: 1/tau (Sobolev, X -> inf)
    assert P.escape_homogeneous(1e-9, 30.0) == pytest.approx(1.0, rel=1e-8)
    assert P.escape_homogeneous(1e6, 30.0) == pytest.approx(1e-6, rel=1e-9)


# ---- recombination feed ------------------------------------------------------
def _homog_run(n=8, n_packets=20000):
    spec = W.BoxSpec(n=(n, n, n), overdensity=W.uniform_box(n), n_packets=n_packets, seed=4)
    r = walker.run_box(spec)
    return spec, r


def test_feed_homogeneous_reduces_to_peebles():
    """T9 (i): in a homogeneous box the mean feed is Eq. (rec) with the
    Monte-Carlo C: -C (alpha n_e^2 - beta n_1s exp(-E_alpha/T))."""
    spec, r = _homog_run()
    f = P.feed(spec, r["A"], r["escaped"], spec.n_packets)
    sc = P.box_scalars(spec)
    xe = float(np.float32(0.1))
    ne, n1s = xe * sc["n_H"], (1 - xe) * sc["n_H"]
    expect = -f["c_mc"] * (sc["alpha"] * ne * ne - sc["beta"] * n1s * f["boltzmann"])
    assert f["ndot_e"].mean() == pytest.approx(expect, rel=1e-10)
    # and the Monte-Carlo C is close to the Peebles value (Sobolev limit)
    assert f["c_mc"] == pytest.approx(f["c_mix"], rel=0.03)


def test_feed_full_mixing_is_dotne_mix():
    """T9 (ii)-(iii): absorptions spread like n_1s (full mixing) turn the feed
    into Eq. (dotne-mix); its mixing term averages to zero."""
    spec = W.make_box("c1", n=8)
    spec.n_packets = 1000
    sc = P.box_scalars(spec)
    n1s = P.n1s_field(spec)
    # x_e arrives as a binary32 value, like every field
    ne = float(np.float32(0.1)) * sc["n_H"] * spec.overdensity.astype(np.float64).reshape(-1)
    wtot = float(spec.w0) * spec.n_packets
    E = 0.004 * wtot
    A = (wtot - E) * n1s / n1s.sum()
    f = P.feed(spec, A, E, spec.n_packets)
    C = f["c_mc"]
    a = sc["alpha"]
    expect = -C * (a * ne ** 2 - sc["beta"] * n1s * f["boltzmann"]) \
        - (1 - C) * a * (ne ** 2 - n1s / n1s.mean() * (ne ** 2).mean())
    assert np.allclose(f["ndot_e"], expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())
    mixing = (1 - C) * a * (ne ** 2 - n1s / n1s.mean() * (ne ** 2).mean())
    assert abs(mixing.mean()) < 1e-12 * np.abs(mixing).max()
    assert np.allclose(f["mix_corr"], 1.0, rtol=1e-12)
