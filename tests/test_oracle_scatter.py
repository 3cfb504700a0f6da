"""Pins of the oracle's resonant-scattering Monte Carlo (App. A, steps 1-8)
against the mathematics and the paper's own checks (CPU only): the atom
velocity law of Eq. (MC), detailed balance of the redistribution of
Eq. (inout), the Peebles C factor of the App. A test problem (Fig. Cfact),
and the frequency x_50 ~ 60 at which a wing photon is lost half the time."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import workloads as W
from oracle import walker, physics as P

A3000 = P.damping(3000.0)


def homog_box(zeta=1.0, profile="doppler", n_packets=2000, seed=7, vel=None):
    od = W.uniform_box(4)
    return W.BoxSpec(n=(4, 4, 4), overdensity=od, zeta=zeta, n_packets=n_packets, seed=seed,
                     profile=profile, velocity=vel)


def _u_cdf(x, a):
    """CDF of the atom-velocity law exp(-u^2) / ((x - u)^2 + a^2) by the
    trapezoid rule on a grid that resolves both the thermal part and the
    resonant spike of width a at u = x."""
    lo, hi = min(-9.0, x - 9.0), max(9.0, x + 9.0)
    spike = x + a * np.tan(np.linspace(-1.55, 1.55, 40001))
    grid = np.unique(np.concatenate([np.linspace(lo, hi, 400001), spike[(spike > lo) & (spike < hi)]]))
    dens = np.exp(-grid ** 2) / ((x - grid) ** 2 + a * a)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    return grid, cdf / cdf[-1]


@pytest.mark.parametrize("x", [0.0, 0.7, -2.2, 3.5, 6.0, -40.0, 300.0])
def test_atom_velocity_law(x):
    """Step 8: the parallel velocity of the scattering atom follows
    exp(-u^2) / ((x - u)^2 + a^2) (the integrand of Eq. (MC)), for photons in
    the core, in the transition and far in the wing (Kolmogorov-Smirnov
    against the law integrated on a grid that resolves its resonant spike)."""
    a = A3000
    u = walker.atom_upar_draws(x, a, 20000, seed=11)
    grid, cdf = _u_cdf(x, a)
    assert stats.kstest(u, lambda v: np.interp(v, grid, cdf)).pvalue > 1e-3
    # and the first moment, computed by quadrature
    f = lambda v: math.exp(-v * v) / ((x - v) ** 2 + a * a)
    pts = sorted({x - 1e-2, x, x + 1e-2, -6.0, 6.0})
    lo, hi = min(-8.0, x - 8.0), max(8.0, x + 8.0)
    edges = [lo] + [p for p in pts if lo < p < hi] + [hi]
    norm = sum(integrate.quad(f, e0, e1, limit=400, epsabs=0)[0] for e0, e1 in zip(edges[:-1], edges[1:]))
    mean = sum(integrate.quad(lambda v: v * f(v), e0, e1, limit=400, epsabs=0)[0]
               for e0, e1 in zip(edges[:-1], edges[1:])) / norm
    assert abs(u.mean() - mean) <= 5 * u.std() / math.sqrt(u.size) + 1e-9


def test_resonant_atoms_without_damping():
    """With the Doppler profile (a = 0) the atom is exactly resonant, u = x."""
    for x in (-3.0, 0.0, 1.25):
        assert np.all(walker.atom_upar_draws(x, 0.0, 100) == x)


@pytest.mark.parametrize("a", [0.0, 0.05])
def test_redistribution_keeps_the_line_profile(a):
    """Detailed balance of the redistribution: repeated re-emission (atom
    velocity, isotropic direction, Eq. (inout)) with no flight in between
    leaves the line profile invariant, so chains started at line centre end
    up distributed like phi (Doppler, or Voigt with a large damping)."""
    n_chain, steps = 3000, 40
    last = np.array([walker.redistribution_chain(0.0, a, steps, seed=5, p=i)[-1] for i in range(n_chain)])
    if a == 0.0:
        law = lambda x: 0.5 * special.erfc(-x)
    else:
        grid = np.linspace(-60, 60, 240001)
        pdf = P.voigt_density(grid, a)
        cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
        cdf += (a / math.pi) / 60.0
        law = lambda x: np.interp(x, grid, cdf)
    assert stats.kstest(last, law).pvalue > 1e-3
    # a wrong sign of the atom's recoil term breaks it
    assert np.abs(last).max() < 60.0


@pytest.mark.parametrize("profile,ptau", [("doppler", 1.0), ("doppler", 10.0), ("voigt", 10.0)])
def test_c_factor_test_problem(profile, ptau):
    """App. A test problem (Fig. Cfact): in a homogeneous universe with
    Lambda_2g = 0 the Monte-Carlo C (the escaped fraction) agrees with
    Eq. (Cfactor), here in its Sobolev form 1 / (1 + p tau_S) for a
    destruction probability p per scattering (raised above the physical p_ab
    so that a photon needs few scatterings)."""
    spec = homog_box(zeta=1e4, profile=profile, n_packets=3000, seed=7)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    tau_s = prep.kappa.mean() / sc["p_ab"]
    r = prep.scatter(sc["p_ab"], p_destroy=ptau / tau_s, records=True)
    rec = r["records"]
    esc = float(np.mean(rec["fate"] == 1))
    c = 1.0 / (1.0 + ptau)
    sig = math.sqrt(c * (1 - c) / rec.size)
    assert abs(esc - c) <= 4 * sig + 0.01
    # the number of scatterings of a photon: tau_S / (1 + p tau_S) on average
    assert rec["scatterings"].mean() == pytest.approx(tau_s / (1 + ptau), rel=0.15)


def test_c_factor_physical_branching():
    """The same with the physical p_ab at zeta = 1e5 against Eq. (Cfactor)
    with Lambda_2g = 0."""
    spec = homog_box(zeta=1e5, n_packets=2000, seed=3)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    rec = prep.scatter(sc["p_ab"], records=True)["records"]
    esc = float(np.mean(rec["fate"] == 1))
    c = P.peebles_c(spec.temp_K, sc["H"], 0.9 * sc["n_H"], lambda_2g=0.0)
    assert abs(esc - c) <= 4 * math.sqrt(c * (1 - c) / rec.size) + 2e-3


def test_x50_wing_photons_lost_half_the_time():
    """App. A: a photon in the red wing drifts back to the core by about
    1/x per scattering while redshifting between scatterings; the two balance
    near x_50 ~ 60, where it is lost half the time. Photons injected at -40
    mostly return to the core (|x| < 3), those at -90 mostly do not."""
    spec = homog_box(profile="voigt", n_packets=1000, seed=5)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    lost = {}
    for X in (40.0, 90.0):
        rec = prep.scatter(sc["p_ab"], p_destroy=0.0, x_inert=400.0, x0=-X, x_return=3.0,
                           records=True)["records"]
        assert np.all((rec["fate"] == 1) | (rec["fate"] == 3))
        lost[X] = float(np.mean(rec["fate"] == 1))
    assert lost[40.0] < 0.4 and lost[90.0] > 0.8
    # linear interpolation of the loss probability puts x_50 between 45 and 80
    x50 = 40.0 + (0.5 - lost[40.0]) / (lost[90.0] - lost[40.0]) * 50.0
    assert 45.0 < x50 < 80.0


def test_scatter_conservation_threads_and_ranges():
    """Integers: sum(A) + escaped + capped = w0 N; the result does not depend
    on the thread count or on splitting the photon range."""
    spec = homog_box(zeta=1e5, profile="voigt", n_packets=600, seed=9)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    full = prep.scatter(sc["p_ab"], p_destroy=1e-3, nthreads=4)
    assert full["A"].sum() + full["escaped"] + full["capped_weight"] == spec.w0 * spec.n_packets
    one = prep.scatter(sc["p_ab"], p_destroy=1e-3, nthreads=1)
    a = prep.scatter(sc["p_ab"], p_destroy=1e-3, p_begin=0, p_end=211, nthreads=2)
    b = prep.scatter(sc["p_ab"], p_destroy=1e-3, p_begin=211, p_end=600, nthreads=3)
    assert np.array_equal(one["A"], full["A"]) and one["escaped"] == full["escaped"]
    assert np.array_equal(a["A"] + b["A"], full["A"])
    for k in ("escaped", "wing", "scatterings", "crossings"):
        assert a[k] + b[k] == full[k] == one[k]


def test_scatter_galilean_invariance():
    """A uniform bulk flow changes nothing (Eq. (inout) depends on velocity
    differences only)."""
    rest = walker.Prepared(homog_box(zeta=1e5, n_packets=300, seed=4))
    vel = np.zeros((3, 4, 4, 4), dtype=np.float32)
    vel[1] += 0.6
    moving = walker.Prepared(homog_box(zeta=1e5, n_packets=300, seed=4, vel=vel))
    p = P.box_scalars(rest.spec)["p_ab"]
    a, b = rest.scatter(p, p_destroy=2e-3), moving.scatter(p, p_destroy=2e-3)
    assert np.array_equal(a["A"], b["A"])
    assert (a["escaped"], a["scatterings"], a["crossings"]) == (b["escaped"], b["scatterings"], b["crossings"])


def _custom(kappa, delta, n_packets, seed, n=4):
    nc = n ** 3
    return walker.Prepared.custom((n, n, n), np.full(nc, float(kappa)), np.ones(nc), n_packets, seed, delta, 6.0)


def _disp(r):
    return np.stack([r["dx"], r["dy"], r["dz"]], axis=1)


def test_displacement_free_streaming():
    """Without line opacity a photon streams straight until the expansion
    redshifts it to -x_inert: its recorded displacement is (x0 + x_inert) /
    delta cell widths along its emission direction, unwrapped across the ten
    or so periodic wraps of a 4^3 box."""
    prep = _custom(0.0, 0.5, 500, 3)
    r = prep.scatter(1.0, x_inert=20.0, p_destroy=0.0, records=True)["records"]
    assert np.all(r["fate"] == 1) and np.all(r["scatterings"] == 0)
    d = _disp(r)
    L = np.linalg.norm(d, axis=1)
    assert np.allclose(L, (r["x0"] + 20.0) / 0.5, rtol=1e-12, atol=1e-9)
    w = prep.records(np.arange(500))                      # the emission's directions
    k = np.stack([w["kx"], w["ky"], w["kz"]], axis=1)
    assert np.allclose(d, L[:, None] * k, atol=1e-9)


@pytest.mark.parametrize("kap,delta", [(5.0, 0.1), (6e4, 192.0)])
def test_displacement_first_flight(kap, delta):
    """A photon destroyed at its first scattering has traveled the free path
    s of kappa_sc (Phi(x0) - Phi(x0 - delta s)) = -ln u (Doppler profile,
    static homogeneous medium), u from the first word of its event block
    (p, 0, 1): the root found here by bisection on erfc against the oracle's
    Newton step, face walk and unwrapping. The second case is the line of
    the zeta = 1e4 test problem, where flights from the wing cross the core."""
    from scipy.optimize import brentq
    seed = 4
    prep = _custom(kap, delta, 400, seed)
    r = prep.scatter(1.0, p_destroy=1.0 - 1e-9, records=True)["records"]
    first = np.nonzero((r["fate"] == 0) & (r["scatterings"] == 1))[0]
    assert first.size > 280                                # the rest escape on their first flight
    L = np.linalg.norm(_disp(r), axis=1)
    for p in first[:150]:
        w = walker.philox4x32_10([int(p) & 0xFFFFFFFF, int(p) >> 32, 0, 1], [seed, 0])
        tau = -math.log(((int(w[0]) >> 9) + 0.5) * 2.0 ** -23)
        x0 = float(r["x0"][p])
        f = lambda s: kap * (P.Phi(x0) - P.Phi(x0 - delta * s)) - tau
        s = brentq(f, 0.0, (x0 + 40.0) / delta, xtol=1e-300, rtol=1e-13)
        assert L[p] == pytest.approx(s, rel=1e-9, abs=1e-14)       # positions are O(1) doubles
    if delta < 1.0:
        assert L[first].max() > 4.0                        # some flights wrap the box
