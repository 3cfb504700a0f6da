"""Pins of the oracle's walk through a bulk-flow gradient (the flow test of
Fig. MCescape, Sec. IV.A.3) against the closed form for a uniform gradient
(CPU only).

A packet moving at direction cosine mu to the axis of a flow with
dv_x/dx = g H drifts in frequency (1 + g mu^2) times as fast as by the
expansion alone, so its escaped weight is exp(-kappa / (1 + g mu^2) dPhi)
(the static closed form with the depth per unit of swept profile divided by
that factor), and the escaped fraction averages it over directions: for
kappa >> 1, (1 + g/3) / kappa, the H -> H + div v / 3 of the figure's
caption. The slab is one wavelength (10 Mpc) of U_x = U0 sin(2 pi x / L),
packets emitted at x = 0 where the gradient is largest; over the few tens of
kpc in which a packet's fate is decided the gradient is uniform to 1e-4.
Per packet the cell-wise flow makes the frequency a staircase around the
straight line, whose first-order effect averages out over emission points:
the mean of (walked - predicted) weight is pinned to its standard error, and
the same comparison with the wrong sign of g, or with g = 0, fails by tens
of standard errors.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import walker, physics as P

N = 65536
CELL = 1e4 * W.KPC_CM / N


def slab(g, n_packets=40000, seed=5):
    delta = P.box_scalars(W.escape_slab(N, 0.0, CELL, 10))["delta"]
    return W.escape_slab(N, g * N * delta / (2.0 * math.pi), CELL, n_packets, seed=seed)


def test_uniform_gradient_formula_limits():
    """g = 0 is the static closed form; tau >> 1 gives (1 + g/3) / tau; the
    direction average lies between the two extreme directions."""
    for tau in (0.5, 10.0, 189.0):
        assert P.escape_uniform_gradient(tau, 0.0, 6.0) == pytest.approx(P.escape_homogeneous(tau, 6.0), rel=1e-12)
    for g in (-0.6, -0.2, 0.3, 0.9):
        tau = 1e6
        assert P.escape_uniform_gradient(tau, g, 6.0) == pytest.approx((1.0 + g / 3.0) / tau, rel=1e-5)
        tau = 5.0
        lo, hi = sorted((P.escape_homogeneous(tau, 6.0), P.escape_homogeneous(tau / (1.0 + g), 6.0)))
        assert lo < P.escape_uniform_gradient(tau, g, 6.0) < hi
    with pytest.raises(ValueError):
        P.escape_uniform_gradient(10.0, -1.0, 6.0)


@pytest.mark.parametrize("g", [-0.5, 0.5, 0.8])
def test_walk_through_flow_gradient(g):
    spec = slab(g)
    r = walker.run_box(spec, records=True)
    rec = r["records"]
    assert r["A"].sum() + r["escaped"] == spec.w0 * spec.n_packets
    kap = float(P.kappa_field(spec).mean())
    X = P.x_eff(spec)
    got = np.where(rec["fate"] == 1, rec["escaped"], 0) / spec.w0
    dphi = np.clip(P.Phi(rec["x0"]) - P.Phi(-X), 0.0, None)

    def diff(gg):
        d = got - np.exp(-kap / (1.0 + gg * rec["kx"] ** 2) * dphi)
        return d.mean(), d.std() / math.sqrt(d.size)

    m, s = diff(g)
    assert abs(m) <= 4.0 * s
    for wrong in (-g, 0.0):
        mw, sw = diff(wrong)
        assert abs(mw) > 10.0 * max(sw, s)
    # the sample mean against the direction average
    f = P.escape_uniform_gradient(kap, g, X)
    assert abs(got.mean() - f) <= 4.0 * got.std() / math.sqrt(got.size)
