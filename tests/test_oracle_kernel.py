"""T5: the spatial kernel of the streaming walk (CPU only).

In a homogeneous, static medium (Delta = 1, U = 0, one opacity kappa = tau
per unit of swept profile) a packet emitted at frequency x0 has, after a path
of D cell widths, redshifted to x0 - delta D and kept the weight
w0 exp(-tau (Phi(x0) - Phi(x0 - delta D))) (App. A, steps 3-4, with the
profile integral of Sec. IV.A.2); it escapes once x reaches -X. The share of
the emitted weight absorbed further than D from the emission point is then

    F(D) = int phi(x0) [exp(-tau (Phi(x0) - Phi(max(x0 - delta D, -X))))
                        - exp(-tau (Phi(x0) - Phi(-X)))] dx0,

the streaming analogue of the travel-distance distribution of Fig. MCtravel
(Sec. III.B). The oracle's per-packet traces (cell, deposit, segment length)
are compared with this 1-D quadrature bin by bin, and every traced segment is
checked to be the chord of the straight ray through the cell it names.

The quadrature is written here with scipy (erfc, quad); it shares nothing with
the oracle's C walk.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import walker

W0 = 1 << 32
X_ESC = 6.0


def _phi(x):
    return math.exp(-x * x) / math.sqrt(math.pi)


def _Phi(x):
    return 0.5 * special.erfc(-x)


def kernel_quadrature(D, tau, delta, X=X_ESC):
    """F(D) above by adaptive quadrature over the emission frequency (packets
    emitted below -X are never walked and contribute nothing)."""
    def integrand(x0):
        lo = max(x0 - delta * D, -X)
        return _phi(x0) * (math.exp(-tau * (_Phi(x0) - _Phi(lo))) - math.exp(-tau * (_Phi(x0) - _Phi(-X))))
    val, err = integrate.quad(integrand, -X, 12.0, points=[0.0], limit=400, epsabs=1e-12, epsrel=1e-10)
    return val


def _box(n, tau, delta, n_packets, seed):
    nc = n ** 3
    return walker.Prepared.custom((n, n, n), np.full(nc, tau), np.ones(nc), n_packets, seed,
                                  delta, X_ESC)


def _beyond(trace, D_grid, tau, delta):
    """Weight (fraction of w0) one packet deposits beyond each path length D:
    the weight it still holds at D, less what it keeps to the end. At D inside
    a segment the weight at D follows from the weight entering that segment and
    the profile swept from the segment's entry to D. Also returns the bound
    on the deposits' integer rounding beyond D (half a unit per segment)."""
    length = trace["length"]
    dep = trace["deposits"].astype(np.float64)
    rec = trace["record"]
    ends = np.cumsum(length)
    starts = ends - length
    before = W0 - np.concatenate(([0.0], np.cumsum(dep)[:-1]))
    final = W0 - dep.sum()
    out = np.zeros(len(D_grid))
    rnd = np.zeros(len(D_grid))
    for j, D in enumerate(D_grid):
        k = int(np.searchsorted(ends, D))
        if k >= len(length):
            continue
        rnd[j] = 0.5 * (len(length) - k) / W0
        xd = max(rec["x0"] - delta * D, -X_ESC)
        w_at = before[k] * math.exp(-tau * max(0.0, _Phi(trace["x_in"][k]) - _Phi(xd)))
        out[j] = (w_at - final) / W0
    return out, rnd


def _check_chords(trace, n):
    """Every segment is the chord of the ray through the cell it names: its
    midpoint lies inside that cell and its end lies on a face of the grid."""
    rec = trace["record"]
    c0 = int(rec["cell0"])
    origin = np.array([c0 % n + rec["fx"], (c0 // n) % n + rec["fy"], c0 // (n * n) + rec["fz"]])
    k = np.array([rec["kx"], rec["ky"], rec["kz"]])
    ends = np.cumsum(trace["length"])
    mids = ends - 0.5 * trace["length"]
    pos = origin[None, :] + mids[:, None] * k[None, :]
    cell = np.floor(pos).astype(np.int64) % n
    flat = cell[:, 0] + n * (cell[:, 1] + n * cell[:, 2])
    assert np.array_equal(flat, trace["cells"])
    assert np.all(trace["length"] > 0.0)
    # the exit point of each segment sits on a grid plane (one coordinate
    # integral to rounding), except the last, cut where the packet escapes
    pe = origin[None, :] + ends[:-1, None] * k[None, :]
    dist = np.min(np.abs(pe - np.rint(pe)), axis=1)
    assert np.all(dist < 1e-9 * (1.0 + ends[:-1]))


# D from a fraction of a cell to where F has fallen to ~1e-4 (further out it is
# carried by a handful of packets emitted deep in the red wing)
@pytest.mark.parametrize("tau,delta,D_grid", [(10.0, 0.02, (0.3, 1.0, 3.0, 10.0, 30.0, 60.0, 100.0)),
                                              (100.0, 0.05, (0.1, 0.3, 1.0, 3.0, 10.0, 20.0))])
def test_spatial_kernel_matches_quadrature(tau, delta, D_grid):
    """T5: F(D) from the oracle's per-packet deposit records equals the
    quadrature within 4 sigma in every D bin."""
    n, npk = 8, 2500
    prep = _box(n, tau, delta, npk, seed=31)
    D_grid = np.array(D_grid)
    vals = np.zeros((npk, len(D_grid)))
    rnd = np.zeros((npk, len(D_grid)))
    for p in range(npk):
        t = prep.trace(p, cap=20000)
        if p % 10 == 0:
            _check_chords(t, n)
        vals[p], rnd[p] = _beyond(t, D_grid, tau, delta)
    mean = vals.mean(axis=0)
    rounding = rnd.mean(axis=0)
    sig = vals.std(axis=0, ddof=1) / math.sqrt(npk)
    expect = np.array([kernel_quadrature(D, tau, delta) for D in D_grid])
    assert np.all(expect[:-1] > expect[1:])            # a decreasing tail
    assert expect[0] > 0.5 and expect[-1] < 0.01      # the grid spans the kernel
    for D, m, s, r, e in zip(D_grid, mean, sig, rounding, expect):
        assert abs(m - e) <= 4.0 * s + r, (D, m, e, s, r)


def test_spatial_kernel_rescales_with_drift():
    """T10 on the kernel: doubling the drift per cell (delta) halves every
    distance at fixed kappa, F_{2 delta}(D / 2) = F_delta(D), both in the
    quadrature and in the oracle's records."""
    tau, npk = 10.0, 2000
    D_grid = np.array([2.0, 8.0, 32.0, 128.0])
    out = []
    for delta, scale in ((0.02, 1.0), (0.04, 0.5)):
        prep = _box(8, tau, delta, npk, seed=41)
        b = [_beyond(prep.trace(p, cap=20000), D_grid * scale, tau, delta) for p in range(npk)]
        v = np.array([x[0] for x in b])
        r = np.array([x[1] for x in b]).mean(axis=0)
        out.append((v.mean(axis=0), v.std(axis=0, ddof=1) / math.sqrt(npk), r))
        q = [kernel_quadrature(D * scale, tau, delta) for D in D_grid]
        assert np.all(np.abs(out[-1][0] - q) <= 4.0 * out[-1][1] + r)
    qa = np.array([kernel_quadrature(D, tau, 0.02) for D in D_grid])
    qb = np.array([kernel_quadrature(D / 2, tau, 0.04) for D in D_grid])
    assert np.allclose(qa, qb, rtol=1e-8, atol=1e-12)
    diff = np.abs(out[0][0] - out[1][0])
    assert np.all(diff <= 4.0 * np.hypot(out[0][1], out[1][1]) + out[0][2] + out[1][2])


def test_kernel_pin_catches_a_wrong_drift():
    """The comparison has the power to see a plausible mistake: records of a
    walk whose drift per cell is 10 % too large fail the quadrature of the
    stated drift."""
    tau, delta, npk = 10.0, 0.02, 2500
    prep = _box(8, tau, delta * 1.1, npk, seed=31)
    D_grid = np.array([10.0, 30.0, 100.0])
    b = [_beyond(prep.trace(p, cap=20000), D_grid, tau, delta) for p in range(npk)]
    v = np.array([x[0] for x in b])
    r = np.array([x[1] for x in b]).mean(axis=0)
    mean, sig = v.mean(axis=0), v.std(axis=0, ddof=1) / math.sqrt(npk)
    expect = np.array([kernel_quadrature(D, tau, delta) for D in D_grid])
    assert np.any(np.abs(mean - expect) > 4.0 * sig + r)
