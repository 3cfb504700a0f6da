"""Pins of the oracle's random numbers, packet initial states and emission
allocation (CPU only)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import walker, brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    out = walker.philox4x32_10(ctr, key)
    assert [int(v) for v in out] == expect


def test_uniform_conversion_exact():
    # u = (m + 1/2) 2^-23 from the top 23 bits: strictly inside (0,1) and
    # exactly representable in binary32
    u = walker.packet_uniforms(seed=12345, p=678)
    assert np.all(u > 0) and np.all(u < 1)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    m = u * 2 ** 23 - 0.5
    assert np.all(m == np.round(m))
    # the packet stream is the Philox block with counter (p_lo, p_hi, s, 0)
    key = [12345 & 0xFFFFFFFF, 12345 >> 32]
    w0 = walker.philox4x32_10([678, 0, 0, 0], key)
    w1 = walker.philox4x32_10([678, 0, 1, 0], key)
    words = np.concatenate([w0, w1]).astype(np.uint64)
    assert np.array_equal(((words >> 9).astype(np.float64) + 0.5) / 2 ** 23, u)


def _custom_homog(n=4, n_packets=20000, seed=7, kappa=5.0, delta=0.05, x_eff=6.0):
    nc = n ** 3
    return walker.Prepared.custom((n, n, n), np.full(nc, kappa), np.ones(nc), n_packets, seed,
                                  delta, x_eff)


def test_initial_state_distributions():
    """Emission frequencies follow the Doppler profile, directions are
    isotropic and positions uniform inside the cell (App. A step 1)."""
    prep = _custom_homog(n_packets=40000)
    rec = prep.transport(records=True)["records"]
    # frequency: Phi is the profile's CDF; KS against it
    phi_cdf = lambda x: 0.5 * __import__("scipy").special.erfc(-x)
    assert stats.kstest(rec["x0"], phi_cdf).pvalue > 1e-3
    # a profile of the wrong width is rejected by the same test
    assert stats.kstest(rec["x0"] * math.sqrt(2.0), phi_cdf).pvalue < 1e-6
    assert stats.kstest(rec["kz"], stats.uniform(-1, 2).cdf).pvalue > 1e-3
    az = np.arctan2(rec["ky"], rec["kx"])
    assert stats.kstest(az, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-3
    norm = rec["kx"] ** 2 + rec["ky"] ** 2 + rec["kz"] ** 2
    assert np.allclose(norm, 1.0, atol=1e-14)
    for f in ("fx", "fy", "fz"):
        assert stats.kstest(rec[f], "uniform").pvalue > 1e-3


def test_quantize_exact():
    s = np.array([0.0, 1.0, 0.5, 3.0, 3.0, 1e-12])
    q = walker.quantize(s)
    assert q[3] == q[4] == 2 ** 32
    assert q[0] == 0
    assert q[2] == math.floor(2 ** 32 * (0.5 / 3.0))
    assert q[5] == math.floor(2 ** 32 * (1e-12 / 3.0))
    with pytest.raises(ValueError):
        walker.quantize(np.array([1.0, -1.0]))
    with pytest.raises(ValueError):
        walker.quantize(np.array([1.0, np.nan]))
    with pytest.raises(ValueError):
        walker.quantize(np.zeros(4))


@pytest.mark.parametrize("n_packets", [1, 7, 1000, 12345])
def test_allocation_matches_per_packet_search(n_packets):
    rng = np.random.default_rng(5)
    s = rng.lognormal(0.0, 1.5, size=300)
    s[rng.integers(0, 300, 40)] = 0.0
    q = walker.quantize(s)
    first = walker.allocate(q, n_packets)
    counts = np.diff(first.astype(np.int64))
    assert counts.sum() == n_packets and first[0] == 0 and first[-1] == n_packets
    assert np.array_equal(counts, brute.allocation_by_search(q, n_packets))
    share = n_packets * q.astype(np.float64) / float(q.astype(np.float64).sum())
    assert np.all(np.abs(counts - share) < 1.0 + 1e-9)
    assert np.all(counts[q == 0] == 0)


@pytest.mark.parametrize("weights,n_packets", [([1, 1, 1, 1], 2), ([1, 1, 1, 1], 6),
                                               ([2, 1, 3, 2], 4), ([1, 0, 1, 0, 2], 8),
                                               ([3, 3, 3], 9)])
def test_allocation_exact_ties(weights, n_packets):
    """Systematic points that land exactly on a cell boundary belong to the
    upper cell (Q_c <= t_p < Q_c+1)."""
    q = walker.quantize(np.array(weights, dtype=np.float64))
    counts = np.diff(walker.allocate(q, n_packets).astype(np.int64))
    assert np.array_equal(counts, brute.allocation_by_search(q, n_packets))


def test_allocation_large_counts_exact():
    # 2^33 packets over cells with 2^32-scale weights needs 128-bit products
    q = np.array([2 ** 32, 1, 2 ** 31, 0, 12345], dtype=np.uint64)
    n = 2 ** 33 + 3
    first = walker.allocate(q, n)
    qt = int(q.sum())
    cum = np.concatenate([[0], np.cumsum(q.astype(object))])
    for c in range(q.size + 1):
        # closed form: odd o with o * Qtot < 2 N Q
        Q = int(cum[c])
        m = 2 * n * Q
        expect = ((m + qt - 1) // qt) // 2
        assert int(first[c]) == expect
