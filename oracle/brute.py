"""Brute-force counterparts used to pin the oracle (test infrastructure only).

Each function here reaches a result of the walker by a different route, so a
mistake in one shows up as a disagreement:

* ``allocation_by_search``: places every packet by its own systematic point
  instead of counting packets below each cell boundary;
* ``planes_crossed``: counts the grid planes a straight ray crosses, in closed
  form, instead of stepping face to face;
* ``march``: the paper's own small-step scheme (App. A, steps 3-4): advance the
  packet by a short path length, redshift it by H dl / v_th, absorb with the
  local cross-section, with the frequency kept in the frame of the expansion
  and the gas-frame frequency recomputed from the local bulk velocity at every
  step, so the face jumps of Eq. (inout) are never applied explicitly.
"""
import math
import numpy as np
from scipy.special import erfc


def allocation_by_search(q, n_packets):
    """Packets per cell from t_p = floor((2p+1) Q / 2N), p = 0..N-1, each
    located among the cumulative weights by a search (exact Python integers)."""
    q = [int(v) for v in q]
    cum = [0]
    for v in q:
        cum.append(cum[-1] + v)
    qtot = cum[-1]
    counts = [0] * len(q)
    import bisect
    for p in range(int(n_packets)):
        t = ((2 * p + 1) * qtot) // (2 * int(n_packets))
        c = bisect.bisect_right(cum, t) - 1
        counts[c] += 1
    return np.array(counts, dtype=np.int64)


def planes_crossed(f, k, length):
    """Number of cells a ray visits: 1 + the integer planes it crosses along
    each axis over a path of ``length`` cell widths from fractional position f."""
    n = 1
    for a in range(3):
        end = f[a] + k[a] * length
        n += abs(math.floor(end) - math.floor(f[a]))
    return n


def march(rec, kappa, vel, shape, delta, x_eff, eps):
    """Small-step march of one packet from its initial state ``rec`` (cell0,
    fx, fy, fz, kx, ky, kz, x0). kappa: FP64 [ncells]; vel: None or FP64
    [3, ncells] in Doppler units; shape = (nx, ny, nz). Steps of ``eps`` cell
    widths; the cell of a step is the one containing its midpoint. Returns
    (per-cell deposited weight fraction [ncells], escaped fraction)."""
    nx, ny, nz = shape
    ncells = nx * ny * nz
    c0 = int(rec["cell0"])
    r0 = np.array([c0 % nx + rec["fx"], (c0 // nx) % ny + rec["fy"], c0 // (nx * ny) + rec["fz"]])
    k = np.array([rec["kx"], rec["ky"], rec["kz"]])

    def cells_at(s):
        pos = r0[None, :] + s[:, None] * k[None, :]
        ix = np.floor(pos[:, 0]).astype(np.int64) % nx
        iy = np.floor(pos[:, 1]).astype(np.int64) % ny
        iz = np.floor(pos[:, 2]).astype(np.int64) % nz
        return ix + nx * (iy + ny * iz)

    def kdotu(cells):
        if vel is None:
            return np.zeros(cells.shape)
        return k[0] * vel[0][cells] + k[1] * vel[1][cells] + k[2] * vel[2][cells]

    # frequency in the frame of the expansion: continuous along the path
    x_hub0 = rec["x0"] + kdotu(np.array([c0]))[0]
    if rec["x0"] <= -x_eff:
        return np.zeros(ncells), 1.0
    # longest possible path: the hubble-frame frequency must fall x_eff plus
    # the largest velocity term below the start
    umax = 0.0 if vel is None else float(np.sqrt((vel ** 2).sum(axis=0)).max())
    smax = (x_hub0 + x_eff + 2.0 * umax) / delta + 2.0 * eps
    nstep = int(math.ceil(smax / eps))
    s_mid = (np.arange(nstep) + 0.5) * eps
    cells = cells_at(s_mid)
    x_gas = x_hub0 - delta * s_mid - kdotu(cells)
    below = np.nonzero(x_gas <= -x_eff)[0]
    stop = int(below[0]) if below.size else nstep
    cells, x_gas = cells[:stop], x_gas[:stop]
    dtau = kappa[cells] * np.exp(-x_gas * x_gas) / math.sqrt(math.pi) * delta * eps
    tau = np.concatenate([[0.0], np.cumsum(dtau)])
    w = np.exp(-tau)
    dep = np.bincount(cells, weights=w[:-1] - w[1:], minlength=ncells)
    return dep, float(w[-1])


def phi_cdf(x):
    return 0.5 * erfc(-x)
