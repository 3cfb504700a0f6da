"""FP64 oracle of recombination histories driven by the local net rate.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. It is written independently of the HIP
library.

What it computes (Jedamzik, Abel & Ali-Haimoud, arXiv:2312.11448):
  - the net recombination rate of a region, Eq. (rec) with the Peebles C of
    Eq. (Cfactor) and the local Lyman-alpha escape rate R_alpha of
    Eq. (R-alpha) (no mixing: each region keeps its own Lyman-alpha photons);
  - the full-mixing rate of Eq. (dotne-mix): C^mix from the averaged n_1s
    (R_alpha^mix = 1 / <1/R_alpha>), plus the mixing term
    -(1 - C^mix) alpha_e (n_e^2 - n_1s <n_e^2> / <n_1s>), which averages to zero;
  - x_e(z) of each region from dx_e/dz = -ndot_e / (n_H (1 + z) H), with
    n_H the region's hydrogen density, integrated in z by the classic fourth-order
    Runge-Kutta method with fixed steps (the paper integrates with a sixth-order
    one), or by scipy's implicit Radau method as a check of the stepping;
  - the 2-zone toy model of Sec. IV.C: two equally likely regions with
    Delta = 1 +- sqrt(b).
Readings: one temperature T = T_cmb0 (1 + z) serves for matter and radiation
(as in the transport); helium is left out (App. B); the start is the hydrogen
Saha equilibrium.
"""
import math

import numpy as np
from scipy import integrate

from . import physics as P


def temperature(z, cosmo):
    return cosmo.t_cmb0 * (1.0 + z)


def saha_xe(z, cosmo, delta=1.0):
    """Hydrogen Saha equilibrium x^2 / (1 - x) = (2 pi m_e k T / h^2)^{3/2}
    exp(-E_I / kT) / n_H, with n_H the region's hydrogen density."""
    T = temperature(z, cosmo)
    nH = P.n_h0(cosmo) * (1.0 + z) ** 3 * delta
    s = (2.0 * math.pi * P.M_E * P.K_B * T / P.H_PLANCK ** 2) ** 1.5 * math.exp(-P.E_ION / (P.K_B * T)) / nH
    return 2.0 / (1.0 + math.sqrt(1.0 + 4.0 / s))            # the positive root, without cancellation


def _scalars(z, cosmo, zeta):
    T = temperature(z, cosmo)
    return dict(T=T, H=P.hubble(z, cosmo, zeta), nH=P.n_h0(cosmo) * (1.0 + z) ** 3, alpha=P.alpha_e(T),
                beta=P.beta_e(T), boltz=math.exp(-P.E_ALPHA / (P.K_B * T)))


def rate_no_mixing(z, xe, delta, cosmo, zeta=1.0):
    """ndot_e (cm^-3 s^-1) of each region, Eq. (rec) with its own C."""
    s = _scalars(z, cosmo, zeta)
    xe = np.asarray(xe, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    ne = xe * s["nH"] * delta
    n1s = (1.0 - xe) * s["nH"] * delta
    R = 8.0 * math.pi * s["H"] / (P.LAMBDA_ALPHA ** 3 * n1s)
    C = (P.LAMBDA_2G + R) / (s["beta"] + P.LAMBDA_2G + R)
    return -C * (s["alpha"] * ne * ne - s["beta"] * n1s * s["boltz"])


def rate_full_mixing(z, xe, delta, weights, cosmo, zeta=1.0):
    """ndot_e of each region, Eq. (dotne-mix): averages over the regions with
    the given volume weights (summing to 1)."""
    s = _scalars(z, cosmo, zeta)
    xe = np.asarray(xe, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    ne = xe * s["nH"] * delta
    n1s = (1.0 - xe) * s["nH"] * delta
    n1s_mean = float((w * n1s).sum())
    ne2_mean = float((w * ne * ne).sum())
    R_mix = 8.0 * math.pi * s["H"] / (P.LAMBDA_ALPHA ** 3 * n1s_mean)
    C_mix = (P.LAMBDA_2G + R_mix) / (s["beta"] + P.LAMBDA_2G + R_mix)
    peebles = -C_mix * (s["alpha"] * ne * ne - s["beta"] * n1s * s["boltz"])
    mixing = -(1.0 - C_mix) * s["alpha"] * (ne * ne - n1s / n1s_mean * ne2_mean)
    return peebles + mixing, mixing


def dxe_dz(rate, z, delta, cosmo, zeta=1.0):
    """dx_e/dz of each region for the net rate `rate` (dt = -dz / ((1+z) H))."""
    s = _scalars(z, cosmo, zeta)
    return -np.asarray(rate) / (s["nH"] * np.asarray(delta, dtype=np.float64) * (1.0 + z) * s["H"])


def rk4(f, z0, z1, n_steps, y0):
    """Classic fourth-order Runge-Kutta in z with n_steps equal steps from z0
    to z1 (z1 < z0 for a history forward in time). Returns (z grid, y)."""
    h = (z1 - z0) / n_steps
    y = np.array(y0, dtype=np.float64)
    zs = [z0]
    ys = [y.copy()]
    z = z0
    for _ in range(n_steps):
        k1 = f(z, y)
        k2 = f(z + 0.5 * h, y + 0.5 * h * k1)
        k3 = f(z + 0.5 * h, y + 0.5 * h * k2)
        k4 = f(z + h, y + h * k3)
        y = y + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        z = z + h
        zs.append(z)
        ys.append(y.copy())
    return np.array(zs), np.array(ys)


def radau(f, z0, z1, y0, z_eval):
    """scipy's implicit Radau IIA integration (tight tolerances), a check of
    the fixed stepping."""
    sol = integrate.solve_ivp(f, (z0, z1), np.asarray(y0, dtype=np.float64), method="Radau", t_eval=z_eval,
                              rtol=1e-10, atol=1e-13)
    return sol.y.T


def two_zone(b=0.5):
    """Delta and weights of the 2-zone toy model (Sec. IV.C)."""
    r = math.sqrt(b)
    return np.array([1.0 + r, 1.0 - r]), np.array([0.5, 0.5])


def global_xe(xe, delta, weights):
    """X_e = <n_e> / <n_H> (Sec. II.A)."""
    w = np.asarray(weights) * np.asarray(delta)
    return (np.asarray(xe) * w).sum(axis=-1) / w.sum()


def rhs(mode, delta, weights, cosmo, zeta=1.0):
    """dx_e/dz of the regions as a function f(z, x_e) for mode "no_mixing" or
    "full_mixing"."""
    delta = np.asarray(delta, dtype=np.float64)
    if mode == "full_mixing":
        return lambda z, y: dxe_dz(rate_full_mixing(z, y, delta, weights, cosmo, zeta)[0], z, delta, cosmo, zeta)
    return lambda z, y: dxe_dz(rate_no_mixing(z, y, delta, cosmo, zeta), z, delta, cosmo, zeta)


def history(mode, delta, weights, cosmo, z0=1600.0, z1=700.0, z_eval=None, zeta=1.0, y0=None):
    """x_e(z) of the regions from Saha equilibrium at z0 (or y0): mode
    "no_mixing", "full_mixing" or "homogeneous" (one region at the mean
    density), by the implicit Radau method (near equilibrium at high z the
    equation is stiff: the relaxation to Saha is many times faster than the
    expansion)."""
    delta = np.asarray(delta, dtype=np.float64)
    if mode == "homogeneous":
        delta, weights, mode = np.array([1.0]), np.array([1.0]), "no_mixing"
    if y0 is None:
        y0 = [saha_xe(z0, cosmo, d) for d in delta]
    if z_eval is None:
        z_eval = np.linspace(z0, z1, 901)
    return np.asarray(z_eval), radau(rhs(mode, delta, weights, cosmo, zeta), z0, z1, y0, z_eval)


def evolve_mc(spec, z0, z1, n_steps, n_packets, seed, nthreads=None):
    """The Monte-Carlo driven history of one box: x_e of every cell from z0 to
    z1 by the same fourth-order Runge-Kutta stages, each an oracle transport
    and feed at the stage's redshift (T = T_cmb0 (1 + z)) with the stage's x_e
    field (binary32, kept inside [0, 1], as the library stores it; the stages
    combine in binary64), emission seed seed + ((4 i + s) << 20). Returns
    (the x_e field at z1, X_e of the field at z0 and after every step)."""
    import dataclasses
    from . import walker
    cosmo = spec.cosmo
    delta = np.asarray(spec.overdensity, dtype=np.float64).reshape(-1)
    y0 = np.asarray(spec.x_e, dtype=np.float32).reshape(-1).astype(np.float64)
    shape = np.asarray(spec.overdensity).shape
    h = (z1 - z0) / n_steps
    cz = (0.0, 0.5, 0.5, 1.0)
    field = lambda y: np.clip(y, 0.0, 1.0).astype(np.float32).reshape(shape)
    X = [float((y0 * delta).sum() / delta.sum())]
    for i in range(n_steps):
        z = z0 + i * h
        ks = []
        for s in range(4):
            y = y0 if s == 0 else y0 + cz[s] * h * ks[-1]
            zs = z + cz[s] * h
            st = dataclasses.replace(spec, z=zs, temp_K=cosmo.t_cmb0 * (1.0 + zs),
                                     x_e=field(y) if s > 0 or i > 0 else np.asarray(spec.x_e, dtype=np.float32),
                                     n_packets=int(n_packets), seed=int(seed) + ((4 * i + s) << 20))
            r = walker.run_box(st, nthreads=nthreads)
            f = P.feed(st, r["A"], r["escaped"], st.n_packets, wing=r["wing"])
            sc = P.box_scalars(st)
            with np.errstate(divide="ignore", invalid="ignore"):
                k = np.where(delta > 0, -f["ndot_e"] / (sc["n_H"] * delta * (1.0 + zs) * sc["H"]), 0.0)
            ks.append(k)
        y0 = y0 + h / 6.0 * (ks[0] + 2.0 * ks[1] + 2.0 * ks[2] + ks[3])
        xf = field(y0).reshape(-1).astype(np.float64)
        X.append(float((xf * delta).sum() / delta.sum()))
    return field(y0).reshape(-1), np.array(X)
