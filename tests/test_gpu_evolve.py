"""GPU tests of the recombination history driven by the Monte Carlo
(mc_lya_evolve: fourth-order Runge-Kutta in z, every stage a whole emit -
transport - feed), against the FP64 oracle driving the same stages with its
own transport and feed, and against the analytic limits of the 2-zone toy
model (Sec. IV.C).

Toleranced: the GPU's x_e after three steps (twelve transports) agrees with
the oracle's to binary32 rounding of the field (2e-6 absolute). With cells far
smaller than the distance a Lyman-alpha packet travels, the Monte Carlo is in
the full-mixing regime and its history follows Eq. (dotne-mix) to the
Monte-Carlo noise (0.3 %). With cells far larger, the global X_e still agrees
with both limits (the paper's statement); the zones' own x_e then do not reach
the no-mixing solution, because the feed takes one box-wide C for the thermal
term (a reading of the paper's full-mixing formula).
"""
import numpy as np
import pytest

import workloads as W
from oracle import recombination as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402

COSMO = W.CosmoParams()
PC = 3.0856775814913673e18
DELTA, WEIGHTS = R.two_zone(0.5)


def _say(msg):
    print(msg, flush=True)


def _start(mode, z=1300.0):
    zs, y = R.history(mode, DELTA, WEIGHTS, COSMO, z0=1600.0, z1=z, z_eval=np.linspace(1600, z, 301))
    return y[-1]


def two_zone_box(cell_pc, xe_pair, n_packets, n=8):
    """An n^3 box of alternating x-slabs with Delta = 1 +- sqrt(b)."""
    plus = np.arange(n) % 2 == 0
    od = np.broadcast_to(np.where(plus, DELTA[0], DELTA[1]).astype(np.float32), (n, n, n)).copy()
    xe = np.broadcast_to(np.where(plus, xe_pair[0], xe_pair[1]).astype(np.float32), (n, n, n)).copy()
    spec = W.BoxSpec(n=(n, n, n), overdensity=od, x_e=xe, z=1300.0, temp_K=COSMO.t_cmb0 * 1301.0,
                     cell_cm=cell_pc * PC, n_packets=n_packets, seed=5)
    return spec, plus


def test_evolve_matches_oracle_driven_history():
    """Three steps (twelve emissions, transports and feeds) from z = 1300 on a
    two-cell box: the GPU's x_e field and X_e against the oracle's."""
    y = _start("full_mixing")
    od = np.array(DELTA, dtype=np.float32).reshape(1, 1, 2)
    xe = np.array(y, dtype=np.float32).reshape(1, 1, 2)
    spec = W.BoxSpec(n=(2, 1, 1), overdensity=od, x_e=xe, z=1300.0, temp_K=COSMO.t_cmb0 * 1301.0,
                     n_packets=5000, seed=5)
    xo, Xo = R.evolve_mc(spec, 1300.0, 1297.0, 3, 5000, 5)
    with M.Simulation(spec, evolve=True) as sim:
        X = sim.evolve(1300.0, 1297.0, 3, [5000], 5)
        xg = sim.x_e_field(0).cpu().numpy().reshape(-1)
    _say(f"  gpu {xg} oracle {xo}; X gpu {X[:, 0]} oracle {Xo}")
    assert np.abs(xg - xo).max() <= 2e-6
    assert np.abs(X[:, 0] - Xo).max() <= 2e-6
    assert np.all(np.diff(X[:, 0]) < 0)                      # recombining


def test_evolve_full_mixing_regime():
    """10 pc slabs (a packet crosses hundreds of them before it is absorbed):
    from z = 1300 to 1100 the zones follow the full-mixing history of
    Eq. (dotne-mix) and not the no-mixing one."""
    y0 = _start("full_mixing")
    spec, plus = two_zone_box(10.0, y0, 20000)
    z1, steps = 1100.0, 400
    with M.Simulation(spec, evolve=True) as sim:
        X = sim.evolve(1300.0, z1, steps, [20000], 7)
        xe = sim.x_e_field(0).cpu().numpy().reshape(spec.overdensity.shape)
    zp, zm = xe[:, :, plus].mean(), xe[:, :, ~plus].mean()
    ze = np.linspace(1300.0, z1, steps + 1)
    _, yf = R.history("full_mixing", DELTA, WEIGHTS, COSMO, z0=1300.0, z1=z1, y0=y0, z_eval=ze)
    _, yn = R.history("no_mixing", DELTA, WEIGHTS, COSMO, z0=1300.0, z1=z1, y0=y0, z_eval=ze)
    _say(f"  mc zones {zp:.5f} {zm:.5f}; full mixing {yf[-1]}; no mixing {yn[-1]}")
    assert abs(zp / yf[-1][0] - 1) < 3e-3 and abs(zm / yf[-1][1] - 1) < 3e-3
    # closer to full mixing than to no mixing, zone by zone
    assert abs(zm - yf[-1][1]) < 0.3 * abs(zm - yn[-1][1])
    Xf = R.global_xe(yf, DELTA, WEIGHTS)
    assert np.abs(X[:, 0] / Xf - 1).max() < 3e-3


def test_evolve_local_regime_global_xe():
    """10 kpc slabs (packets absorbed where they are emitted): the global
    X_e agrees with both analytic limits, as the paper finds for the 2-zone
    model."""
    y0 = _start("no_mixing")
    spec, plus = two_zone_box(1e4, y0, 20000)
    z1, steps = 1100.0, 400
    with M.Simulation(spec, evolve=True) as sim:
        X = sim.evolve(1300.0, z1, steps, [20000], 7)
    ze = np.linspace(1300.0, z1, steps + 1)
    for mode in ("no_mixing", "full_mixing"):
        _, y = R.history(mode, DELTA, WEIGHTS, COSMO, z0=1300.0, z1=z1, y0=y0, z_eval=ze)
        rel = np.abs(X[:, 0] / R.global_xe(y, DELTA, WEIGHTS) - 1).max()
        _say(f"  X_e against {mode}: {rel:.2e}")
        assert rel < 1e-2


def test_evolve_errors():
    spec, _ = two_zone_box(10.0, (0.5, 0.5), 100, n=2)
    with M.Simulation(spec, evolve=True) as sim:
        with pytest.raises(M.MCLyaError):
            sim.evolve(1100.0, 1300.0, 1)                       # backwards in time
        with pytest.raises(M.MCLyaError):
            sim.evolve(1300.0, 1200.0, 0)
    # a context reserved without the evolve buffers refuses the call
    with M.Simulation(spec) as sim:
        with pytest.raises(M.MCLyaError) as e:
            sim.evolve(1300.0, 1299.0, 1)
        assert e.value.status == M.MC_LYA_ESTATE and "evolve" in str(e.value)
    uniform = W.make_box("c1", n=4, n_packets=100)
    with M.Simulation(uniform, evolve=True) as sim:
        with pytest.raises((M.MCLyaError, ValueError)):
            sim.evolve(1300.0, 1200.0, 1)                       # no x_e field
