"""GPU tests of the walk through a bulk-flow gradient (the flow test of
Fig. MCescape) and of the experiment drivers, through the C ABI.

The 10 Mpc slab of the oracle's pin (U_x = U0 sin(2 pi x / L), packets
emitted at x = 0): the per-cell tallies and the escaped weight against the
oracle to the parity tolerances, and every packet's escaped weight against
exp(-kappa / (1 + g mu^2) dPhi), its closed form for a uniform gradient
dv_x/dx = g H (mean difference within four standard errors). Flows much
shorter than the distance over which a streaming packet crosses the line
(v_th / H, about 5 kpc comoving) leave f_z at its static value.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import walker, physics as P
from tests.gpu_helpers import gpu_run, compare_cells, GLOBAL_REL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402
from paper_2312_11448_amd import experiments as X  # noqa: E402

N = 65536
CELL = 1e4 * W.KPC_CM / N


def _say(msg):
    print(msg, flush=True)


def slab(g, n_packets, seed=5, n=N, cell=CELL):
    delta = P.box_scalars(W.escape_slab(n, 0.0, cell, 10))["delta"]
    return W.escape_slab(n, g * n * delta / (2.0 * math.pi), cell, n_packets, seed=seed)


@pytest.mark.parametrize("g", [-0.5, 0.8])
def test_flow_slab_tallies_match_oracle(g):
    spec = slab(g, 200_000)
    ref = walker.run_box(spec)
    gr = gpu_run(spec)
    w_total = float(spec.w0) * spec.n_packets
    assert np.array_equal(gr["emitted"], ref["emitted"])
    assert gr["stats"].conserved == 1
    cmp = compare_cells(gr["A"], ref["A"], w_total)
    esc_rel = abs(gr["escaped"] - ref["escaped"]) / ref["escaped"]
    _say(f"  g {g}: {cmp}; escaped rel {esc_rel:.2e}; crossings gpu {gr['crossings']} orc {ref['crossings']}")
    assert cmp["bad"] == 0
    assert cmp["f_rel"] <= GLOBAL_REL
    # the escaped weight is 0.5 % of the emitted: its absolute error is the absorbed one's
    assert abs(gr["escaped"] - ref["escaped"]) <= GLOBAL_REL * ref["A"].sum()


@pytest.mark.parametrize("g", [-0.5, 0.5])
def test_flow_slab_packets_follow_uniform_gradient(g):
    spec = slab(g, 400_000, seed=9)
    kap = float(P.kappa_field(spec).mean())
    X_eff = P.x_eff(spec)
    with M.Simulation(spec) as sim:
        sim.emit()
        tr = sim.trace(0, spec.n_packets)
    got = np.where(tr["fate"] == 1, tr["escaped"], 0) / spec.w0
    mu2 = tr["kx"].astype(np.float64) ** 2
    dphi = np.clip(P.Phi(tr["x0"].astype(np.float64)) - P.Phi(-X_eff), 0.0, None)
    d = got - np.exp(-kap / (1.0 + g * mu2) * dphi)
    m, s = d.mean(), d.std() / math.sqrt(d.size)
    f = P.escape_uniform_gradient(kap, g, X_eff)
    _say(f"  g {g}: f_z {got.mean():.5e} (direction average {f:.5e}); mean(walked - closed form) {m:.2e} +- {s:.2e}")
    assert abs(m) <= 4.0 * s
    assert abs(got.mean() - f) <= 4.0 * got.std() / math.sqrt(got.size)


def test_escape_vs_flow_experiment():
    """The experiment driver: with lambda = 1 Mpc f_z follows (1 + g/3) f_z(0)
    (the caption's analytic result, to the statistics of 10^6 packets); with
    lambda = 0.1 kpc it stays at f_z(0)."""
    rows = X.escape_vs_flow(lams_kpc=(0.1, 1000.0), gs=(-0.5, 0.0, 0.5), n_packets=1_000_000, echo=_say)
    f = {(r["lam_kpc"], r["div_v_over_H"]): r["f_z"] for r in rows}
    for r in rows:
        assert r["crossings"] > 0
    tau = rows[0]["tau_ab"]
    f0 = P.escape_homogeneous(tau, 6.0)
    for g in (-0.5, 0.0, 0.5):
        assert f[(0.1, g)] == pytest.approx(f[(0.1, 0.0)], rel=1e-3)
        assert f[(1000.0, g)] / f[(1000.0, 0.0)] == pytest.approx(P.escape_uniform_gradient(tau, g, 6.0) / f0, rel=0.02)
    assert f[(0.1, 0.0)] == pytest.approx(f0, rel=0.06)          # four standard errors of 10^6 packets


def test_global_loss_experiment():
    """C_MC and C^mix of a clumpy box with and without its flow: the two
    C's agree to a few per cent (the paper's finding for the global loss
    rate), and removing a flow of rms 0.1 v_th changes C_MC by less than that."""
    spec = W.make_box("c2", n=48, n_packets=1_000_000)
    rows = X.global_loss(spec, echo=_say)
    by = {r["case"]: r for r in rows}
    for r in rows:
        assert 0.9 < r["loss_ratio"] < 1.1
    assert abs(by["flow"]["c_mc"] / by["no_flow"]["c_mc"] - 1.0) < 0.05
