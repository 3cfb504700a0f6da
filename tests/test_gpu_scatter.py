"""GPU parity of the resonant-scattering Monte Carlo (App. A, steps 1-8)
against the FP64 oracle, through the C ABI.

Both sides draw every random number from the same Philox counters, so a
photon's history is the same on both until a binary32 / binary64 difference
flips a decision (a rejection trial, a face-or-scattering choice): most short
histories agree event for event, and the rest agree in distribution. The
destruction test is an exact 64-bit integer comparison on both sides.
Compared: per-photon histories (the share that agrees exactly), the C factor
of the App. A test problem against Eq. (Cfactor) and against the oracle
within their combined statistical error, the loss frequency x_50, and the
integer bookkeeping (conservation, range splits).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import walker, physics as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def homog_box(zeta=1.0, profile="doppler", n_packets=2000, seed=7, n=4):
    return W.BoxSpec(n=(n, n, n), overdensity=W.uniform_box(n), zeta=zeta, n_packets=n_packets, seed=seed,
                     profile=profile)


@pytest.mark.parametrize("profile", ["doppler", "voigt"])
def test_scatter_histories_match_oracle(profile):
    """Short histories (tau_S = 6000 at zeta = 1e5, p raised to 1e-3): most
    photons have the same fate, number of scatterings and crossings and end
    cell on both sides; the rest are a few per cent."""
    spec = homog_box(zeta=1e5, profile=profile, n_packets=3000, seed=21)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    ref = prep.scatter(sc["p_ab"], p_destroy=1e-3, records=True)["records"]
    with M.Simulation(spec) as sim:
        sim.emit()
        rec = sim.scatter(p_destroy=1e-3, records=True)
        t = sim.tally()
    assert t["stats"][0].conserved == 1
    same = ((rec["fate"] == ref["fate"]) & (rec["scatterings"] == ref["scatterings"]) &
            (rec["crossings"] == ref["crossings"]) & (rec["cell_end"] == ref["cell_end"]))
    _say(f"  {profile}: identical histories {same.mean():.4f}; destroyed gpu {np.mean(rec['fate'] == 0):.4f} "
         f"orc {np.mean(ref['fate'] == 0):.4f}; mean scatterings gpu {rec['scatterings'].mean():.1f} "
         f"orc {ref['scatterings'].mean():.1f}")
    assert same.mean() > 0.9
    assert np.all(rec["cell0"] == ref["cell0"])
    assert np.abs(rec["x0"] - ref["x0"]).max() < 1e-4 * (1 + np.abs(ref["x0"]).max())
    both = same & (rec["fate"] == 1)
    assert np.all(np.abs(rec["x_end"][both] - ref["x_end"][both]) <= 1e-3 * (1 + np.abs(ref["x_end"][both])))
    assert rec["scatterings"].sum() == t["stats"][0].scatterings
    # the unwrapped displacement from emission to the last event: the counts
    # above do not pin a photon's path (a destroyed photon's scattering count
    # is set by its destruction words alone), so a trajectory that parted
    # after a flipped rejection trial can still count as the same history
    dg = np.stack([rec["dx"], rec["dy"], rec["dz"]], axis=1).astype(np.float64)
    do = np.stack([ref["dx"], ref["dy"], ref["dz"]], axis=1)
    scale = np.linalg.norm(do, axis=1)[:, None]
    close = np.all(np.abs(dg - do) <= 1e-3 * scale + 1e-7, axis=1)         # 1e-7 cell: 0.01 pc
    _say(f"  displacements within 1e-3: {close[same].mean():.4f} of the same histories")
    assert close[same].mean() > 0.98


@pytest.mark.parametrize("profile,ptau", [("doppler", 1.0), ("voigt", 10.0)])
def test_scatter_c_factor_test_problem(profile, ptau):
    """App. A test problem (Fig. Cfact) on the GPU with many photons: the
    escaped fraction against 1 / (1 + p tau_S) and against the oracle on a
    subset, within the combined statistical error."""
    spec = homog_box(zeta=1e4, profile=profile, n_packets=40000, seed=7)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    tau_s = prep.kappa.mean() / sc["p_ab"]
    pd = ptau / tau_s
    with M.Simulation(spec) as sim:
        sim.emit()
        rec = sim.scatter(p_destroy=pd, records=True)
        t = sim.tally()
        f = sim.feed()
    st = t["stats"][0]
    esc = float(np.mean(rec["fate"] == 1))
    c = 1.0 / (1.0 + ptau)
    sig = math.sqrt(c * (1 - c) / rec.size)
    ref = prep.scatter(sc["p_ab"], p_destroy=pd, records=True, p_end=3000)["records"]
    esc_o = float(np.mean(ref["fate"] == 1))
    sig_o = math.sqrt(c * (1 - c) / ref.size)
    _say(f"  {profile} p tau_S = {ptau}: gpu {esc:.4f} +- {sig:.4f}, oracle {esc_o:.4f} +- {sig_o:.4f}, "
         f"theory {c:.4f}; scatterings {st.scatterings}")
    assert abs(esc - c) <= 4 * sig + 0.01
    assert abs(esc - esc_o) <= 4 * math.hypot(sig, sig_o)
    assert st.conserved == 1
    assert st.escaped == int(np.sum(rec["escaped"]))
    # the feed's C_MC with Lambda_2g counted is the escaped fraction plus the
    # two-photon share of the destroyed weight
    lam = P.LAMBDA_2G
    w = spec.w0 * spec.n_packets
    c_mc = ((st.escaped - st.wing) + (st.absorbed + st.wing) * lam / (sc["beta"] + lam)) / w
    assert f["stats"][0].c_mc == pytest.approx(c_mc, rel=1e-12)


def test_scatter_x50():
    """Photons injected in the red wing at -40 mostly return to the core,
    those at -90 mostly do not (x_50 ~ 60, App. A)."""
    spec = homog_box(profile="voigt", n_packets=4000, seed=5)
    lost = {}
    with M.Simulation(spec) as sim:
        sim.emit()
        for X in (40.0, 90.0):
            rec = sim.scatter(p_destroy=0.0, x_inert=400.0, x0=-X, x_return=3.0, records=True)
            assert np.all((rec["fate"] == 1) | (rec["fate"] == 3))
            lost[X] = float(np.mean(rec["fate"] == 1))
    _say(f"  lost from -40: {lost[40.0]:.3f}, from -90: {lost[90.0]:.3f}")
    assert lost[40.0] < 0.4 and lost[90.0] > 0.8
    x50 = 40.0 + (0.5 - lost[40.0]) / (lost[90.0] - lost[40.0]) * 50.0
    assert 45.0 < x50 < 80.0


def test_scatter_clumpy_box_with_flow():
    """A clumpy 16^3 box with a flow (Voigt, p raised to 1e-4): the
    per-cell destroyed weight, the escaped and wing totals, agree with the
    oracle up to the few photons whose histories part; the tallies are
    conserved and the same over any split of the photon range."""
    spec = W.make_box("c2", n=16, n_packets=6000, profile="voigt", zeta=100.0, field_seed=4, seed=6)
    prep = walker.Prepared(spec)
    sc = P.box_scalars(spec)
    ref = prep.scatter(sc["p_ab"], p_destroy=1e-4, records=True)
    with M.Simulation(spec) as sim:
        sim.emit()
        rec = sim.scatter(p_destroy=1e-4, records=True)
        t = sim.tally()
        A = t["absorbed"].cpu().numpy()
        st = t["stats"][0]
    with M.Simulation(spec) as sim:
        sim.emit()
        sim.scatter(0, 1777, p_destroy=1e-4)
        sim.scatter(1777, spec.n_packets - 1777, p_destroy=1e-4)
        t2 = sim.tally()
        assert np.array_equal(t2["absorbed"].cpu().numpy(), A)
        assert t2["stats"][0].escaped == st.escaped and t2["stats"][0].scatterings == st.scatterings
    assert st.conserved == 1
    w0 = spec.w0
    rr = ref["records"]
    parted = np.mean((rec["fate"] != rr["fate"]) | (rec["cell_end"] != rr["cell_end"]))
    mismatch = np.abs(A - ref["A"]).sum() / (w0 * spec.n_packets)
    _say(f"  parted histories {parted:.4f}; tally mismatch {mismatch:.4f}; escaped gpu {st.escaped / w0:.0f} "
         f"orc {ref['escaped'] / w0:.0f}; scatterings gpu {st.scatterings} orc {ref['scatterings']}")
    assert mismatch <= 2 * parted + 1e-12
    assert parted < 0.1
    assert abs(st.escaped - ref["escaped"]) <= 2 * parted * w0 * spec.n_packets + 1


def test_scatter_batch_equals_boxes_alone():
    """Two boxes in one context (the multi-box kernel) give, box by box, the
    same tallies, totals and histories as each box scattered alone (a
    photon's random numbers depend on its box's seed and its id in the box)."""
    a = W.make_box("c2", n=12, n_packets=3000, profile="voigt", zeta=1e3, field_seed=8, seed=11)
    b = homog_box(zeta=1e5, profile="doppler", n_packets=2000, seed=12, n=6)
    alone = []
    for spec in (a, b):
        with M.Simulation(spec) as sim:
            sim.emit()
            rec = sim.scatter(p_destroy=2e-4, records=True)
            t = sim.tally()
            alone.append((t["absorbed"].cpu().numpy(), t["stats"][0], rec))
    with M.Simulation([a, b]) as sim:
        sim.emit()
        rec = sim.scatter(p_destroy=2e-4, records=True)
        t = sim.tally()
        A = t["absorbed"].cpu().numpy()
        off = sim.cell_off
    for i, (A1, st1, rec1) in enumerate(alone):
        st = t["stats"][i]
        assert np.array_equal(A[off[i]:off[i + 1]], A1), i
        assert (st.escaped, st.wing, st.scatterings, st.crossings) == (st1.escaped, st1.wing, st1.scatterings,
                                                                       st1.crossings), i
        assert st.conserved == 1
    n0 = a.n_packets
    for f in ("fate", "scatterings", "crossings", "x_end"):
        assert np.array_equal(rec[f][:n0], alone[0][2][f]) and np.array_equal(rec[f][n0:], alone[1][2][f]), f


def test_scatter_default_options_use_p_ab():
    """NULL options: each box's own p_ab, the same as asking for it."""
    spec = homog_box(zeta=1e5, n_packets=20000, seed=3)
    out = []
    for opts in (None, -1.0):
        with M.Simulation(spec) as sim:
            sim.emit()
            if opts is None:
                M.mc_lya_scatter(sim.ctx, 0, spec.n_packets)
            else:
                sim.scatter(p_destroy=opts)
            t = sim.tally()
            out.append((t["absorbed"].cpu().numpy(), t["stats"][0].escaped, t["stats"][0].scatterings))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]
    assert out[0][0].sum() > 0                       # some photons are destroyed


def test_scatter_errors():
    """Invalid calls return an error status, leave the context usable, and
    scatter nothing."""
    spec = homog_box(zeta=1e5, n_packets=500, seed=2)
    with M.Simulation(spec) as sim:
        with pytest.raises(M.MCLyaError):
            sim.scatter()                                       # before any emission
        sim.emit()
        bad = [dict(first=400, count=101), dict(x_inert=-1.0), dict(x_inert=float("inf")),
               dict(p_destroy=1.5), dict(p_destroy=float("nan")), dict(max_events=1 << 33),
               dict(x_return=-0.5), dict(x0=float("nan"))]
        for kw in bad:
            with pytest.raises(M.MCLyaError):
                sim.scatter(**kw)
        t = sim.tally()
        assert t["stats"][0].scatterings == 0 and int(t["absorbed"].sum().item()) == 0
        sim.scatter(0, 0)                                       # an empty range is fine
        rec = sim.scatter(p_destroy=1.0, records=True)          # every photon destroyed at its first scattering
        assert np.all((rec["fate"] == 0) | (rec["fate"] == 1))
        assert np.all(rec["scatterings"][rec["fate"] == 0] == 1)
        assert sim.tally()["stats"][0].conserved == 1
