"""Pins of the oracle's packet walk against closed forms, brute force and
invariants (CPU only)."""
import math

import numpy as np
import pytest

from oracle import walker, brute, physics as P

W0 = 1 << 32


def homog(n=4, n_packets=20000, seed=7, kappa=5.0, delta=0.05, x_eff=6.0, vel=None):
    nc = n ** 3
    return walker.Prepared.custom((n, n, n), np.full(nc, kappa), np.ones(nc), n_packets, seed,
                                  delta, x_eff, vel=vel)


def predicted_escape(x0, kappa, x_eff):
    """Homogeneous static medium: the weight left after redshifting from x0 to
    -x_eff is w0 exp(-kappa (Phi(x0) - Phi(-x_eff)))."""
    out = np.where(x0 <= -x_eff, 1.0,
                   np.exp(-kappa * np.clip(P.Phi(x0) - P.Phi(-x_eff), 0.0, None)))
    return out * W0


@pytest.mark.parametrize("kappa,delta,x_eff", [(0.5, 0.05, 6.0), (5.0, 0.2, 6.0),
                                               (190.0, 0.0192, 6.0), (3.0, 0.1, 0.5),
                                               (40.0, 0.3, 1.5)])
def test_per_packet_escape_closed_form(kappa, delta, x_eff):
    """T1 per packet: drift, deposit and escape reproduce the exact weight
    exp(-tau_ab dPhi) of every packet (Sec. IV.A.2 solution), to the integer
    rounding of its segments, for any escape threshold."""
    prep = homog(kappa=kappa, delta=delta, n_packets=5000, x_eff=x_eff)
    r = prep.transport(records=True)
    rec = r["records"]
    pred = predicted_escape(rec["x0"], kappa, x_eff)
    got = np.where(rec["fate"] == 1, rec["escaped"], 0).astype(np.float64)
    assert np.all(np.abs(got - pred) <= 0.5 * rec["crossings"] + 1.0)
    assert np.all(rec["absorbed"] + np.where(rec["fate"] > 0, rec["escaped"], 0) == W0)


@pytest.mark.parametrize("tau", [0.1, 1.0, 10.0, 100.0, 1000.0])
def test_escape_fraction_tau_sweep(tau):
    """T1/T2: the escaped fraction equals Phi(-X) + (1 - exp(-tau(1-Phi(-X))))/tau
    over the optical-depth range of the paper's C-factor test (App. A)."""
    prep = homog(kappa=tau, delta=0.1, n_packets=40000, seed=11)
    rec = prep.transport(records=True)["records"]
    esc = np.where(rec["fate"] == 1, rec["escaped"], 0) / W0
    expect = P.escape_homogeneous(tau, 6.0)
    sigma = esc.std() / math.sqrt(esc.size)
    assert abs(esc.mean() - expect) <= 4 * sigma + 1e-12


def test_c_factor_vs_peebles_lambda0(monkeypatch):
    """App. A test problem: homogeneous universe with Lambda_2g = 0 and H -> zeta H.
    The escaped fraction is the Monte-Carlo C; it agrees with Eq. (Cfactor) to
    O(1/tau) (the streaming model keeps the exact profile integral)."""
    import workloads as W
    monkeypatch.setattr(P, "LAMBDA_2G", 0.0)
    for zeta in (1.0, 10.0, 100.0):
        spec = W.BoxSpec(n=(4, 4, 4), overdensity=W.uniform_box(4), zeta=zeta, n_packets=20000,
                         seed=3)
        r = walker.run_box(spec, records=True)
        esc = np.where(r["records"]["fate"] == 1, r["records"]["escaped"], 0) / spec.w0
        sc = P.box_scalars(spec)
        n1s = 0.9 * sc["n_H"]
        tau = sc["kappa_per_n1s"] * n1s
        c_peebles = P.peebles_c(spec.temp_K, sc["H"], n1s, lambda_2g=0.0)
        sig = esc.std() / math.sqrt(esc.size)
        assert abs(esc.mean() - c_peebles) <= 1.5 * c_peebles / tau + 4 * sig


def test_crossings_count_planes():
    """DDA pin: in a transparent homogeneous box every escaping packet visits
    exactly 1 + (grid planes crossed) cells along its straight path of length
    (x0 + X)/delta."""
    delta, x_eff = 0.07, 6.0
    prep = homog(kappa=1e-3, delta=delta, n_packets=3000, seed=21)
    rec = prep.transport(records=True)["records"]
    assert np.all(rec["fate"] == 1)
    for r in rec:
        if r["x0"] <= -x_eff:
            assert r["crossings"] == 0
            continue
        length = (r["x0"] + x_eff) / delta
        expect = brute.planes_crossed((r["fx"], r["fy"], r["fz"]), (r["kx"], r["ky"], r["kz"]),
                                      length)
        assert r["crossings"] == expect


def test_trace_path_length_scales_with_delta():
    """T10: the path walked to escape is (x0 + X)/delta cell widths, so the
    spatial kernel rescales with delta while the escaped weight depends on kappa
    alone."""
    for delta in (0.02, 0.08, 0.32):
        prep = homog(kappa=2.0, delta=delta, n_packets=200, seed=5)
        for p in range(0, 200, 17):
            t = prep.trace(p)
            rec = t["record"]
            if rec["fate"] != 1 or rec["x0"] <= -6.0:
                continue
            # the last segment is cut where x reaches -X
            last = (t["x_in"][-1] + 6.0) / delta
            assert 0.0 <= last <= t["length"][-1] + 1e-12
            walked = t["length"][:-1].sum() + last
            assert abs(walked - (rec["x0"] + 6.0) / delta) < 1e-9 * (1 + walked)
            pred = predicted_escape(np.array([rec["x0"]]), 2.0, 6.0)[0]
            assert abs(rec["escaped"] - pred) <= 0.5 * rec["crossings"] + 1


def test_conservation_and_additivity():
    """T4: sum(A) + E == w0 N exactly; packet ranges and thread counts add up
    bit for bit (integer tallies)."""
    import workloads as W
    spec = W.make_box("c1", n=16, n_packets=20000)
    prep = walker.Prepared(spec)
    full = prep.transport(nthreads=4)
    assert full["A"].sum() + full["escaped"] + full["capped_weight"] == spec.w0 * 20000
    assert full["capped"] == 0
    one = prep.transport(nthreads=1)
    assert np.array_equal(one["A"], full["A"]) and one["escaped"] == full["escaped"]
    a = prep.transport(0, 7001, nthreads=3)
    b = prep.transport(7001, 20000, nthreads=2)
    assert np.array_equal(a["A"] + b["A"], full["A"])
    assert a["escaped"] + b["escaped"] == full["escaped"]
    assert a["crossings"] + b["crossings"] == full["crossings"]


def test_galilean_invariance_uniform_flow():
    """T6: only velocity differences enter Eq. (inout); a uniform flow changes
    nothing, bit for bit."""
    import workloads as W
    base = W.make_box("c1", n=8, n_packets=5000)
    u = np.zeros((3, 8, 8, 8), dtype=np.float32)
    u[0], u[1], u[2] = 0.3, -0.2, 0.1
    moving = W.BoxSpec(**{**base.__dict__, "velocity": u})
    a = walker.run_box(base)
    b = walker.run_box(moving)
    assert P.x_eff(moving) == P.x_eff(base)
    assert np.array_equal(a["A"], b["A"]) and a["escaped"] == b["escaped"]
    assert a["crossings"] == b["crossings"]


def test_converging_flow_blueshifts():
    """Sign of the face jump: a photon moving along +x from gas receding along
    +x into gas approaching along -x sees the line shifted to the blue."""
    n = 8
    vel = np.zeros((3, n, n, n))
    vel[0, :, :, : n // 2] = 0.5
    vel[0, :, :, n // 2:] = -0.5
    prep = homog(n=n, kappa=0.01, delta=0.05, n_packets=400, vel=vel, seed=9)
    checked = 0
    for p in range(400):
        t = prep.trace(p)
        rec = t["record"]
        if rec["kx"] < 0.5:
            continue
        ix = t["cells"] % n
        for i in range(1, t["cells"].size):
            if ix[i - 1] == n // 2 - 1 and ix[i] == n // 2:
                assert t["x_in"][i] > t["x_out"][i - 1]
                assert abs(t["x_in"][i] - t["x_out"][i - 1] - rec["kx"] * 1.0) < 1e-12
                checked += 1
    assert checked > 10


@pytest.mark.parametrize("seed", [1, 2])
def test_brute_force_march_small_box(seed):
    """T7: the paper's small-step scheme (App. A steps 3-4, with the frequency
    carried in the expansion frame) converges to the walk's per-cell deposits
    as the step shrinks, on a 6^3 box with random opacity and flow."""
    n = 6
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.5, 6.0, n ** 3)
    vel = rng.normal(0.0, 0.25, (3, n ** 3))
    vmean = vel.mean(axis=1, keepdims=True)
    x_eff = 4.0 + 2.0 * np.sqrt(((vel - vmean) ** 2).sum(axis=0)).max()
    delta = 0.15
    prep = walker.Prepared.custom((n, n, n), kappa, np.ones(n ** 3), 64, seed, delta, x_eff,
                                  vel=vel)
    errs = {1e-3: 0.0, 2.5e-4: 0.0}
    for p in range(0, 64, 4):
        t = prep.trace(p)
        orc = np.bincount(t["cells"], weights=t["deposits"].astype(np.float64),
                          minlength=n ** 3) / W0
        rec = t["record"]
        esc_orc = (rec["escaped"] if rec["fate"] == 1 else 0) / W0
        for eps in errs:
            dep, esc = brute.march(rec, kappa, vel, (n, n, n), delta, x_eff, eps)
            e = max(np.abs(dep - orc).max(), abs(esc - esc_orc))
            errs[eps] = max(errs[eps], e)
    # first-order convergence in the step (the cell of a step is taken at its
    # midpoint, so each face costs O(eps))
    assert errs[2.5e-4] < 1.5e-4
    assert errs[1e-3] > 2.5 * errs[2.5e-4]


def test_escape_margin_is_final():
    """The escape threshold X_esc + 2 max|U - <U>| is final: a march that keeps
    the packet going far deeper into the red wing deposits nothing more."""
    import workloads as W
    n = 6
    rng = np.random.default_rng(3)
    vel = rng.normal(0.0, 0.5, (3, n, n, n)).astype(np.float32)
    od = rng.uniform(0.5, 1.5, (n, n, n)).astype(np.float32)
    spec = W.BoxSpec(n=(n, n, n), overdensity=od, velocity=vel, zeta=60.0, x_esc=1.0,
                     n_packets=64, seed=2)
    prep = walker.Prepared(spec)
    v = P.velocity_field(spec)
    assert prep.x_eff > 1.0 + 2.0 * 0.5
    worst = 0.0
    for p in range(64):
        t = prep.trace(p)
        rec = t["record"]
        esc_orc = (rec["escaped"] if rec["fate"] == 1 else 0) / prep.w0
        dep, esc = brute.march(rec, prep.kappa, v, (n, n, n), prep.scal["delta"],
                               prep.x_eff + 8.0, 2e-4)
        worst = max(worst, abs(esc - esc_orc))
    assert worst < 2e-3


def test_drift_per_cell_from_friedmann_light_travel():
    """delta, the red drift per cell, from first principles: light crossing a
    comoving cell while the universe expands by da redshifts by da/a; the
    comoving path is int c da / (a^2 H). One Doppler width is v_th/c in dnu/nu."""
    import workloads as W
    from scipy.integrate import quad
    spec = W.BoxSpec(n=(4, 4, 4), overdensity=W.uniform_box(4))
    sc = P.box_scalars(spec)
    a1 = 1.0 / (1.0 + spec.z)
    da = 1e-6 * a1
    hub = lambda a: P.hubble(1.0 / a - 1.0, spec.cosmo)
    chi = quad(lambda a: P.C_LIGHT / (a * a * hub(a)), a1, a1 + da, epsabs=0, epsrel=1e-12)[0]
    dnu_over_nu = da / a1
    drift_per_cm = dnu_over_nu / (sc["v_th"] / P.C_LIGHT) / chi
    assert sc["delta"] == pytest.approx(drift_per_cm * spec.cell_cm, rel=1e-5)


def test_deposits_never_negative():
    """Phi is non-decreasing, so no segment, however short, deposits a negative
    weight; the packet weight never grows."""
    import workloads as W
    spec = W.make_box("c2", n=24, n_packets=400)
    prep = walker.Prepared(spec)
    for p in range(400):
        t = prep.trace(p)
        assert (t["deposits"] >= 0).all()
