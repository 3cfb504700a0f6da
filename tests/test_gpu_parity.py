"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bit-exact: Philox words, emission allocation, the conservation identity on
each side, and the GPU's own run-to-run / launch-configuration / range-split /
batch-vs-alone equality. Toleranced (FP32 walk vs FP64 oracle): per-cell
absorbed weight within 1e-3 relative plus a floor of 1e-6 of the mean cell,
global absorbed fraction within 1e-5 relative.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import walker
from tests.gpu_helpers import gpu_run, compare_cells, GLOBAL_REL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_TILED = 1_000_000            # MC_LYA_OPT_TILE_SHARE value that tiles every box


def _say(msg):
    print(msg, flush=True)


def test_philox_known_answers_on_device():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(t, 16) for t in line.split()])
    rows = np.array(rows, dtype=np.uint64).astype(np.uint32)
    rng = np.random.default_rng(0)
    extra = rng.integers(0, 2 ** 32, size=(1000, 6), dtype=np.uint64).astype(np.uint32)
    ctr = np.concatenate([rows[:, 0:4], extra[:, 0:4]])
    key = np.concatenate([rows[:, 4:6], extra[:, 4:6]])
    d_ctr = torch.from_numpy(ctr.view(np.int32).copy()).cuda()
    d_key = torch.from_numpy(key.view(np.int32).copy()).cuda()
    d_out = torch.empty_like(d_ctr)
    M.mc_lya_philox4x32_10(d_ctr.data_ptr(), d_key.data_ptr(), d_out.data_ptr(), ctr.shape[0])
    torch.cuda.synchronize()
    out = d_out.cpu().numpy().view(np.uint32)
    assert np.array_equal(out[:3], rows[:, 6:10])
    for i in range(3, ctr.shape[0], 97):
        assert np.array_equal(out[i], walker.philox4x32_10(ctr[i], key[i]))


def test_packet_initial_states_match_oracle():
    spec = W.make_box("c2", n=16, n_packets=4000)
    prep = walker.Prepared(spec)
    ref = prep.transport(records=True)["records"]
    with M.Simulation(spec) as sim:
        sim.emit()
        tr = sim.trace(0, spec.n_packets)
    assert np.array_equal(tr["cell0"].astype(np.int64), ref["cell0"])
    for f in ("fx", "fy", "fz"):
        assert np.array_equal(tr[f].astype(np.float64), ref[f])      # exact binary32 uniforms
    for f in ("kx", "ky", "kz"):
        assert np.abs(tr[f] - ref[f]).max() < 1e-6
    assert np.abs(tr["x0"] - ref["x0"]).max() < 1e-5 * (1 + np.abs(ref["x0"]).max())
    # per-packet outcomes
    assert np.mean(tr["fate"] == ref["fate"]) > 0.999
    both = tr["fate"] == ref["fate"]
    assert np.mean(tr["crossings"][both] == ref["crossings"][both]) > 0.995
    w0 = float(spec.w0)
    esc_diff = np.abs(tr["escaped"].astype(np.float64) - ref["escaped"]) / w0
    assert esc_diff.max() < 1e-3


@pytest.mark.parametrize("case", ["c1", "ragged_flow_source", "c2_small", "max_weight"])
def test_tallies_match_oracle(case):
    if case == "c1":
        spec = W.make_box("c1")
    elif case == "max_weight":
        # the largest packet weight the ABI takes, 2^32 - 1: its binary32 value
        # is 2^32 itself, so every deposit of a whole packet must be capped
        # at the integer weight without leaving the unsigned range
        spec = W.make_box("c2", n=24, n_packets=200_000, w0=(1 << 32) - 1, zeta=0.3)
    elif case == "ragged_flow_source":
        rng = np.random.default_rng(12)
        n = (13, 7, 11)
        od = rng.lognormal(0.0, 0.5, size=n[::-1]).astype(np.float32)
        vel = rng.normal(0.0, 0.2, size=(3,) + n[::-1]).astype(np.float32)
        src = (od * od * rng.uniform(0.5, 1.5, size=n[::-1])).astype(np.float32)
        src[0, 0, :3] = 0.0
        spec = W.BoxSpec(n=n, overdensity=od, velocity=vel, source=src, n_packets=30_000,
                         seed=77, zeta=3.0)
    else:
        spec = W.make_box("c2", n=48, n_packets=300_000)
    _say(f"case {case}: {spec.n} packets {spec.n_packets}")
    ref = walker.run_box(spec)
    g = gpu_run(spec)
    w_total = float(spec.w0) * spec.n_packets
    assert np.array_equal(g["emitted"], ref["emitted"])
    assert g["stats"].conserved == 1
    assert ref["A"].sum() + ref["escaped"] == spec.w0 * spec.n_packets
    cmp = compare_cells(g["A"], ref["A"], w_total)
    _say(f"  {cmp}; crossings gpu {g['crossings']} orc {ref['crossings']}")
    assert cmp["bad"] == 0
    assert cmp["f_rel"] <= GLOBAL_REL
    assert abs(g["crossings"] - ref["crossings"]) <= 1e-4 * ref["crossings"] + 10


def test_c2_full_size_parity():
    spec = W.make_box("c2")
    _say(f"c2 full: {spec.n} packets {spec.n_packets}")
    ref = walker.run_box(spec)
    g = gpu_run(spec)
    w_total = float(spec.w0) * spec.n_packets
    assert np.array_equal(g["emitted"], ref["emitted"])
    assert g["stats"].conserved == 1
    cmp = compare_cells(g["A"], ref["A"], w_total)
    _say(f"  {cmp}; crossings gpu {g['crossings']} orc {ref['crossings']}")
    if cmp["bad"]:
        tol = 1e-3 * np.abs(ref["A"]) + 1e-6 * ref["A"].mean()
        idx = np.nonzero(np.abs(g["A"] - ref["A"]) > tol)[0][:10]
        for i in idx:
            _say(f"  cell {i}: gpu {g['A'][i]} orc {ref['A'][i]} tol {tol[i]:.0f}")
    assert cmp["bad"] == 0
    assert cmp["f_rel"] <= GLOBAL_REL


def test_launch_configuration_and_ranges_bitwise():
    spec = W.make_box("c2", n=32, n_packets=200_000)
    base = gpu_run(spec)
    variants = [
        {M.MC_LYA_OPT_KERNEL: 1},
        {M.MC_LYA_OPT_KERNEL: 0},
        {M.MC_LYA_OPT_KERNEL: 2, M.MC_LYA_OPT_TILE_SHARE: ALL_TILED},
        {M.MC_LYA_OPT_TILE_SHARE: ALL_TILED, M.MC_LYA_OPT_TILE_CHUNK: 7, M.MC_LYA_OPT_TILE_REFILL: 1},
        {M.MC_LYA_OPT_TILE_SHARE: ALL_TILED, M.MC_LYA_OPT_TILE_CHUNK: 1024, M.MC_LYA_OPT_TILE_REFILL: 64},
        {M.MC_LYA_OPT_KERNEL: 2, M.MC_LYA_OPT_TILE_SHARE: 0},
        {M.MC_LYA_OPT_BLOCK: 64, M.MC_LYA_OPT_WAVES_PER_CU: 8},
        {M.MC_LYA_OPT_CHUNK: 7, M.MC_LYA_OPT_REFILL: 1, M.MC_LYA_OPT_QUEUES: 1},
        {M.MC_LYA_OPT_QUEUES: 64, M.MC_LYA_OPT_CHUNK: 1},
        {M.MC_LYA_OPT_CHUNK: 4096, M.MC_LYA_OPT_REFILL: 64, M.MC_LYA_OPT_BLOCK: 128},
    ]
    for opt in variants:
        g = gpu_run(spec, options=opt)
        assert np.array_equal(g["A"], base["A"]), opt
        assert g["escaped"] == base["escaped"] and g["crossings"] == base["crossings"]
    split = gpu_run(spec, ranges=[(0, 12345), (12345, 150000), (150000, 200000)])
    assert np.array_equal(split["A"], base["A"])
    assert split["escaped"] == base["escaped"]
    again = gpu_run(spec)
    assert np.array_equal(again["A"], base["A"])


def test_tiled_batches_give_the_same_integers():
    """A context that reserves hand-over state for fewer packets than an
    emission (mc_lya_limits.batch_packets) walks it in batches: the same
    integers as one batch."""
    spec = W.make_box("c2", n=32, n_packets=200_000)
    tiled = {M.MC_LYA_OPT_TILE_SHARE: ALL_TILED}
    base = gpu_run(spec, options=tiled)
    with M.Simulation(spec, batch_packets=47_000) as sim:
        sim.set_option(M.MC_LYA_OPT_TILE_SHARE, ALL_TILED)
        sim.emit()
        sim.transport()
        t = sim.tally()
    assert np.array_equal(t["absorbed"].cpu().numpy(), base["A"])
    assert t["stats"][0].escaped == base["escaped"] and t["stats"][0].crossings == base["crossings"]


def test_batch_equals_boxes_alone():
    boxes = [W.make_box("c2", n=n, n_packets=p, field_seed=fs, seed=s)
             for n, p, fs, s in ((12, 20000, 5, 1), (20, 50000, 6, 2), (9, 7000, 7, 3))]
    boxes[1].z = 900.0
    boxes[1].temp_K = 2.7255 * 901
    alone = [gpu_run(b) for b in boxes]
    with M.Simulation(boxes) as sim:
        sim.emit()
        sim.transport()
        t = sim.tally()
    A = t["absorbed"].cpu().numpy()
    for i, b in enumerate(boxes):
        lo, hi = sim.cell_off[i], sim.cell_off[i + 1]
        assert np.array_equal(A[lo:hi], alone[i]["A"])
        assert t["stats"][i].escaped == alone[i]["escaped"]
        assert t["stats"][i].crossings == alone[i]["crossings"]
        assert t["stats"][i].conserved == 1


def test_uniform_flow_changes_nothing():
    base = W.make_box("c1", n=16, n_packets=20000)
    u = np.zeros((3, 16, 16, 16), dtype=np.float32)
    u[0], u[1], u[2] = 0.3, -0.2, 0.1
    moving = W.BoxSpec(**{**base.__dict__, "velocity": u})
    zero = W.BoxSpec(**{**base.__dict__, "velocity": np.zeros_like(u)})
    a, b, c = gpu_run(base), gpu_run(moving), gpu_run(zero)
    assert np.array_equal(b["A"], c["A"]) and b["escaped"] == c["escaped"]
    assert b["stats"].x_eff == base.x_esc
    # the kappa-only record and the (kappa, U) record walk identically
    assert np.array_equal(a["A"], c["A"])


def test_feed_matches_oracle_feed():
    """The feed (ndot_e, M_c, C_MC, C^mix, x_e) from the library's own
    transport against the oracle's feed from the oracle's own walk of the same
    box (no input of the oracle comes from the GPU). The tallies agree per cell
    within 1e-3 A_c + 1e-6 mean(A) and globally within 1e-5, so: M_c within
    2e-3 relative where A_c is not tiny, ndot_e per cell within 2e-3 of its
    absorbed term plus 2e-3 of the thermal term, C_MC within 1e-3 relative;
    C^mix and x_e depend on the fields only (1e-9)."""
    from oracle import physics as P
    spec = W.make_box("c2", n=24, n_packets=50000)
    with M.Simulation(spec) as sim:
        sim.emit()
        sim.transport()
        sim.tally()
        f = sim.feed()
    orc = walker.run_box(spec)
    ref = P.feed(spec, orc["A"], orc["escaped"], spec.n_packets)
    nd = f["ndot_e"].cpu().numpy()
    sc = P.box_scalars(spec)
    reion = sc["beta"] / (sc["beta"] + P.LAMBDA_2G)
    a = np.abs(ref["absorbed_rate"])
    thermal = np.abs(ref["c_mc"] * sc["beta"] * P.n1s_field(spec) * ref["boltzmann"])
    tol = reion * (2e-3 * a + 2e-6 * a.mean()) + 2e-3 * thermal + 1e-12 * np.abs(ref["ndot_e"]).max()
    assert (np.abs(nd - ref["ndot_e"]) <= tol).all()
    mix = f["mix_corr"].cpu().numpy().astype(np.float64)
    big = orc["A"] > 1e-2 * orc["A"].mean()
    assert np.allclose(mix[big], ref["mix_corr"][big], rtol=2e-3, atol=0.0)
    st = f["stats"][0]
    assert st.c_mc == pytest.approx(ref["c_mc"], rel=1e-3)
    assert st.c_mix == pytest.approx(ref["c_mix"], rel=1e-9)
    assert st.x_e_global == pytest.approx(ref["x_e_global"], rel=1e-9)


def test_sampled_packets_at_full_256_size():
    spec = W.make_box("c3")
    prep = walker.Prepared(spec)
    n = spec.n_packets
    ids = np.unique(np.linspace(0, n - 1, 3000).astype(np.uint64))
    ref = prep.records(ids)
    with M.Simulation(spec) as sim:
        sim.emit()
        sim.transport()
        t = sim.tally(want_emitted=True)
        st = t["stats"][0]
        assert st.conserved == 1 and st.capped_packets == 0
        em = t["emitted"].cpu().numpy()
        assert np.array_equal(em, prep.emitted_per_cell)
        recs = np.concatenate([sim.trace(int(i), 1) for i in ids])
    assert np.array_equal(recs["cell0"].astype(np.int64), ref["cell0"])
    same = recs["fate"] == ref["fate"]
    assert same.mean() > 0.995
    w0 = float(spec.w0)
    assert np.abs(recs["escaped"][same].astype(np.float64) - ref["escaped"][same]).max() / w0 < 2e-3
    # global absorbed fraction vs the oracle's estimate from the sample
    f_gpu = t["absorbed"].sum().item() / (w0 * n)
    esc = np.where(ref["fate"] == 1, ref["escaped"], 0) / w0
    f_orc = 1.0 - esc.mean()
    assert abs(f_gpu - f_orc) <= 4 * esc.std() / np.sqrt(esc.size) + 1e-6


def test_errors_and_cap():
    bad = W.make_box("c1", n=8, n_packets=100)
    bad.overdensity = bad.overdensity.copy()
    bad.overdensity[1, 2, 3] = np.nan
    with pytest.raises(M.MCLyaError) as e:
        M.Simulation(bad)
    assert e.value.status == M.MC_LYA_EINVAL and "overdensity" in str(e.value)
    neg = W.make_box("c1", n=8, n_packets=100)
    neg.x_e = np.full((8, 8, 8), 0.1, dtype=np.float32)
    neg.x_e[0, 0, 0] = 1.5
    with pytest.raises(M.MCLyaError) as e:
        M.Simulation(neg)
    assert "x_e" in str(e.value)
    spec = W.make_box("c1", n=8, n_packets=1000)
    with M.Simulation(spec) as sim:
        with pytest.raises(M.MCLyaError) as e:
            sim.transport()
        assert e.value.status == M.MC_LYA_ESTATE
        with pytest.raises(M.MCLyaError) as e:
            sim.emit(n_packets=[1 << 33])
        assert e.value.status == M.MC_LYA_EOVERFLOW
        # more packets than the context reserved room for at init
        with pytest.raises(M.MCLyaError) as e:
            sim.emit(n_packets=[1001])
        assert e.value.status == M.MC_LYA_EINVAL and "max_packets" in str(e.value)
        sim.emit(n_packets=[0])
        sim.transport()
        t = sim.tally()
        assert t["stats"][0].conserved == 1 and int(t["absorbed"].sum().item()) == 0
        sim.set_option(M.MC_LYA_OPT_MAX_CROSSINGS, 3)
        sim.emit()
        sim.transport()
        t = sim.tally(check=False)
        assert t["status"] == M.MC_LYA_ECAP
        st = t["stats"][0]
        assert st.capped_packets > 0 and st.conserved == 1
        with pytest.raises(M.MCLyaError) as e:
            M.mc_lya_transport_range(sim.ctx, 900, 200)
        assert e.value.status == M.MC_LYA_EINVAL
        # options outside their ranges are refused and leave the context usable
        for opt, bad in ((M.MC_LYA_OPT_KERNEL, 3), (M.MC_LYA_OPT_BLOCK, 96), (M.MC_LYA_OPT_REFILL, 0),
                         (M.MC_LYA_OPT_TILE_CHUNK, 2000), (M.MC_LYA_OPT_TILE_REFILL, 65),
                         (M.MC_LYA_OPT_DEFER, -1), (M.MC_LYA_OPT_TILE_SHARE, -5), (M.MC_LYA_OPT_GRAPH, 2),
                         (M.MC_LYA_OPT_GRAPH_GENS, 8), (M.MC_LYA_OPT_QUEUES, 0), (M.MC_LYA_OPT_TAIL, -1),
                         (M.MC_LYA_OPT_BESIDE, 33), (99, 1)):
            with pytest.raises(M.MCLyaError) as e:
                sim.set_option(opt, bad)
            assert e.value.status == M.MC_LYA_EINVAL, opt
        with pytest.raises(M.MCLyaError) as e:
            M.mc_lya_autotune(sim.ctx, 0)
        assert e.value.status == M.MC_LYA_EINVAL
        sim.set_option(M.MC_LYA_OPT_MAX_CROSSINGS, 1_000_000)
        sim.emit()
        sim.transport()
        assert sim.tally()["stats"][0].conserved == 1


@pytest.mark.parametrize("shape", [(16, 16, 16), (9, 9, 9), (20, 33, 17), (48, 16, 40), (5, 70, 3),
                                   (1, 33, 40), (40, 1, 1), (1, 1, 1)])
def test_tiled_walk_equals_global_walk(shape):
    """The tile-decomposed walk (LDS tallies, packets handed between tiles)
    gives the same integers as the walk with device-wide atomics: tiles that
    span an axis and wrap onto themselves, thin last tiles, two tiles along an
    axis (one neighbour on both sides), axes one cell thick (a packet crossing
    such a face re-enters its own cell) and a single-cell box."""
    rng = np.random.default_rng(sum(shape))
    od = rng.lognormal(0.0, 0.6, size=shape[::-1]).astype(np.float32)
    vel = rng.normal(0.0, 0.15, size=(3,) + shape[::-1]).astype(np.float32)
    spec = W.BoxSpec(n=shape, overdensity=od, velocity=vel, n_packets=60_000, seed=5)
    ref = gpu_run(spec, options={M.MC_LYA_OPT_KERNEL: 0})
    tiled = {M.MC_LYA_OPT_KERNEL: 2, M.MC_LYA_OPT_TILE_SHARE: ALL_TILED}
    # deferral of thin waves (off, default, always) with every generation
    # walked by tiles (tail 0); the tail walk taking over after generation 0
    # (tail: the whole batch) or once under a third of it is in flight
    for defer, tail in ((0, 0), (8, 0), (64, 0), (16, 1_000_000), (16, 333_333)):
        g = gpu_run(spec, options={**tiled, M.MC_LYA_OPT_DEFER: defer, M.MC_LYA_OPT_TAIL: tail})
        assert np.array_equal(g["A"], ref["A"]), (defer, tail)
        assert g["escaped"] == ref["escaped"] and g["crossings"] == ref["crossings"]
    part = gpu_run(spec, options={**tiled, M.MC_LYA_OPT_TAIL: 0}, ranges=[(0, 17), (17, 31000), (31000, 60000)])
    assert np.array_equal(part["A"], ref["A"])
    part = gpu_run(spec, options={**tiled, M.MC_LYA_OPT_TAIL: 100_000}, ranges=[(0, 17), (17, 31000), (31000, 60000)])
    assert np.array_equal(part["A"], ref["A"])


def _batch_run(boxes, options, ranges=None):
    with M.Simulation(boxes) as sim:
        sim.set_option(M.MC_LYA_OPT_TIMING, 1)
        for k, v in options.items():
            sim.set_option(k, v)
        sim.emit()
        if ranges is None:
            sim.transport()
        else:
            for a, b in ranges:
                sim.transport(a, b - a)
        t = sim.tally()
        _, launches = sim.kernel_time()
        return (t["absorbed"].cpu().numpy(), [(s.escaped, s.crossings, s.conserved) for s in t["stats"]],
                launches)


def test_mixed_tiled_and_persistent_batch():
    """Kernel 2 on a batch walks boxes with enough tiles by tiles and a box
    with a single, crowded tile by the persistent walk, in the same
    transport (beside the tile generations on a stream of its own, or after
    them); the integers equal those of either walk alone, also over packet
    ranges that cut through boxes."""
    boxes = [W.make_box("c2", n=64, n_packets=20_000, field_seed=11, seed=1),
             W.make_box("c2", n=16, n_packets=100_000, field_seed=12, seed=2),
             W.make_box("c2", n=40, n_packets=5_000, field_seed=13, seed=3)]
    ref_A, ref_s, _ = _batch_run(boxes, {M.MC_LYA_OPT_KERNEL: 0})
    assert all(c == 1 for _, _, c in ref_s)
    tiled_A, tiled_s, n_tiled = _batch_run(boxes, {M.MC_LYA_OPT_TILE_SHARE: ALL_TILED, M.MC_LYA_OPT_TAIL: 0})
    mixed_A, mixed_s, n_mixed = _batch_run(boxes, {M.MC_LYA_OPT_TAIL: 0})
    # all-tiled: whole rounds of 16 generations; mixed: the same plus one persistent launch
    assert n_tiled % 16 == 0 and n_mixed % 16 == 1
    tail_A, tail_s, n_tail = _batch_run(boxes, {})
    assert np.array_equal(tail_A, ref_A) and tail_s == ref_s
    assert np.array_equal(tiled_A, ref_A) and tiled_s == ref_s
    assert np.array_equal(mixed_A, ref_A) and mixed_s == ref_s
    after_A, after_s, n_after = _batch_run(boxes, {M.MC_LYA_OPT_TAIL: 0, M.MC_LYA_OPT_BESIDE: 0})
    assert np.array_equal(after_A, ref_A) and after_s == ref_s and n_after == n_mixed
    split_A, split_s, _ = _batch_run(boxes, {}, ranges=[(0, 15_000), (15_000, 118_000), (118_000, 125_000)])
    assert np.array_equal(split_A, ref_A) and split_s == ref_s


def _low_z_box(n, packets, seed):
    """A box at z = 830: small opacity, packets walk hundreds of cells."""
    b = W.make_box("c2", n=n, n_packets=packets, field_seed=20 + seed, seed=seed)
    b.z = 830.0
    b.temp_K = 2.7255 * 831.0
    return b


def test_graph_replay_equals_eager():
    """MC_LYA_OPT_GRAPH: the captured transport (tile generations plus the
    persistent walk of the untiled box), replayed over several emissions with
    eager work in between, gives the eager integers every time; a replay that
    needs more generations than were captured finishes eagerly and the next
    capture takes enough."""
    boxes = [W.make_box("c2", n=64, n_packets=20_000, field_seed=11, seed=1),
             W.make_box("c2", n=16, n_packets=100_000, field_seed=12, seed=2),
             _low_z_box(40, 5_000, 3)]
    seeds_list = [[1, 2, 3], [7, 8, 9], [1, 2, 3]]
    eager = []
    for seeds in seeds_list[:2]:
        with M.Simulation(boxes) as sim:
            sim.emit(seeds)
            sim.transport()
            t = sim.tally()
            eager.append((t["absorbed"].cpu().numpy(), [(s.escaped, s.crossings) for s in t["stats"]]))
    eager.append(eager[0])
    with M.Simulation(boxes) as sim:
        sim.set_option(M.MC_LYA_OPT_GRAPH, 1)
        sim.set_option(M.MC_LYA_OPT_GRAPH_GENS, 16)
        sim.set_option(M.MC_LYA_OPT_TAIL, 0)          # every generation by tiles: the budget runs out
        sim.set_option(M.MC_LYA_OPT_TIMING, 1)
        launches = []
        for seeds, (ref_A, ref_s) in zip(seeds_list, eager):
            sim.emit(seeds)
            sim.transport()
            t = sim.tally()
            launches.append(sim.kernel_time()[1])
            assert np.array_equal(t["absorbed"].cpu().numpy(), ref_A)
            assert [(s.escaped, s.crossings) for s in t["stats"]] == ref_s
            assert all(s.conserved == 1 for s in t["stats"])
        _say(f"  launches per transport (graph replay + eager rounds): {launches}")
        # the first replay ran out of captured generations; later ones did not
        assert launches[0] > 1 and launches[1] == 1 and launches[2] == 1


def test_coarse_timing_counts_the_same_launches():
    """Timing 2 (one event pair around each transport's walk) counts the walk
    launches that timing 1 (a pair around every launch) times one by one, on
    the same emission; on a graph replay it counts the captured generations
    and the tail walk. The integers do not depend on the timing mode."""
    box = W.make_box("c2", n=64, n_packets=50_000, field_seed=11, seed=1)
    with M.Simulation([box]) as sim:
        sim.set_option(M.MC_LYA_OPT_TILE_SHARE, ALL_TILED)
        res = {}
        for mode in (0, 1, 2):
            sim.set_option(M.MC_LYA_OPT_TIMING, mode)
            sim.emit()
            sim.transport()
            t = sim.tally()
            res[mode] = (t["absorbed"].cpu().numpy(), sim.kernel_time())
        assert np.array_equal(res[1][0], res[0][0]) and np.array_equal(res[2][0], res[0][0])
        (ms1, n1), (ms2, n2) = res[1][1], res[2][1]
        _say(f"  timing 1: {n1} launches {ms1:.3f} ms; timing 2: {n2} launches {ms2:.3f} ms")
        assert n1 == n2 and n1 >= 2
        assert ms1 > 0 and 0.25 * ms1 < ms2 < 4.0 * ms1
        sim.set_option(M.MC_LYA_OPT_GRAPH, 1)
        for _ in range(2):
            sim.emit()
            sim.transport()
            t = sim.tally()
            ms, n = sim.kernel_time()
            assert np.array_equal(t["absorbed"].cpu().numpy(), res[0][0])
            assert n == 64 + 1 and ms > 0          # the default budget of 64 generations, and the tail walk


def test_autotune_changes_speed_only():
    boxes = [W.make_box("c2", n=48, n_packets=60_000, field_seed=31, seed=4),
             _low_z_box(24, 20_000, 5)]
    with M.Simulation(boxes) as sim:
        sim.emit()
        sim.transport()
        ref = sim.tally()
        sim.emit()
        r = sim.autotune(1)
        _say(f"  tuned: kernel {r.kernel} share {r.tile_share} block {r.block} waves {r.waves_per_cu} "
             f"chunk {r.chunk} refill {r.refill}: {r.best_ms:.3f} ms (start {r.start_ms:.3f} ms, "
             f"{r.trials} trials)")
        assert r.trials >= 11 and r.best_ms <= r.start_ms
        sim.transport()
        t = sim.tally()
        assert np.array_equal(t["absorbed"].cpu().numpy(), ref["absorbed"].cpu().numpy())
        assert [s.escaped for s in t["stats"]] == [s.escaped for s in ref["stats"]]


@pytest.mark.parametrize("case", ["transparent", "opaque", "single_source_cell", "one_cell", "one_cell_thick"])
def test_degenerate_boxes_match_oracle(case):
    """x_e = 1 (no neutral hydrogen: nothing is absorbed, every packet walks
    to -x_eff), a box 100 times more opaque than the paper's (absorption in
    the emission cell), all emission in one cell, a box of one cell (every
    face leads back into it) and a box one cell thick along x."""
    base = W.make_box("c2", n=20, n_packets=40_000, field_seed=8, seed=9)
    if case == "transparent":
        spec = W.BoxSpec(**{**base.__dict__, "x_e_uniform": 1.0})
    elif case == "opaque":
        spec = W.BoxSpec(**{**base.__dict__, "zeta": 0.01})
    elif case in ("one_cell", "one_cell_thick"):
        shape = (1, 1, 1) if case == "one_cell" else (1, 24, 24)
        rng = np.random.default_rng(77)
        od = rng.lognormal(0.0, 0.5, size=shape[::-1]).astype(np.float32)
        vel = rng.normal(0.0, 0.1, size=(3,) + shape[::-1]).astype(np.float32)
        spec = W.BoxSpec(**{**base.__dict__, "n": shape, "overdensity": od, "velocity": vel,
                            "n_packets": 20_000})
    else:
        src = np.zeros_like(base.overdensity)
        src[7, 3, 11] = 1.0
        spec = W.BoxSpec(**{**base.__dict__, "source": src})
    ref = walker.run_box(spec)
    g = gpu_run(spec)
    w_total = float(spec.w0) * spec.n_packets
    assert np.array_equal(g["emitted"], ref["emitted"])
    assert g["stats"].conserved == 1
    cmp = compare_cells(g["A"], ref["A"], w_total)
    _say(f"  {case}: {cmp}; escaped gpu {g['escaped']} orc {ref['escaped']}")
    assert cmp["bad"] == 0
    if case == "transparent":
        assert int(g["A"].sum()) == 0 and g["escaped"] == spec.w0 * spec.n_packets
        assert ref["escaped"] == spec.w0 * spec.n_packets
    else:
        assert cmp["f_rel"] <= GLOBAL_REL
    assert abs(g["crossings"] - ref["crossings"]) <= 1e-4 * ref["crossings"] + 10


def test_largest_batch_of_boxes():
    """1024 boxes (the most one context takes) of 4^3 cells: every box
    conserves, and sampled boxes equal the same box alone, bit for bit."""
    boxes = [W.make_box("c1", n=4, n_packets=200, field_seed=1000 + b, seed=b) for b in range(1024)]
    with M.Simulation(boxes) as sim:
        sim.emit()
        sim.transport()
        t = sim.tally()
        A = t["absorbed"].cpu().numpy()
        assert all(s.conserved == 1 for s in t["stats"])
        for b in (0, 511, 1023):
            alone = gpu_run(boxes[b])
            lo, hi = sim.cell_off[b], sim.cell_off[b + 1]
            assert np.array_equal(A[lo:hi], alone["A"]) and t["stats"][b].escaped == alone["escaped"]


def test_loaded_fields_give_a_fresh_contexts_integers():
    """Fields loaded into an open context (mc_lya_refresh over the same device
    arrays) walk to the same integers as a context made for them."""
    a = W.make_box("c2", n=24, n_packets=40_000, field_seed=11, seed=5)
    b = W.make_box("c2", n=24, n_packets=40_000, field_seed=12, seed=6)
    fresh = gpu_run(b)
    with M.Simulation(a) as sim:
        sim.emit()
        sim.transport()
        sim.tally()
        sim.load_fields(b)
        sim.emit()
        sim.transport()
        t = sim.tally()
    assert np.array_equal(t["absorbed"].cpu().numpy(), fresh["A"])
    assert t["stats"][0].escaped == fresh["escaped"]
