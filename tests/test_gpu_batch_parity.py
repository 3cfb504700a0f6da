"""The batch path against the FP64 oracle: one context over boxes of uneven
size (16^3 to 96^3), redshift (830 to 1390, the Monte-Carlo redshifts of
Fig. MCtravel), contrast and temperature T = T0 (1 + z), x_e = 0.1. The
transport splits the boxes between the tile-decomposed walk and the
persistent walk (asserted from the per-box stats) and runs eagerly (the
persistent part beside the tiles or after them) and as a replayed HIP graph,
with the default options and again after the autotuner; every box is
compared cell by cell with the oracle run of that box alone, at the stated
tolerances (per cell 1e-3 relative plus 1e-6 of the mean cell, absorbed
fraction 1e-5), and its emission counts bit for bit."""
import numpy as np
import pytest

import workloads as W
from oracle import walker
from tests.gpu_helpers import compare_cells, GLOBAL_REL

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402

T0 = W.CosmoParams().t_cmb0
# (edge, redshift, rms contrast, packets): a long-walking low-redshift box
# with many tiles, a crowded single-tile box at high redshift, and boxes in
# between
BOXES = [(96, 830.0, 0.4, 100_000), (64, 1000.0, 1.5, 400_000), (16, 1390.0, 1.8, 300_000),
         (40, 1200.0, 0.8, 100_000), (24, 900.0, 0.6, 50_000)]


def _specs():
    out = []
    for b, (n, z, rms, npk) in enumerate(BOXES):
        od, vel = W.grf_k2(n, rms, max(1, n // 4), 500 + b, vel_rms=0.1)
        out.append(W.BoxSpec(n=(n, n, n), overdensity=od, velocity=vel, z=z, temp_K=T0 * (1.0 + z),
                             n_packets=npk, seed=40 + b, name=f"{n}^3 z={z:g} rms={rms:g}"))
    return out


@pytest.fixture(scope="module")
def batch():
    specs = _specs()
    refs = []
    for s in specs:
        r = walker.run_box(s)
        print(f"  oracle {s.name}: {r['crossings']} crossings", flush=True)
        refs.append(r)
    return specs, refs


def _check(specs, refs, sim, t, label):
    A = t["absorbed"].cpu().numpy()
    em = t["emitted"].cpu().numpy()
    for i, (s, r) in enumerate(zip(specs, refs)):
        lo, hi = sim.cell_off[i], sim.cell_off[i + 1]
        st = t["stats"][i]
        assert st.conserved == 1 and st.capped_packets == 0
        assert np.array_equal(em[lo:hi], r["emitted"]), (label, s.name)
        cmp = compare_cells(A[lo:hi], r["A"], float(s.w0) * s.n_packets)
        print(f"  {label} {s.name} tiled={st.tiled}: {cmp}; crossings gpu {st.crossings} orc {r['crossings']}",
              flush=True)
        assert cmp["bad"] == 0, (label, s.name)
        assert cmp["f_rel"] <= GLOBAL_REL, (label, s.name)
        assert abs(st.crossings - r["crossings"]) <= 1e-4 * r["crossings"] + 10


def test_batch_graph_replay_matches_oracle(batch):
    specs, refs = batch
    with M.Simulation(specs) as sim:
        sim.set_option(M.MC_LYA_OPT_GRAPH, 1)
        kinds = None
        for rep in range(2):          # the first transport captures the graph, the second replays it
            sim.emit()
            sim.transport()
            t = sim.tally(want_emitted=True)
            _check(specs, refs, sim, t, f"graph run {rep}")
            kinds = [s.tiled for s in t["stats"]]
        # the batch took both walks: tiles for some boxes, the persistent walk for others
        assert 1 in kinds and 0 in kinds, kinds
        assert kinds[0] == 1 and kinds[2] == 0


@pytest.mark.parametrize("beside", [4, 0])
def test_batch_eager_matches_oracle(batch, beside):
    """The eager transport, with the persistent walk of the untiled boxes
    beside the tile generations on the context's second stream (and after
    them, beside = 0), and with the batch's tail switch at 20 % in flight."""
    specs, refs = batch
    with M.Simulation(specs) as sim:
        sim.set_option(M.MC_LYA_OPT_BESIDE, beside)
        sim.set_option(M.MC_LYA_OPT_TAIL, 200_000)
        sim.emit()
        sim.transport()
        t = sim.tally(want_emitted=True)
        _check(specs, refs, sim, t, f"eager beside={beside}")
        kinds = [s.tiled for s in t["stats"]]
        assert 1 in kinds and 0 in kinds, kinds


def test_batch_after_autotune_matches_oracle(batch):
    specs, refs = batch
    with M.Simulation(specs) as sim:
        sim.set_option(M.MC_LYA_OPT_GRAPH, 1)
        sim.emit()
        r = sim.autotune(1)
        print(f"  tuned: kernel {r.kernel} share {r.tile_share} tile chunk {r.tile_chunk} "
              f"refill {r.tile_refill}: {r.best_ms:.2f} ms (defaults {r.start_ms:.2f} ms)", flush=True)
        sim.transport()
        t = sim.tally(want_emitted=True)
        _check(specs, refs, sim, t, "tuned")
