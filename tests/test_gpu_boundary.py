"""The boundary's memory contract: a context allocates its device memory in
mc_lya_init (sized by the boxes and mc_lya_limits) and no later call
allocates. Every call of the path, and the other entry points that work on a
context (trace, features, scattering Monte Carlo, recombination history), runs
through the C ABI on caller-allocated buffers while the device's free memory
is watched; a first context warms the HIP runtime's own pools."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402


def _spec():
    spec = W.make_box("c2", n=24, n_packets=20_000, field_seed=31, seed=3)
    spec.x_e = np.full(spec.overdensity.shape, 0.1, dtype=np.float32)
    return spec


def _every_call(sim, bufs, check):
    """emit -> transport -> tally -> feed -> trace -> features -> scattering
    -> evolve, calling check(name) after each."""
    L = M.load()
    n = sim.total_cells
    M.mc_lya_emit(sim.ctx, [3], [20_000])
    check("emit")
    M.mc_lya_transport(sim.ctx)
    check("transport")
    M.mc_lya_tally(sim.ctx, bufs["A"].data_ptr(), bufs["E"].data_ptr(), 1)
    check("tally")
    M.mc_lya_feed(sim.ctx, bufs["nd"].data_ptr(), bufs["mix"].data_ptr(), 1)
    check("feed")
    M.mc_lya_trace(sim.ctx, 0, 1000, bufs["trace"].data_ptr())
    check("trace")
    M.mc_lya_features(sim.ctx, bufs["feat"].data_ptr())
    check("features")
    o = M.mc_lya_scatter_opts(x_inert=0.0, p_destroy=0.05, max_events=0, fixed_x0=0, x0=0.0, x_return=0.0)
    M.mc_lya_scatter(sim.ctx, 0, 2000, o, bufs["srec"].data_ptr())
    check("scatter")
    X = (C.c_double * 2)()
    ptrs = (C.c_void_p * 1)(sim._descs[0].x_e)
    npk = (C.c_uint64 * 1)(20_000)
    st = L.mc_lya_evolve(sim.ctx, 1300.0, 1299.0, 1, npk, 7, ptrs, X)
    assert st == M.MC_LYA_OK, M.mc_lya_last_error(sim.ctx)
    check("evolve")
    assert n == sim.total_cells


def test_no_device_allocation_after_init():
    spec = _spec()
    n = spec.ncells
    dev = torch.device("cuda")
    bufs = dict(A=torch.empty(n, dtype=torch.int64, device=dev), E=torch.empty(n, dtype=torch.int64, device=dev),
                nd=torch.empty(n, dtype=torch.float64, device=dev), mix=torch.empty(n, dtype=torch.float32, device=dev),
                trace=torch.empty(1000 * 64, dtype=torch.uint8, device=dev),
                feat=torch.empty((n, 8), dtype=torch.float32, device=dev),
                srec=torch.empty(2000 * 72, dtype=torch.uint8, device=dev))
    # a first context warms the runtime (code object, kernel-argument pools)
    with M.Simulation(spec, evolve=True) as warm:
        _every_call(warm, bufs, lambda name: None)
    torch.cuda.synchronize()
    with M.Simulation(spec, evolve=True) as sim:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        seen = []

        def check(name):
            torch.cuda.synchronize()
            free = torch.cuda.mem_get_info()[0]
            seen.append((name, free0 - free))
            assert free == free0, (name, free0 - free)

        _every_call(sim, bufs, check)
    print(f"  device memory taken after init: {seen}", flush=True)


def test_read_probe_checks_its_arguments_and_runs():
    """The read-bandwidth probe (a measurement utility): bad sizes are
    rejected; a valid call reads and leaves the sink alone (finite data)."""
    buf = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    M.mc_lya_probe_read(buf.data_ptr(), buf.numel() * 4, 3, 64, sink.data_ptr())
    torch.cuda.synchronize()
    assert sink.item() == 0.0
    for nbytes, passes, grid in ((12, 1, 1), (buf.numel() * 4, 0, 1), (buf.numel() * 4, 1, 0)):
        with pytest.raises(M.MCLyaError):
            M.mc_lya_probe_read(buf.data_ptr(), nbytes, passes, grid, sink.data_ptr())
