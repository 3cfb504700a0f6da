"""Shared helpers of the GPU parity tests (run the HIP path and the oracle on
the same seeded inputs, compare to the stated tolerances)."""
import numpy as np

# Tolerances of the FP32 GPU walk against the FP64 oracle:
#  per cell  |A_gpu - A_orc| <= 1e-3 A_orc + 1e-6 mean(A_orc)
#  global    |f_abs_gpu - f_abs_orc| <= 1e-5 f_abs_orc
CELL_REL, CELL_FLOOR, GLOBAL_REL = 1e-3, 1e-6, 1e-5


def gpu_run(spec, options=None, ranges=None, seeds=None, n_packets=None):
    import paper_2312_11448_amd as M
    cap = None if n_packets is None else max(1, sum(int(n) for n in n_packets))
    with M.Simulation(spec, max_packets=cap) as sim:
        for k, v in (options or {}).items():
            sim.set_option(k, v)
        sim.emit(seeds, n_packets)
        if ranges is None:
            sim.transport()
        else:
            for a, b in ranges:
                sim.transport(a, b - a)
        t = sim.tally()
        st = t["stats"][0]
        return dict(A=t["absorbed"].cpu().numpy(), emitted=t["emitted"].cpu().numpy(),
                    escaped=st.escaped, crossings=st.crossings, stats=st)


def compare_cells(gpu_A, orc_A, w_total):
    tol = CELL_REL * np.abs(orc_A) + CELL_FLOOR * max(orc_A.mean(), 1.0)
    diff = np.abs(gpu_A.astype(np.float64) - orc_A.astype(np.float64))
    bad = diff > tol
    f_g = gpu_A.sum() / w_total
    f_o = orc_A.sum() / w_total
    # a box that absorbs nothing (x_e = 1) compares its fractions exactly
    f_rel = abs(f_g - f_o) / f_o if f_o > 0 else (0.0 if f_g == f_o else float("inf"))
    return dict(bad=int(bad.sum()), worst=float((diff / np.maximum(tol, 1)).max()),
                f_gpu=f_g, f_orc=f_o, f_rel=f_rel)
