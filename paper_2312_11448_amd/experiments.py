"""The paper's Monte-Carlo experiments of Sec. IV.A.3 on synthetic fields,
run through the library.

* ``escape_vs_flow``: the flow test of Fig. MCescape. A homogeneous medium at
  z = 1100 carries the bulk flow v_x = v0 sin(2 pi x / lambda); packets are
  emitted at x = 0, where div v is largest, and the fraction lost to
  redshifting, f_z, is recorded against div v / H there for several
  wavelengths lambda.
* ``global_loss``: the global loss-rate comparison of Sec. IV.A.3. The Monte
  Carlo's C (the emission-weighted integral of C alpha_e n_e^2 over
  the emission-weighted integral of alpha_e n_e^2) against the fully mixed
  C^mix, with and without the peculiar flow.
* ``travel_distances``: Fig. MCtravel. The comoving distance between a
  photon's creation and its destruction, from the resonant-scattering Monte
  Carlo (App. A), as f_alpha(D), the fraction that traveled further than D.

The streaming walk follows packets without scattering (the paper's
no-diffusion limit, Sec. IV.A.2), so in ``escape_vs_flow`` and
``global_loss`` a packet's fate is decided over the distance in which the
expansion sweeps it across the line core, about v_th / H (5 kpc comoving at
z = 1100), rather than over the paper's diffusion length. The flows that
average out are those shorter than that. ``travel_distances`` runs the
scattering Monte Carlo itself.

Run as ``python -m paper_2312_11448_amd.experiments escape|loss|travel``; each
prints one JSON line per measurement.
"""
import argparse
import dataclasses
import json
import math
import time

import numpy as np

from .sim import Simulation

KPC_CM = 3.0856775814913673e21           # cm per comoving kpc


def _stats(spec):
    """Emits and transports one box; returns its box statistics."""
    with Simulation(spec) as sim:
        sim.emit()
        sim.transport()
        return sim.tally()["stats"][0]


def drift_per_cell(spec):
    """The red drift per cell width (Doppler units) that the library computes
    for ``spec``'s cell size, redshift and temperature."""
    return _stats(dataclasses.replace(spec, velocity=None, n_packets=64)).delta


def cells_per_wavelength(lam_kpc, max_cell_pc=100.0, min_cells=16):
    """A power of two of at least ``min_cells`` cells per wavelength, with
    cells no larger than ``max_cell_pc``: the flow's cell-to-cell jumps stay
    far below a Doppler width."""
    n = int(min_cells)
    while lam_kpc * 1e3 / n > max_cell_pc:
        n *= 2
    return n


def escape_vs_flow(lams_kpc=(0.1, 1.0, 10.0, 1000.0), gs=(-0.8, -0.4, 0.0, 0.4, 0.8), n_packets=4_000_000,
                   seed=1, z=1100.0, temp_K=3000.0, echo=None):
    """f_z against div v / H at the emission point, per wavelength (kpc,
    comoving). div v / H = g sets the flow amplitude 2 pi U0 / N = g delta
    (U0 in v_th, N cells per wavelength, delta the drift per cell)."""
    import workloads as W
    rows = []
    for lam in lams_kpc:
        n = cells_per_wavelength(lam)
        cell = lam * KPC_CM / n
        delta = drift_per_cell(W.escape_slab(n, 0.0, cell, 64, seed=seed, z=z, temp_K=temp_K))
        for g in gs:
            u0 = g * n * delta / (2.0 * math.pi)
            spec = W.escape_slab(n, u0, cell, n_packets, seed=seed, z=z, temp_K=temp_K)
            t0 = time.perf_counter()
            st = _stats(spec)
            row = dict(experiment="escape_vs_flow", lam_kpc=lam, cells=n, cell_pc=cell / KPC_CM * 1e3,
                       delta=delta, amplitude_vth=u0, div_v_over_H=g, f_z=st.escaped / st.emitted,
                       tau_ab=st.tau_ab_mean, packets=n_packets, crossings=st.crossings,
                       seconds=time.perf_counter() - t0)
            rows.append(row)
            if echo:
                echo(row)
    return rows


def global_loss(spec, echo=None):
    """C_MC / C^mix of one box with its flow and with the flow removed."""
    rows = []
    for name, s in (("flow", spec), ("no_flow", dataclasses.replace(spec, velocity=None))):
        if name == "flow" and spec.velocity is None:
            continue
        t0 = time.perf_counter()
        with Simulation(s) as sim:
            sim.emit()
            sim.transport()
            sim.tally()
            f = sim.feed()["stats"][0]
        row = dict(experiment="global_loss", case=name, workload=spec.name, c_mc=f.c_mc, c_mix=f.c_mix,
                   loss_ratio=f.c_mc / f.c_mix, f_escape=f.f_escape, packets=s.n_packets,
                   seconds=time.perf_counter() - t0)
        rows.append(row)
        if echo:
            echo(row)
    return rows


def travel_box(z, x_e, n_photons, seed=1, cell_kpc=1.0, n=4):
    """The medium of Fig. MCtravel: homogeneous hydrogen at the mean density,
    at rest in the Hubble flow, at redshift z with matter and radiation at
    T = T_cmb0 (1 + z), free-electron fraction x_e, the Voigt profile and the
    physical expansion rate (zeta = 1). The periodic box is n cells of
    ``cell_kpc`` comoving on a side; the displacements are unwrapped."""
    import workloads as W
    t_cmb0 = W.CosmoParams().t_cmb0
    return W.BoxSpec(n=(n, n, n), overdensity=W.uniform_box(n), x_e_uniform=float(x_e), z=float(z),
                     temp_K=t_cmb0 * (1.0 + z), profile="voigt", zeta=1.0, cell_cm=cell_kpc * KPC_CM,
                     n_packets=int(n_photons), seed=int(seed),
                     name=f"homogeneous, z={z:g}, x_e={x_e:.4g}, Voigt, zeta=1, {n}^3 cells of {cell_kpc:g} kpc")


def travel_distances(spec):
    """Scatters every photon of ``spec`` (App. A) and returns the comoving
    distance in kpc from creation to destruction of the destroyed ones, the
    records, and the wall time."""
    t0 = time.perf_counter()
    with Simulation(spec) as sim:
        sim.emit()
        rec = sim.scatter(records=True)
    dt = time.perf_counter() - t0
    d = np.sqrt(rec["dx"].astype(np.float64) ** 2 + rec["dy"].astype(np.float64) ** 2 +
                rec["dz"].astype(np.float64) ** 2) * (spec.cell_cm / KPC_CM)
    return d[rec["fate"] == 0], rec, dt


def fraction_beyond(dist_kpc, D_kpc):
    """f_alpha(D): the fraction of the distances larger than each D."""
    dist_kpc = np.sort(np.asarray(dist_kpc, dtype=np.float64))
    D = np.atleast_1d(np.asarray(D_kpc, dtype=np.float64))
    return 1.0 - np.searchsorted(dist_kpc, D, side="right") / max(1, dist_kpc.size)


def diffusion_beyond(dist_kpc, D_kpc):
    """The same fraction for diffusion with the same mean square distance:
    a 3-D Gaussian of per-axis variance s^2 = <d^2> / 3, whose distance
    exceeds D with probability erfc(q / sqrt 2) + sqrt(2 / pi) q exp(-q^2 / 2),
    q = D / s (the dotted line of Fig. MCtravel)."""
    s = math.sqrt(float(np.mean(np.square(dist_kpc))) / 3.0)
    q = np.atleast_1d(np.asarray(D_kpc, dtype=np.float64)) / s
    return np.array([math.erfc(v / math.sqrt(2.0)) for v in q]) + math.sqrt(2.0 / math.pi) * q * np.exp(-0.5 * q * q)


def travel_row(spec, D_kpc=(0.1, 0.3, 1.0, 3.0, 10.0)):
    """One redshift of Fig. MCtravel: f_alpha(D) and its diffusive
    counterpart, with the photons' fates and the run's cost."""
    d, rec, dt = travel_distances(spec)
    events = rec["scatterings"].astype(np.float64) + rec["crossings"]
    return dict(experiment="travel_distances", z=spec.z, x_e=spec.x_e_uniform, photons=int(rec.size),
                destroyed=int(d.size), lost_to_line=int(np.sum(rec["fate"] == 1)),
                capped=int(np.sum(rec["fate"] == 2)), D_kpc=list(D_kpc),
                f_alpha=fraction_beyond(d, D_kpc).tolist(), f_diffusion=diffusion_beyond(d, D_kpc).tolist(),
                rms_kpc=float(np.sqrt(np.mean(d * d))), median_kpc=float(np.median(d)),
                mean_scatterings=float(rec["scatterings"].mean()), max_events=int(events.max()),
                seconds=dt, scatterings_per_s=float(rec["scatterings"].sum()) / dt)


def _echo(row):
    print(json.dumps(row), flush=True)


def main(argv=None):
    import workloads as W
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("experiment", choices=["escape", "loss", "travel"])
    ap.add_argument("--packets", type=float, default=4e6, help="packets (escape, loss) or photons (travel)")
    ap.add_argument("--z", type=float, nargs="*", default=[1400.0, 1300.0, 1200.0],
                    help="travel: redshifts")
    ap.add_argument("--xe", type=float, nargs="*", default=None,
                    help="travel: x_e at each redshift (the caller's recombination history)")
    a = ap.parse_args(argv)
    if a.experiment == "escape":
        escape_vs_flow(n_packets=int(a.packets), echo=_echo)
    elif a.experiment == "loss":
        for key, n in (("c2", 128), ("c3", 128)):
            global_loss(W.make_box(key, n=n, n_packets=int(a.packets)), echo=_echo)
    else:
        if a.xe is None or len(a.xe) != len(a.z):
            raise SystemExit("travel needs one --xe value per --z value")
        for z, xe in zip(a.z, a.xe):
            _echo(travel_row(travel_box(z, xe, int(a.packets))))


if __name__ == "__main__":
    main()
