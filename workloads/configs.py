"""Named workload presets.

Five presets: a 32^3 lognormal box (the small case), a 128^3 k^2 field with a
curl-free flow (the benchmark workload), a 256^3 high-contrast field, a batch of
64 uneven boxes and the surrogate's training/evaluation set. The cosmology is
the one the paper fixes for all its runs (Sec. II.C); the comoving cell edge is
the paper's 24 kpc / 256 resolution, kept fixed so that the box edge is N cells
of 93.75 pc.
"""
from dataclasses import dataclass, field, replace
from typing import Optional
import numpy as np

from . import fields as F

KPC_CM = 3.0856775814913673e21
DEFAULT_CELL_CM = 24.0 * KPC_CM / 256.0


@dataclass(frozen=True)
class CosmoParams:
    h: float = 0.67
    omega_b_h2: float = 0.0224
    omega_c_h2: float = 0.12
    y_p: float = 0.24
    t_cmb0: float = 2.7255
    n_eff: float = 3.046


@dataclass
class BoxSpec:
    """One periodic box: geometry, physics and the field arrays (host numpy)."""
    n: tuple                       # (nx, ny, nz)
    overdensity: np.ndarray        # float32 [nz, ny, nx]
    velocity: Optional[np.ndarray] = None   # float32/float16 [3, nz, ny, nx], units of v_th
    x_e: Optional[np.ndarray] = None        # float32 [nz, ny, nx] or None
    x_e_uniform: float = 0.1
    source: Optional[np.ndarray] = None     # float32 [nz, ny, nx] or None
    temp_K: float = 3000.0
    profile: str = "doppler"               # line profile: "doppler" or "voigt" (damping wing)
    z: float = 1100.0
    zeta: float = 1.0
    x_esc: float = 6.0
    cell_cm: float = DEFAULT_CELL_CM
    w0: int = 1 << 31
    cosmo: CosmoParams = field(default_factory=CosmoParams)
    n_packets: int = 0
    seed: int = 1
    name: str = ""

    @property
    def ncells(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


CONFIGS = {
    "c1": dict(name="32^3 lognormal(ln-sigma 0.3), T=3000K, x_e=0.1, z=1100, 1e5 packets",
               n=32, field="lognormal", ln_sigma=0.3, field_seed=1,
               n_packets=100_000, seed=1),
    "c2": dict(name="128^3 k^2 GRF (kmax 32, rms 0.5) + curl-free flow (rms 0.1 v_th), "
                    "T=3000K, x_e=0.1, z=1100, 1e7 packets",
               n=128, field="grf", rms=0.5, kmax=32, vel_rms=0.1, field_seed=2,
               n_packets=10_000_000, seed=2),
    "c3": dict(name="256^3 k^2 GRF (kmax 64, rms 2, clip 1e-2..1e2) + curl-free flow, "
                    "T=3000K, x_e=0.1, z=1100, 2^28 packets",
               n=256, field="grf", rms=2.0, kmax=64, vel_rms=0.1, field_seed=3,
               n_packets=1 << 28, seed=3),
}


def make_box(key, n=None, n_packets=None, field_seed=None, seed=None, device=None, **overrides):
    """Build the BoxSpec for preset ``key`` ("c1", "c2", "c3"), optionally resized
    (device: a torch GPU device for the k^2 field's FFTs)."""
    cfg = dict(CONFIGS[key])
    n = int(n or cfg["n"])
    fs = cfg["field_seed"] if field_seed is None else field_seed
    if cfg["field"] == "lognormal":
        od = F.lognormal_white(n, cfg["ln_sigma"], fs)
        vel = None
    else:
        kmax = max(1, int(round(cfg["kmax"] * n / cfg["n"])))
        od, vel = F.grf_k2(n, cfg["rms"], kmax, fs, vel_rms=cfg["vel_rms"], device=device)
    box = BoxSpec(n=(n, n, n), overdensity=od, velocity=vel,
                  n_packets=int(n_packets if n_packets is not None else cfg["n_packets"]),
                  seed=int(cfg["seed"] if seed is None else seed), name=cfg["name"])
    return replace(box, **overrides) if overrides else box


def batch_specs(n_boxes=64, packets_each=1_000_000, seed=1000, nmin=16, nmax=96):
    """The batched workload: boxes of uneven size, redshift and contrast.

    Edges N ~ U{nmin..nmax}, redshift z ~ U[800, 1400], contrast rms ~ U[0.2, 2],
    field seed 1000+b, packet seed b, gas temperature equal to the radiation
    temperature T0 (1+z), x_e = 0.1.
    """
    rng = np.random.Generator(np.random.Philox(seed))
    boxes = []
    t0 = CosmoParams().t_cmb0
    for b in range(n_boxes):
        n = int(rng.integers(nmin, nmax + 1))
        z = float(rng.uniform(800.0, 1400.0))
        rms = float(rng.uniform(0.2, 2.0))
        od, vel = F.grf_k2(n, rms, max(1, n // 4), seed + b, vel_rms=0.1)
        boxes.append(BoxSpec(n=(n, n, n), overdensity=od, velocity=vel, z=z,
                             temp_K=t0 * (1.0 + z), n_packets=packets_each, seed=b,
                             name=f"batch box {b}: {n}^3 z={z:.0f} rms={rms:.2f}"))
    return boxes


def escape_slab(wavelength_cells, amplitude, cell_cm, n_packets, seed=1, ny=1, nz=1, **overrides):
    """The flow test of Fig. MCescape on the grid: a homogeneous box one
    wavelength long in x with the bulk flow U_x = amplitude sin(2 pi x / L)
    (v_th units, cell-centred), packets emitted only in the two cells that
    meet at x = 0, where the flow's gradient is largest: 2 pi amplitude / L
    per cell. ``ny`` x ``nz`` cells across (the medium is uniform across, so
    1 x 1 suffices)."""
    nx = int(wavelength_cells)
    od = np.ones((nz, ny, nx), dtype=np.float32)
    vel = np.zeros((3, nz, ny, nx), dtype=np.float32)
    vel[0] = F.sinusoidal_profile(nx, amplitude)[None, None, :]
    src = np.zeros((nz, ny, nx), dtype=np.float32)
    src[:, :, 0] = 1.0
    src[:, :, nx - 1] = 1.0
    box = BoxSpec(n=(nx, ny, nz), overdensity=od, velocity=vel, source=src, cell_cm=float(cell_cm),
                  n_packets=int(n_packets), seed=int(seed),
                  name=f"escape slab: {nx} cells of {cell_cm / KPC_CM * 1e3:.4g} pc, flow amplitude "
                       f"{amplitude:.4g} v_th")
    return replace(box, **overrides) if overrides else box
