"""Seeded inputs of the mixing-correction surrogate: the network's initial
parameters and the boxes it is trained and evaluated on.

The boxes follow the 128^3 / 256^3 field family (k^2 Gaussian field with its
curl-free flow) over the redshift and contrast range of the batch workload;
the evaluation boxes use field seeds the training never sees.
"""
import numpy as np

from . import fields as F
from .configs import BoxSpec, CosmoParams

N_PARAMS = 4801
FAN_IN = ((0, 512, 8), (576, 4672, 64), (4736, 4800, 64))    # weight blocks: (start, end, fan-in)


def initial_params(seed):
    """Weights uniform in +-1/sqrt(fan_in), biases zero (float32)."""
    u = np.random.Generator(np.random.Philox(int(seed))).random(N_PARAMS)
    p = np.zeros(N_PARAMS)
    for a, b, fan in FAN_IN:
        p[a:b] = (2.0 * u[a:b] - 1.0) / np.sqrt(fan)
    return p.astype(np.float32)


def surrogate_box(n, rms, z, field_seed, packets, seed):
    od, vel = F.grf_k2(n, rms, max(1, n // 4), field_seed, vel_rms=0.1)
    t0 = CosmoParams().t_cmb0
    return BoxSpec(n=(n, n, n), overdensity=od, velocity=vel, z=float(z), temp_K=t0 * (1.0 + z),
                   n_packets=int(packets), seed=int(seed),
                   name=f"{n}^3 rms {rms:.2f} z {z:.0f} field seed {field_seed}")


def training_specs(n_boxes=24, n=64, packets_per_cell=128, seed=5000):
    """Training boxes: contrast rms ~ U[0.2, 2], z ~ U[800, 1400]."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    for b in range(n_boxes):
        rms = float(rng.uniform(0.2, 2.0))
        z = float(rng.uniform(800.0, 1400.0))
        out.append(surrogate_box(n, rms, z, seed + 1 + b, packets_per_cell * n ** 3, 100 + b))
    return out


def evaluation_specs(n=128, packets_per_cell=256, seed=9000):
    """Held-out boxes (field seeds outside the training range) at three
    redshifts and contrasts."""
    cases = ((0.5, 1100.0), (1.5, 1000.0), (1.0, 1300.0))
    return [surrogate_box(n, rms, z, seed + i, packets_per_cell * n ** 3, 200 + i)
            for i, (rms, z) in enumerate(cases)]
