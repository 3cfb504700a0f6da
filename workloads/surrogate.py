"""Seeded inputs of the mixing-correction surrogate: the network's initial
parameters and the boxes it is trained and evaluated on.

The stated set trains on 200 field seeds of the three single-box workloads
(the 32^3 lognormal box, the 128^3 k^2 field of rms 0.5 and the 256^3 k^2
field of rms 2, all with their flows and the physics of z = 1100, T = 3000 K,
x_e = 0.1) and evaluates on held-out 256^3 seeds. Field seeds of the
training boxes start at 10001 (32^3), 20001 (128^3) and 30001 (256^3); the
held-out boxes use 39001 and on, which no training box uses.

`small_training_specs` / `small_evaluation_specs` are the same families on
32^3 and 64^3 grids (the k^2 field keeps k_max = N/4, so its cell-scale
statistics do not depend on N), sized for a GPU test.
"""
import numpy as np

from .configs import make_box

N_PARAMS = 4801
FAN_IN = ((0, 512, 8), (576, 4672, 64), (4736, 4800, 64))    # weight blocks: (start, end, fan-in)
HELD_OUT_SEED = 39001


def initial_params(seed):
    """Weights uniform in +-1/sqrt(fan_in), biases zero (float32)."""
    u = np.random.Generator(np.random.Philox(int(seed))).random(N_PARAMS)
    p = np.zeros(N_PARAMS)
    for a, b, fan in FAN_IN:
        p[a:b] = (2.0 * u[a:b] - 1.0) / np.sqrt(fan)
    return p.astype(np.float32)


def family_box(key, field_seed, packets_per_cell, seed, n=None, device=None):
    """A box of workload family `key` ("c1", "c2", "c3") with its own field
    seed and packet count (packets_per_cell per cell on average); device: a
    torch GPU device for the k^2 field's FFTs."""
    box = make_box(key, n=n, field_seed=int(field_seed), seed=int(seed), device=device)
    box.n_packets = int(packets_per_cell * box.ncells)
    box.name = f"{key} family {box.n[0]}^3, field seed {field_seed}"
    return box


# the stated training set: (family, boxes, first field seed, packets per cell)
TRAINING = (("c1", 100, 10001, 512), ("c2", 70, 20001, 128), ("c3", 30, 30001, 64))


def training_boxes():
    """The 200 training boxes as (family, field seed, packets per cell, packet
    seed) tuples; `family_box` builds each (the 256^3 fields take seconds
    apiece, so they are built one at a time)."""
    out = []
    for key, count, first, ppc in TRAINING:
        for i in range(count):
            out.append((key, first + i, ppc, 100 + len(out)))
    return out


def evaluation_boxes(n_boxes=3):
    """Held-out 256^3 boxes of the rms-2 family, as (family, field seed,
    packet seed) tuples."""
    return [("c3", HELD_OUT_SEED + i, 7000 + i) for i in range(n_boxes)]


def small_training_specs():
    """40 boxes for a GPU test: 24 of the 32^3 lognormal family, 8 each of the
    rms-0.5 and rms-2 k^2 families on 64^3 grids."""
    out = [family_box("c1", 11001 + i, 512, 300 + i) for i in range(24)]
    out += [family_box("c2", 21001 + i, 128, 330 + i, n=64) for i in range(8)]
    out += [family_box("c3", 31001 + i, 128, 340 + i, n=64) for i in range(8)]
    return out


def small_evaluation_specs(packets_per_cell=512):
    """Held-out 64^3 boxes for a GPU test: two of the rms-2 family and one of
    the rms-0.5 family."""
    return [family_box("c3", HELD_OUT_SEED + 100, packets_per_cell, 7100, n=64),
            family_box("c3", HELD_OUT_SEED + 101, packets_per_cell, 7101, n=64),
            family_box("c2", HELD_OUT_SEED + 102, packets_per_cell, 7102, n=64)]
