"""Training and evaluation of the mixing-correction surrogate.

The Monte Carlo (``Simulation``: emit, transport, targets) gives every cell
its mixing correction M_c = A_c / A_c^fm (Sec. IV.B, Eq. (dotne-mix)) as the
regression target y = ln M_c, with the cell's share of its box's emission as
its weight in the loss (the cells that feed recombination most count most);
the feature kernel gives its eight local features. The network (``Mlp``) is
trained on those cells, then gives M for new boxes without a transport; cells
whose features leave the training envelope take the Monte Carlo's M instead
(``predict``). Its error is judged against a high-statistics Monte-Carlo
reference of held-out boxes.

Every arithmetic step of the method runs in the HIP library; this module only
moves tensors between the calls (choosing cells and mini-batches,
concatenating boxes) and computes the reported error statistics.
"""
import time

import numpy as np
import torch

# packets per tiled-walk batch that a context reserves hand-over state for
# (234 bytes a packet): larger emissions walk in batches
BATCH = 1 << 28

from .sim import Simulation
from .mlp import Mlp


def mc_cells(specs, seeds=None, device="cuda", keep=None, pick_seed=0, sim=None):
    """Run the Monte Carlo on `specs` (one context) and return per-cell
    features [n, 8], target ln M [n], weight [n] and M itself, as device
    tensors, with the time of the transport. keep: if given, at most this
    many cells of each box, drawn uniformly (seeded) with their weights scaled
    by cells / kept, so that every box keeps its total weight. sim: an open
    Simulation of boxes of the same shapes and physics to load `specs`'
    fields into (no new context), else one is made for them."""
    specs = list(specs) if isinstance(specs, (list, tuple)) else [specs]
    n_all = max(1, sum(int(s.n_packets) for s in specs))
    if sim is None:
        with Simulation(specs, device=device, max_packets=n_all, batch_packets=min(n_all, BATCH)) as own:
            return _cells(own, seeds, keep, pick_seed)
    sim.load_fields(specs)
    return _cells(sim, seeds, keep, pick_seed)


def _cells(sim, seeds, keep, pick_seed):
    sim.emit(seeds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.transport()
    sim.tally(want_emitted=False)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t0
    y, w = sim.targets()
    M = sim.feed()["mix_corr"]
    feats = sim.features()
    off = sim.cell_off.copy()
    if keep is None:
        return dict(features=feats, y=y, w=w, M=M, t_mc=t_mc, cell_off=off)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(pick_seed))
    idx, scale = [], []
    for b in range(len(off) - 1):
        lo, hi = int(off[b]), int(off[b + 1])
        n = hi - lo
        if n <= keep:
            idx.append(torch.arange(lo, hi))
            scale.append(torch.ones(n))
        else:
            idx.append(lo + torch.randperm(n, generator=gen)[:keep])
            scale.append(torch.full((keep,), n / keep))
    idx = torch.cat(idx).to(feats.device)
    scale = torch.cat(scale).to(feats.device, torch.float32)
    return dict(features=feats[idx].contiguous(), y=y[idx].contiguous(), w=(w[idx] * scale).contiguous(),
                M=M[idx].contiguous(), t_mc=t_mc, cell_off=None)


def concat(parts):
    """One training set from several mc_cells results."""
    return dict(features=torch.cat([p["features"] for p in parts]), y=torch.cat([p["y"] for p in parts]),
                w=torch.cat([p["w"] for p in parts]), t_mc=sum(p["t_mc"] for p in parts))


def train(mlp, data, steps=3000, batch=65536, lr=3e-3, lr_final=3e-4, seed=0, log_every=0):
    """Adam on mini-batches drawn (seeded) from the cells with weight > 0;
    the learning rate decays geometrically from lr to lr_final."""
    idx_all = torch.nonzero(data["w"] > 0).squeeze(1)
    # batches drawn on the device (a seeded generator there): a host
    # generator draws 65 536 indices a step far slower than the device
    # trains on them
    gen = torch.Generator(device=idx_all.device)
    gen.manual_seed(int(seed))
    n = idx_all.numel()
    b = min(batch, n)
    chunk = max(1, min(steps, (1 << 24) // b))
    losses = []
    for s0 in range(0, steps, chunk):
        k = min(chunk, steps - s0)
        picks = torch.randint(0, n, (k, b), generator=gen, device=idx_all.device)
        rates = [lr * (lr_final / lr) ** (s / max(1, steps - 1)) for s in range(s0, s0 + k)]
        logged = [s for s in range(s0, s0 + k) if log_every and (s % log_every == 0 or s == steps - 1)]
        # the chunk's steps in one library call (gather, gradient, Adam per step)
        out = mlp.train_steps(data["features"], data["y"], data["w"], idx_all[picks], rates,
                              want_losses=bool(logged))
        losses.extend((s, out[s - s0]) for s in logged)
    return losses


def envelope(features, q=0.001):
    """Per-feature bounds of the training features (quantiles q and 1 - q,
    widened by 5 % of the range)."""
    f = features.float()
    sub = f[:: max(1, f.shape[0] // 1_000_000)]
    lo = torch.quantile(sub, q, dim=0)
    hi = torch.quantile(sub, 1 - q, dim=0)
    pad = 0.05 * (hi - lo)
    return (lo - pad).cpu().numpy().astype(np.float32), (hi + pad).cpu().numpy().astype(np.float32)


def predict(mlp, specs, fallback_packets_per_cell=64, fallback_seed=None, device="cuda"):
    """The surrogate's M for every cell of `specs` (one context), with the
    Monte Carlo as fallback: if any cell's features leave the training
    envelope, the boxes are transported (fallback_packets_per_cell packets
    per cell, in a context that reserves them only then) and those cells take
    the Monte Carlo's M. Returns dict(M, y, outside, n_outside, fallback_run,
    features)."""
    specs = list(specs) if isinstance(specs, (list, tuple)) else [specs]
    with Simulation(specs, device=device, max_packets=1) as sim:
        feats = sim.features()
    M, y, flags, n_out = mlp.correction(feats)
    ran = False
    if n_out:
        n_pk = [int(fallback_packets_per_cell * s.ncells) for s in specs]
        with Simulation(specs, device=device, max_packets=max(1, sum(n_pk)),
                        batch_packets=min(max(1, sum(n_pk)), BATCH)) as sim:
            sim.emit(seeds=fallback_seed, n_packets=n_pk)
            sim.transport()
            sim.tally(want_emitted=False)
            M_mc = sim.feed()["mix_corr"]
        M, y, flags, n_out = mlp.correction(feats, fallback=M_mc)
        ran = True
    return dict(M=M, y=y, outside=flags, n_outside=n_out, fallback_run=ran, features=feats)


def reference(specs, runs, packets_per_cell, seed0, device="cuda"):
    """High-statistics Monte-Carlo M of each box in `specs`: the mean of
    `runs` independent transports (packet seeds seed0 + r) of
    packets_per_cell packets per cell each, run box by box. Returns dict(M,
    features, w, cell_off) over all boxes (w: emission share, from the
    library's targets)."""
    Ms, fs, ws = [], [], []
    for s in specs:
        n_pk = int(packets_per_cell * s.ncells)
        with Simulation(s, device=device, max_packets=n_pk, batch_packets=min(n_pk, BATCH)) as sim:
            acc = torch.zeros(s.ncells, dtype=torch.float64, device=device)
            w = None
            for r in range(runs):
                sim.emit(seeds=[seed0 + r], n_packets=[n_pk])
                sim.transport()
                sim.tally(want_emitted=False)
                acc += sim.feed()["mix_corr"].to(torch.float64)
                if w is None:
                    _, w = sim.targets()
            Ms.append((acc / runs).to(torch.float32))
            fs.append(sim.features())
            ws.append(w)
    off = np.concatenate([[0], np.cumsum([s.ncells for s in specs])]).astype(np.int64)
    return dict(M=torch.cat(Ms), features=torch.cat(fs), w=torch.cat(ws), cell_off=off)


def _weighted_stats(err, w):
    w = w.to(torch.float64)
    err = err.to(torch.float64)
    keep = w > 0
    err, w = err[keep], w[keep]
    mean = float((w * err).sum() / w.sum())
    order = torch.argsort(err)
    cw = torch.cumsum(w[order], 0) / w.sum()
    p95 = float(err[order][torch.searchsorted(cw, torch.tensor(0.95, dtype=torch.float64, device=cw.device))
                           .clamp(max=err.numel() - 1)])
    return mean, p95


def evaluate(M_pred, ref, ref2):
    """Error statistics of the predicted M against the reference Monte Carlo
    `ref` (weighted by emission share), beside the reference's own noise
    (`ref2`: the same boxes with other packet seeds; the difference of two
    independent references, so about sqrt(2) times the noise of one) and two
    analytic comparators: full mixing (M = 1) and no mixing (every cell
    absorbs its own emission, M = emission share / n_1s share)."""
    M_ref = ref["M"].to(torch.float64)
    w = ref["w"]
    ok = M_ref > 0
    rel = lambda M: torch.where(ok, (M.to(torch.float64) - M_ref).abs() / torch.where(ok, M_ref, torch.ones_like(M_ref)),
                                torch.zeros_like(M_ref))
    delta = torch.exp(ref["features"][:, 0].to(torch.float64))
    n1s = delta * (1.0 - ref["features"][:, 5].to(torch.float64))
    M_nm = torch.zeros_like(M_ref)
    off = ref["cell_off"]
    for b in range(len(off) - 1):
        lo, hi = int(off[b]), int(off[b + 1])
        e = w[lo:hi].to(torch.float64)
        M_nm[lo:hi] = (e / e.sum()) / (n1s[lo:hi] / n1s[lo:hi].sum())
    out = {}
    for name, M in (("surrogate", M_pred), ("reference_noise", ref2["M"]),
                    ("full_mixing", torch.ones_like(M_ref)), ("no_mixing", M_nm)):
        m, p = _weighted_stats(rel(M), w)
        out[name] = {"weighted_mean_rel_err": m, "weighted_p95_rel_err": p}
    return out


def time_inference(mlp, sim, reps=5):
    """Seconds per features + inference pass over every cell of `sim`
    (device time, averaged over passes queued back to back, with events
    between the calls), with the time of the inference alone."""
    n = sim.total_cells
    y = None
    for _ in range(2):
        f = sim.features()
        y = mlp.forward(f)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps + 1)]
    e[0].record()
    for r in range(reps):
        f = sim.features()
        e[2 * r + 1].record()
        y = mlp.forward(f)
        e[2 * r + 2].record()
    torch.cuda.synchronize()
    tf = sum(e[2 * r].elapsed_time(e[2 * r + 1]) for r in range(reps)) / 1e3
    ti = sum(e[2 * r + 1].elapsed_time(e[2 * r + 2]) for r in range(reps)) / 1e3
    return (tf + ti) / reps, ti / reps, n, y


def forward_flops_per_cell():
    """Multiply-adds of the 8-64-64-1 network, counted as 2 flops each."""
    return 2 * (8 * 64 + 64 * 64 + 64)


def summary_line(stats):
    return ", ".join(f"{k}: mean {v['weighted_mean_rel_err']:.4f} p95 {v['weighted_p95_rel_err']:.4f}"
                     for k, v in stats.items())
