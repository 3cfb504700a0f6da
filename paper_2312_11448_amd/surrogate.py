"""Training and evaluation of the mixing-correction surrogate.

The Monte Carlo (``Simulation``: emit, transport, feed) gives every cell its
mixing correction M_c = A_c / A_c^fm (Sec. IV.B, Eq. (dotne-mix)); the
feature kernel gives its eight local features. The network (``Mlp``) is
trained on y = ln M_c with weights proportional to each cell's emission (the
cells that feed recombination most count most), then evaluated on held-out
boxes against a high-statistics Monte-Carlo reference.

Every arithmetic step of the method runs in the HIP library; this module only
moves tensors between the calls (sampling mini-batches, concatenating boxes)
and computes the reported error statistics.
"""
import time

import numpy as np
import torch

from .sim import Simulation
from .mlp import Mlp


def mc_cells(specs, seeds=None, device="cuda"):
    """Run the Monte Carlo on `specs` (one context) and return per-cell
    features [n, 8], target ln M [n], weight [n] (emission share of the cell in
    its box, 0 where M = 0) and M itself, as device tensors, plus the time of
    the transport."""
    with Simulation(specs, device=device) as sim:
        sim.emit(seeds)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.transport()
        tal = sim.tally(want_emitted=True)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t0
        fd = sim.feed()
        feats = sim.features()
        mix = fd["mix_corr"]
        em = tal["emitted"].to(torch.float64)
        w = torch.zeros_like(em)
        for b in range(len(specs)):
            lo, hi = int(sim.cell_off[b]), int(sim.cell_off[b + 1])
            s = em[lo:hi].sum()
            if s > 0:
                w[lo:hi] = em[lo:hi] / s
        ok = mix > 0
        y = torch.where(ok, torch.log(torch.where(ok, mix, torch.ones_like(mix))), torch.zeros_like(mix))
        w = torch.where(ok, w, torch.zeros_like(w)).to(torch.float32)
        torch.cuda.synchronize()
        return dict(features=feats, y=y.to(torch.float32), w=w, M=mix, emitted=em, t_mc=t_mc,
                    stats=fd["stats"], cell_off=sim.cell_off.copy())


def train(mlp, data, steps=3000, batch=65536, lr=3e-3, lr_final=3e-4, seed=0, log_every=0):
    """Adam on mini-batches drawn (seeded) from the cells with weight > 0;
    the learning rate decays geometrically from lr to lr_final."""
    idx_all = torch.nonzero(data["w"] > 0).squeeze(1)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(seed))
    n = idx_all.numel()
    losses = []
    for s in range(steps):
        pick = torch.randint(0, n, (min(batch, n),), generator=gen).to(idx_all.device)
        idx = idx_all[pick]
        X = data["features"][idx].contiguous()
        t = data["y"][idx].contiguous()
        w = data["w"][idx].contiguous()
        rate = lr * (lr_final / lr) ** (s / max(1, steps - 1))
        want = log_every and (s % log_every == 0 or s == steps - 1)
        loss = mlp.train_step(X, t, w, rate, want_loss=bool(want))
        if want:
            losses.append((s, loss))
    return losses


def envelope(features, q=0.001):
    """Per-feature bounds of the training features (quantiles q and 1 - q,
    widened by 5 % of the range)."""
    f = features.float()
    lo = torch.quantile(f[:: max(1, f.shape[0] // 1_000_000)], q, dim=0)
    hi = torch.quantile(f[:: max(1, f.shape[0] // 1_000_000)], 1 - q, dim=0)
    pad = 0.05 * (hi - lo)
    return (lo - pad).cpu().numpy().astype(np.float32), (hi + pad).cpu().numpy().astype(np.float32)


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


def evaluate(mlp, ref, ref2):
    """Error statistics of the surrogate's M against the reference Monte
    Carlo `ref` (weighted by emission), beside the reference's own noise
    (`ref2`: the same boxes with other packet seeds) and two analytic
    comparators: full mixing (M = 1) and no mixing (every cell absorbs its own
    emission, M = emission share / n_1s share)."""
    y = mlp.forward(ref["features"])
    M_pred = torch.exp(y.to(torch.float64))
    M_ref = ref["M"].to(torch.float64)
    w = ref["w"]
    ok = M_ref > 0
    rel = lambda M: torch.where(ok, (M - M_ref).abs() / torch.where(ok, M_ref, torch.ones_like(M_ref)),
                                torch.zeros_like(M_ref))
    delta = torch.exp(ref["features"][:, 0].to(torch.float64))
    n1s = delta * (1.0 - ref["features"][:, 5].to(torch.float64))
    M_nm = torch.zeros_like(M_ref)
    off = ref["cell_off"]
    for b in range(len(off) - 1):
        lo, hi = int(off[b]), int(off[b + 1])
        e = ref["emitted"][lo:hi]
        M_nm[lo:hi] = (e / e.sum()) / (n1s[lo:hi] / n1s[lo:hi].sum())
    out = {}
    for name, M in (("surrogate", M_pred), ("reference_noise", ref2["M"].to(torch.float64)),
                    ("full_mixing", torch.ones_like(M_ref)), ("no_mixing", M_nm)):
        m, p = _weighted_stats(rel(M), w)
        out[name] = {"weighted_mean_rel_err": m, "weighted_p95_rel_err": p}
    return out


def time_inference(mlp, sim, reps=5):
    """Seconds per features + inference pass over every cell of `sim`
    (device time, averaged), with the time of the inference alone."""
    n = sim.total_cells
    y = None
    for _ in range(2):
        f = sim.features()
        y = mlp.forward(f)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf = ti = 0.0
    for _ in range(reps):
        e[0].record()
        f = sim.features()
        e[1].record()
        y = mlp.forward(f)
        e[2].record()
        torch.cuda.synchronize()
        tf += e[0].elapsed_time(e[1]) / 1e3
        ti += e[1].elapsed_time(e[2]) / 1e3
    return (tf + ti) / reps, ti / reps, n, y


def forward_flops_per_cell():
    """Multiply-adds of the 8-64-64-1 network, counted as 2 flops each."""
    return 2 * (8 * 64 + 64 * 64 + 64)


def summary_line(stats):
    return ", ".join(f"{k}: mean {v['weighted_mean_rel_err']:.4f} p95 {v['weighted_p95_rel_err']:.4f}"
                     for k, v in stats.items())
