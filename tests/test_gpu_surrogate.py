"""GPU parity of the mixing-correction surrogate (through the C ABI) against
the FP64 oracle: features, BF16 matrix-core inference, FP32 gradient and
Adam, the envelope flags.

Tolerances (derived from the arithmetic):
* features: FP32 sums of at most 27 terms, |error| <= 27 * 2^-24 * sum|terms|
  per sum; tested as 1e-5 of each feature's natural scale;
* inference rounds W1, W2, the features and the layer-1 activations to BF16
  (relative error <= 2^-9 each); first-order propagation through ReLU
  (|relu'| <= 1; 1.1 is used) gives, per cell,
    |dy| <= 1.1 sum_m |w3_m| (sum_k |W2_mk| (1.1 e_k + 2^-8 |h1_k|)),
    e_k = 2^-8 sum_j |W1_kj| |x_j|,
  and the test allows 1.5 times that plus 1e-5 against the FP64 network;
  against the oracle's BF16 network (the same roundings) what is left is FP32
  accumulation (~1e-6 of the scale) and, rarely, an activation that FP32 and
  FP64 round to neighbouring BF16 values;
* gradient: the straight-through gradient of the BF16 network. The kernel
  also rounds the error signals dL/dz2, dL/dz1 and the product w3 W2 to BF16
  for the matrix cores, at most four roundings of 2^-8 relative in any
  product, so each entry is checked against 2^-5 times the same chain rule
  taken with absolute values (plus 1e-6 of the largest entry, for the FP32
  sums); loss to 1e-4 relative.
"""
import numpy as np
import pytest

import workloads as W
from workloads import surrogate as WS
from oracle import surrogate as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402
from paper_2312_11448_amd import _abi as A  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _box_features_oracle(spec):
    return S.features(spec.overdensity, spec.velocity, np.float32(spec.x_e_uniform), spec.temp_K, spec.z)


@pytest.mark.parametrize("shape,vel", [((24, 24, 24), True), ((9, 13, 7), True), ((16, 8, 5), False),
                                       ((11, 6, 10), "f16"), ((1, 1, 3), True), ((300, 2, 3), "f16")])
def test_features_match_oracle(shape, vel):
    rng = np.random.default_rng(sum(shape))
    od = rng.lognormal(0.0, 0.7, size=shape[::-1]).astype(np.float32)
    v = rng.normal(0.0, 0.2, size=(3,) + shape[::-1]).astype(np.float16 if vel == "f16" else np.float32) \
        if vel else None
    spec = W.BoxSpec(n=shape, overdensity=od, velocity=v, z=950.0, temp_K=2.7255 * 951, n_packets=1)
    with M.Simulation(spec) as sim:
        f = sim.features().cpu().numpy().astype(np.float64)
    ref = _box_features_oracle(spec)
    scale = np.array([1.0, ref[:, 1].max(), ref[:, 1].max() ** 2, 0.2 if vel else 1.0, 1.0, 1.0, 1.0, 1.0])
    err = np.abs(f - ref) / scale
    _say(f"  worst feature error / scale: {err.max(axis=0)}")
    assert err.max() <= 1e-5


@pytest.mark.parametrize("shape", [(13, 5, 9), (12, 5, 9), (4, 1, 1)])
def test_features_with_a_per_cell_electron_fraction(shape):
    rng = np.random.default_rng(8)
    od = rng.lognormal(0.0, 0.5, size=shape[::-1]).astype(np.float32)
    xe = rng.uniform(0.0, 1.2, size=shape[::-1]).astype(np.float32)
    v = rng.normal(0.0, 0.2, size=(3,) + shape[::-1]).astype(np.float32)
    spec = W.BoxSpec(n=shape, overdensity=od, velocity=v, x_e=xe, z=1000.0, temp_K=2.7255 * 1001, n_packets=1)
    with M.Simulation(spec) as sim:
        f = sim.features().cpu().numpy().astype(np.float64)
    ref = S.features(spec.overdensity, spec.velocity, spec.x_e, spec.temp_K, spec.z)
    assert np.array_equal(f[:, 5], ref[:, 5])            # x_e itself, unchanged
    assert np.abs(f - ref).max() <= 1e-5 * max(1.0, ref[:, 1].max() ** 2)


def test_features_follow_new_fields_after_a_refresh():
    """The per-box table (pointers, box clumping) is uploaded once per
    refresh: features taken twice agree bit for bit, and after new field
    contents are loaded they are those of the new fields."""
    shape = (16, 12, 8)
    rng = np.random.default_rng(21)
    specs = []
    for sig in (0.4, 1.1):
        od = rng.lognormal(0.0, sig, size=shape[::-1]).astype(np.float32)
        v = rng.normal(0.0, 0.2, size=(3,) + shape[::-1]).astype(np.float32)
        specs.append(W.BoxSpec(n=shape, overdensity=od, velocity=v, z=1000.0, temp_K=2.7255 * 1001, n_packets=1))
    with M.Simulation(specs[0]) as sim:
        f0 = sim.features().cpu().numpy()
        f0b = sim.features().cpu().numpy()
        sim.load_fields(specs[1])
        f1 = sim.features().cpu().numpy().astype(np.float64)
    assert np.array_equal(f0, f0b)
    for f, spec in ((f0.astype(np.float64), specs[0]), (f1, specs[1])):
        ref = _box_features_oracle(spec)
        assert np.abs(f - ref).max() <= 1e-5 * max(1.0, ref[:, 1].max() ** 2)
    assert f1[0, 7] != f0[0, 7]          # the box clumping moved with the field


def test_features_of_a_batch_are_per_box():
    boxes = [W.make_box("c2", n=12, field_seed=3), W.make_box("c1", n=10)]
    boxes[1].z = 1250.0
    with M.Simulation(boxes) as sim:
        f = sim.features().cpu().numpy().astype(np.float64)
    off = 0
    for b in boxes:
        ref = _box_features_oracle(b)
        assert np.abs(f[off:off + b.ncells] - ref).max() <= 1e-5 * max(1.0, ref[:, 1].max() ** 2)
        off += b.ncells


def _test_params(seed, scale=1.0):
    p = WS.initial_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    p[512:576] = rng.normal(0.0, 0.3, 64)          # non-zero biases exercise the bias layout
    p[4672:4736] = rng.normal(0.0, 0.3, 64)
    p[4800] = 0.25
    return (p * scale).astype(np.float32)


def _forward_bound(p, X):
    W1, b1, W2, b2, w3, b3 = S.unpack(p)
    _, c = S.forward(p, X)
    e1 = 2.0 ** -8 * (np.abs(X) @ np.abs(W1).T)
    dz2 = (1.1 * e1 + 2.0 ** -8 * np.abs(c["h1"])) @ np.abs(W2).T
    return 1.1 * (dz2 @ np.abs(w3))


def _forward_sigma(p, X):
    """Standard deviation of the same first-order error when every BF16
    rounding is an independent error of standard deviation 2^-9/sqrt(3)
    relative (uniform within half an ulp): the worst case above adds all
    terms with one sign, this adds their squares."""
    W1, b1, W2, b2, w3, b3 = S.unpack(p)
    _, c = S.forward(p, X)
    u2 = (2.0 ** -9) ** 2 / 3.0
    v1 = 2.0 * u2 * ((X * X) @ (W1 * W1).T)                  # W1 and x rounded
    v2 = (1.21 * v1 + 2.0 * u2 * c["h1"] ** 2) @ (W2 * W2).T  # through ReLU; W2 and h1 rounded
    return np.sqrt(1.21 * (v2 @ (w3 * w3)))


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 65537])
def test_forward_matches_oracle_within_bf16_bound(n):
    rng = np.random.default_rng(n)
    X = rng.normal(0.0, 1.0, size=(n, 8)).astype(np.float32)
    X[:, 7] = 0.0
    p = _test_params(7, 1.5)
    with M.Mlp(p) as mlp:
        y = mlp.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = S.forward(p.astype(np.float64), X.astype(np.float64))
    bound = 1.5 * _forward_bound(p.astype(np.float64), X.astype(np.float64)) + 1e-5
    sigma = _forward_sigma(p.astype(np.float64), X.astype(np.float64))
    ratio = np.abs(y - ref) / bound
    z = np.abs(y - ref) / (sigma + 1e-6)
    _say(f"  n={n}: max |dy| {np.abs(y - ref).max():.3e}, max |dy|/bound {ratio.max():.3f}, "
         f"max |dy|/sigma {z.max():.2f}, rms |dy|/sigma {np.sqrt(np.mean(z * z)):.2f}")
    assert np.all(ratio <= 1.0)
    # and statistically: no cell beyond 7 sigma, the RMS near one sigma
    assert z.max() <= 7.0 and np.sqrt(np.mean(z * z)) <= 2.0
    # the oracle's BF16 network makes the same roundings: only FP32
    # accumulation is left, and now and then an activation that FP32 and
    # FP64 round to neighbouring BF16 values (within the bound above)
    yb, cb = S.forward_bf16(p.astype(np.float64), X.astype(np.float64))
    scale = np.abs(cb["h2"]) @ np.abs(cb["w3"]) + abs(float(p[4800]))
    close = np.abs(y - yb) <= 1e-5 * scale + 1e-6
    _say(f"  against the BF16 network: {np.mean(~close):.2e} of the cells beyond 1e-5 of the scale")
    assert np.mean(close) >= 0.99


def test_forward_sampled_at_256cube_size():
    """The inference launch of the 256^3 box (16.7 M cells): sampled cells
    against the oracle, and the flags of an envelope against plain float32
    comparisons (bit-exact)."""
    spec = W.make_box("c3", n_packets=1)
    with M.Simulation(spec) as sim:
        feats = sim.features()
    idx = np.random.default_rng(1).choice(spec.ncells, 4000, replace=False)
    X = feats[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    ref_f = _box_features_oracle(spec)[idx]
    assert np.abs(X - ref_f).max() <= 1e-5 * max(1.0, ref_f[:, 1].max() ** 2)
    p = _test_params(11)
    lo = np.quantile(X, 0.02, axis=0).astype(np.float32)
    hi = np.quantile(X, 0.98, axis=0).astype(np.float32)
    lo[4:] = -1.0
    hi[4:] = 1.0
    with M.Mlp(p) as mlp:
        mlp.set_envelope(lo, hi)
        y, flags, count = mlp.forward(feats, outside=True, count=True)
    y = y.cpu().numpy()[idx].astype(np.float64)
    # the oracle's network on the oracle's own features (within 1e-5 of the
    # library's, checked above; the BF16 bound dwarfs what that moves)
    ref, _ = S.forward(p.astype(np.float64), ref_f)
    bound = 1.5 * _forward_bound(p.astype(np.float64), ref_f) + 1e-4
    assert np.all(np.abs(y - ref) <= bound)
    f32 = feats.cpu().numpy()
    want = np.any((f32 < lo) | (f32 > hi), axis=1)
    got = flags.cpu().numpy().astype(bool)
    assert np.array_equal(got, want) and count == int(want.sum())
    _say(f"  {count} of {spec.ncells} cells outside the envelope")


@pytest.mark.parametrize("n", [1, 33, 5000])
def test_flags_follow_the_envelope_and_its_clearing(n):
    """No envelope flags nothing; an envelope flags exactly the cells a plain
    float32 comparison puts outside, ragged tiles included; clearing it
    flags nothing again. y does not depend on the envelope."""
    rng = np.random.default_rng(n + 5)
    X = rng.normal(0.0, 1.0, size=(n, 8)).astype(np.float32)
    lo = np.full(8, -1.5, np.float32)
    hi = np.full(8, 1.5, np.float32)
    Xd = torch.from_numpy(X).cuda()
    with M.Mlp(_test_params(3)) as mlp:
        y0, f0, c0 = mlp.forward(Xd, outside=True, count=True)
        mlp.set_envelope(lo, hi)
        y1, f1, c1 = mlp.forward(Xd, outside=True, count=True)
        mlp.set_envelope(None, None)
        y2, f2, c2 = mlp.forward(Xd, outside=True, count=True)
    want = np.any((X < lo) | (X > hi), axis=1)
    assert c0 == 0 and not f0.cpu().numpy().any()
    assert np.array_equal(f1.cpu().numpy().astype(bool), want) and c1 == int(want.sum())
    assert c2 == 0 and not f2.cpu().numpy().any()
    assert torch.equal(y0, y1) and torch.equal(y0, y2)


def test_train_steps_equal_single_steps_bit_for_bit():
    """Several steps in one call take the same batches, learning rates and
    Adam step counts as single steps: the same parameters and losses bit for
    bit. An index outside the set is reported."""
    X, t, w = _train_data(5000, 4)
    Xd, td, wd = (torch.from_numpy(a.astype(np.float32)).cuda() for a in (X, t, w))
    rng = np.random.default_rng(9)
    idx = torch.from_numpy(rng.integers(0, 5000, size=(7, 1000))).cuda()
    lrs = [3e-3 * 0.9 ** s for s in range(7)]
    p0 = _test_params(5)
    with M.Mlp(p0) as one, M.Mlp(p0) as many:
        want = [one.train_step(Xd[i].contiguous(), td[i].contiguous(), wd[i].contiguous(), lr, want_loss=True)
                for i, lr in zip(idx, lrs)]
        got = many.train_steps(Xd, td, wd, idx[:3], lrs[:3], want_losses=True)
        got += many.train_steps(Xd, td, wd, idx[3:], lrs[3:], want_losses=True)
        assert got == want
        assert np.array_equal(np.array(one.params()), np.array(many.params()))
        assert many.train_steps(Xd, td, wd, idx[:0], []) is None
        bad = idx[:1].clone()
        bad[0, 17] = 5000
        with pytest.raises(A.MCLyaError, match="outside"):
            many.train_steps(Xd, td, wd, bad, [1e-3])


def _train_data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, size=(n, 8))
    X[:, 7] = 0.0
    t = np.tanh(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2] - 0.2 * X[:, 3]
    w = rng.uniform(0.0, 2.0, size=n)
    return X.astype(np.float32), t.astype(np.float32), w.astype(np.float32)


def _away_from_kinks(p, X, t, w, margin=1e-3):
    """Keep the cells whose pre-activations (of the BF16 network) all stay at
    least `margin` from zero, where ReLU's derivative jumps: FP32 and FP64
    then take the same branch everywhere."""
    _, c = S.forward_bf16(p.astype(np.float64), X.astype(np.float64))
    keep = (np.abs(c["z1"]).min(axis=1) > margin) & (np.abs(c["z2"]).min(axis=1) > margin)
    return X[keep], t[keep], w[keep]


def _check_gradient(p, X, t, w):
    with M.Mlp(p) as mlp:
        g, loss = mlp.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(w).cuda())
        g2, loss2 = mlp.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(w).cuda())
    g = np.array(g, dtype=np.float64)
    L, gref, gabs = S.loss_and_grad_bf16(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64),
                                         w.astype(np.float64), abs_bound=True)
    err = np.abs(g - gref)
    tol = 2.0 ** -5 * gabs + 1e-6 * np.abs(gref).max()
    _say(f"  n={X.shape[0]}: loss gpu {loss:.7g} orc {L:.7g}; max |dg| / max |g| = "
         f"{err.max() / np.abs(gref).max():.2e}; max |dg| / tol = {(err / tol).max():.3f}")
    assert abs(loss - L) <= 1e-4 * L
    assert np.all(err <= tol)
    assert np.array_equal(g, np.array(g2)) and loss == loss2      # fixed summation order
    return err, gref


def test_gradient_matches_oracle():
    """The gradient of the BF16 network on the matrix cores against the
    oracle's straight-through gradient of the same network."""
    p = _test_params(5)
    X, t, w = _away_from_kinks(p, *_train_data(40000, 3))
    assert X.shape[0] > 10000
    err, gref = _check_gradient(p, X, t, w)
    assert err.max() <= 1e-2 * np.abs(gref).max()                # a gradient, not noise


@pytest.mark.parametrize("n", [1, 31, 33, 4097])
def test_gradient_ragged_batches(n):
    """Batches that fill no tile, a tile and a cell, and many tiles with a
    ragged tail: the cells past n must weigh nothing."""
    p = _test_params(8)
    X, t, w = _away_from_kinks(p, *_train_data(4 * n + 64, 10 + n))
    assert X.shape[0] >= n
    _check_gradient(p, X[:n].copy(), t[:n].copy(), w[:n].copy())


def test_adam_steps_match_oracle():
    """One step: the oracle's Adam on the oracle's gradient; coordinates with
    a clear gradient move by the same amount (Adam's first step is about
    -lr sign(g)). Thirty steps: the same loss trajectory; two runs identical."""
    p = _test_params(6)
    X, t, w = _away_from_kinks(p, *_train_data(16384, 4))
    lr = 1e-3
    Xd, td, wd = (torch.from_numpy(a).cuda() for a in (X, t, w))
    with M.Mlp(p) as mlp:
        mlp.train_step(Xd, td, wd, lr)
        p1 = np.array(mlp.params(), dtype=np.float64)
    X64, t64, w64 = X.astype(np.float64), t.astype(np.float64), w.astype(np.float64)
    _, g = S.loss_and_grad_bf16(p.astype(np.float64), X64, t64, w64)
    q, _, _ = S.adam_step(p.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, lr)
    clear = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.abs(p1 - q)[clear].max() <= 1e-2 * lr + 1e-6
    assert np.abs(p1 - q).max() <= 2 * lr + 1e-6
    runs = []
    for _ in range(2):
        losses = []
        with M.Mlp(p) as mlp:
            for _s in range(30):
                losses.append(mlp.train_step(Xd, td, wd, lr, want_loss=True))
            runs.append((losses, mlp.params()))
    assert runs[0] == runs[1]
    pq, m, v = p.astype(np.float64), np.zeros(S.N_PARAMS), np.zeros(S.N_PARAMS)
    ref_losses = []
    for s in range(1, 31):
        L, g = S.loss_and_grad_bf16(pq, X64, t64, w64)
        ref_losses.append(L)
        pq, m, v = S.adam_step(pq, m, v, g, s, lr)
    rel = np.abs(np.array(runs[0][0]) - np.array(ref_losses)) / np.array(ref_losses)
    _say(f"  loss {ref_losses[0]:.4f} -> {ref_losses[-1]:.4f}; max relative gap {rel.max():.2e}")
    assert ref_losses[-1] < 0.9 * ref_losses[0]
    assert rel.max() <= 1e-3


def test_mlp_errors():
    with pytest.raises(M.MCLyaError):
        M.Mlp([float("nan")] * 4801)
    with M.Mlp(_test_params(1)) as mlp:
        X = torch.zeros((4, 8), device="cuda")
        with pytest.raises(M.MCLyaError):
            mlp.set_envelope([1.0] * 8, [0.0] * 8)
        with pytest.raises(M.MCLyaError):
            mlp.gradient(X, torch.zeros(4, device="cuda"), torch.zeros(4, device="cuda"))
        with pytest.raises(M.MCLyaError):
            mlp.train_step(X, torch.zeros(4, device="cuda"), torch.ones(4, device="cuda"), lr=-1.0)
        assert mlp.forward(X[:0]).numel() == 0


def test_targets_match_oracle():
    """ln M_c and the emission-share weights from the library's tallies
    against the oracle's targets from the oracle's own walk of the same box.
    y differs by the tallies' difference (per cell within 1e-3 of A_c plus
    1e-6 of the mean, so |dy| <= ~1e-3 where A_c is not tiny); the weights
    depend only on the fields (FP32 products against FP64: 1e-6)."""
    from oracle import walker
    spec = W.make_box("c2", n=24, n_packets=60_000)
    with M.Simulation(spec) as sim:
        sim.emit()
        sim.transport()
        sim.tally()
        y, w = sim.targets()
    y, w = y.cpu().numpy().astype(np.float64), w.cpu().numpy().astype(np.float64)
    ref = walker.run_box(spec)
    y_o, w_o = S.targets(spec, ref["A"], ref["escaped"], spec.n_packets)
    assert np.array_equal(w > 0, w_o > 0)
    assert np.allclose(w, w_o, rtol=1e-6, atol=0.0)
    A_o = ref["A"].astype(np.float64)
    big = A_o > 1e-2 * A_o.mean()
    _say(f"  worst |dy| where A_c > 1% of the mean: {np.abs(y - y_o)[big].max():.2e}")
    assert np.abs(y - y_o)[big].max() <= 2e-3
    assert np.sum(w_o) <= 1.0 + 1e-12
