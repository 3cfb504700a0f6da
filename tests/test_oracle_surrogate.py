"""Pins of the surrogate oracle (features, network, loss gradient, Adam)
against closed forms, finite differences and hand-built networks."""
import math

import numpy as np
import pytest

from oracle import surrogate as S


def _sine_box(n, amp, axis):
    """Delta = 1 + amp sin(2 pi i / n) along one array axis."""
    i = np.arange(n)
    prof = 1.0 + amp * np.sin(2.0 * np.pi * i / n)
    shape = [1, 1, 1]
    shape[axis] = n
    return np.broadcast_to(prof.reshape(shape), (n, n, n)).copy(), prof


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_neighbourhood_mean_and_variance_closed_form(axis):
    """For Delta varying along one axis as 1 + a sin(theta), the 27 cells hold
    the three values at theta - h, theta, theta + h nine times each:
    mean = 1 + a sin(theta)(1 + 2 cos h)/3 and the variance is the spread of
    those three values."""
    n, a = 16, 0.4
    od, _ = _sine_box(n, a, axis)
    f = S.features(od)
    h = 2.0 * math.pi / n
    theta = 2.0 * math.pi * np.arange(n) / n
    mean = 1.0 + a * np.sin(theta) * (1.0 + 2.0 * math.cos(h)) / 3.0
    vals = np.stack([a * np.sin(theta - h), a * np.sin(theta), a * np.sin(theta + h)])
    var = (vals ** 2).mean(axis=0) - vals.mean(axis=0) ** 2
    idx = [0, 0, 0]
    got_m, got_v = [], []
    for i in range(n):
        idx[axis] = i
        c = (idx[0] * n + idx[1]) * n + idx[2]
        got_m.append(f[c, 1])
        got_v.append(f[c, 2])
    assert np.allclose(got_m, mean, rtol=0, atol=1e-13)
    assert np.allclose(got_v, var, rtol=0, atol=1e-13)
    assert np.allclose(np.exp(f[:, 0]), od.reshape(-1), rtol=1e-14)
    # clumping: <(1 + a sin)^2> = 1 + a^2 / 2 over whole periods, <Delta> = 1
    assert np.allclose(f[:, 7], math.log(1.0 + a * a / 2.0), rtol=0, atol=1e-13)


def test_clumping_of_a_two_phase_box():
    """Half the cells at 1 + a, half at 1 - a: <Delta^2>/<Delta>^2 = 1 + a^2,
    whatever the arrangement (Eq. (clumpingfactor), b = a^2)."""
    rng = np.random.default_rng(9)
    a = 0.6
    v = np.where(rng.permutation(512) < 256, 1.0 + a, 1.0 - a).reshape(8, 8, 8)
    f = S.features(v)
    assert np.allclose(f[:, 7], math.log(1.0 + a * a), atol=1e-14)
    f2 = S.features(3.0 * v)           # a uniform rescaling leaves it unchanged
    assert np.allclose(f2[:, 7], f[:, 7], atol=1e-14)


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_divergence_central_difference_closed_form(comp):
    """U_comp = b sin(2 pi k / n) along its own coordinate k: the central
    difference is b cos(theta) sin(h); components along other axes add nothing."""
    n, b = 12, 0.3
    od = np.ones((n, n, n))
    vel = np.zeros((3, n, n, n))
    i = np.arange(n)
    prof = b * np.sin(2.0 * np.pi * i / n)
    axis = 2 - comp                 # x is the last array axis
    shape = [1, 1, 1]
    shape[axis] = n
    vel[comp] = np.broadcast_to(prof.reshape(shape), (n, n, n))
    # a transverse component (varies across its own direction) has no divergence
    other = (comp + 1) % 3
    vel[other] = np.broadcast_to(prof.reshape(shape), (n, n, n))
    f = S.features(od, vel)
    h = 2.0 * math.pi / n
    want = b * np.cos(2.0 * math.pi * i / n) * math.sin(h)
    idx = [0, 0, 0]
    for k in range(n):
        idx[axis] = k
        c = (idx[0] * n + idx[1]) * n + idx[2]
        assert abs(f[c, 3] - want[k]) < 1e-14


def test_scalar_features():
    od = np.full((4, 4, 4), 2.0)
    f = S.features(od, None, x_e=0.25, temp_K=3000.0 * math.e, z=800.0)
    assert np.allclose(f[:, 0], math.log(2.0)) and np.allclose(f[:, 1], 2.0) and np.allclose(f[:, 2], 0.0)
    assert np.allclose(f[:, 3], 0.0) and np.allclose(f[:, 4], 1.0) and np.allclose(f[:, 5], 0.25)
    assert np.allclose(f[:, 6], -0.3) and np.allclose(f[:, 7], 0.0)


def _random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, S.N_PARAMS) * np.concatenate(
        [np.full(512, 1 / math.sqrt(8)), np.full(64, 0.1), np.full(4096, 1 / 8.0), np.full(64, 0.1),
         np.full(64, 1 / 8.0), [0.1]])


def test_hand_built_network():
    """Only W1[0][0] = W2[0][0] = w3[0] = 1: y = max(x0, 0) + b3; a hidden
    unit fed only by a bias adds relu(relu(b)) through w3; a unit with a
    negative pre-activation adds nothing."""
    W1 = np.zeros((64, 8)); W1[0, 0] = 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.0
    w3 = np.zeros(64); w3[0] = 1.0
    p = S.pack(W1, np.zeros(64), W2, np.zeros(64), w3, 0.5)
    X = np.zeros((5, 8)); X[:, 0] = [-3.0, -0.5, 0.0, 0.7, 4.0]
    y, _ = S.forward(p, X)
    assert np.allclose(y, [0.5, 0.5, 0.5, 1.2, 4.5], rtol=0, atol=1e-15)
    b1 = np.zeros(64); b1[5] = 2.0; b1[6] = -1.0
    W2b = W2.copy(); W2b[7, 5] = 1.5; W2b[8, 6] = 1.0
    w3b = w3.copy(); w3b[7] = -1.0; w3b[8] = 10.0
    y2, _ = S.forward(S.pack(W1, b1, W2b, np.zeros(64), w3b, 0.5), X)
    assert np.allclose(y2 - y, -3.0, atol=1e-15)
    # a sign flip of the first layer: y = max(-x0, 0) + b3
    y3, _ = S.forward(S.pack(-W1, np.zeros(64), W2, np.zeros(64), w3, 0.5), X)
    assert np.allclose(y3, [3.5, 1.0, 0.5, 0.5, 0.5], atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = _random_params(1)
    X = rng.normal(size=(40, 8))
    t = rng.normal(size=40)
    w = rng.uniform(0.1, 2.0, size=40)
    L, g = S.loss_and_grad(p, X, t, w)
    idx = np.concatenate([rng.choice(512, 12, replace=False), 512 + rng.choice(64, 6, replace=False),
                          576 + rng.choice(4096, 20, replace=False), 4672 + rng.choice(64, 6, replace=False),
                          4736 + rng.choice(64, 6, replace=False), [4800]])
    for i in idx:
        e = np.zeros_like(p)
        step = 1e-6 * max(1.0, abs(p[i]))
        e[i] = step
        Lp, _ = S.loss_and_grad(p + e, X, t, w)
        Lm, _ = S.loss_and_grad(p - e, X, t, w)
        fd = (Lp - Lm) / (2 * step)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_loss_is_weighted_mean_and_scale_free():
    rng = np.random.default_rng(4)
    p = _random_params(2)
    X = rng.normal(size=(30, 8))
    t = rng.normal(size=30)
    w = rng.uniform(0.0, 1.0, size=30)
    L1, g1 = S.loss_and_grad(p, X, t, w)
    L2, g2 = S.loss_and_grad(p, X, t, 7.5 * w)
    assert abs(L1 - L2) < 1e-14 * L1 and np.allclose(g1, g2, rtol=1e-12, atol=1e-15)
    y, _ = S.forward(p, X)
    # equal weights: the plain mean of squared residuals
    L3, _ = S.loss_and_grad(p, X, t, np.ones(30))
    assert abs(L3 - np.mean((y - t) ** 2)) < 1e-13


def test_adam_constant_gradient_moves_by_lr():
    """With bias correction and a constant gradient g, m_hat = g and
    v_hat = g^2 at every step, so each parameter moves by
    -lr g / (|g| + eps) per step (Kingma & Ba 2015, Sec. 2)."""
    rng = np.random.default_rng(5)
    g = rng.normal(size=50)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    p0 = p.copy()
    for step in range(1, 6):
        p, m, v = S.adam_step(p, m, v, g, step, lr, 0.9, 0.999, eps)
        want = p0 - step * lr * g / (np.abs(g) + eps)
        assert np.allclose(p, want, rtol=0, atol=1e-15 * step + 1e-16)


def test_adam_reaches_minimum_of_quadratic():
    """On f(x) = sum a_i (x_i - c_i)^2 / 2 Adam converges to c."""
    rng = np.random.default_rng(6)
    a = rng.uniform(0.5, 3.0, 20)
    c = rng.normal(size=20)
    x = np.zeros(20)
    m = np.zeros(20)
    v = np.zeros(20)
    for step in range(1, 4001):
        lr = 0.05 if step < 2000 else 0.005
        x, m, v = S.adam_step(x, m, v, a * (x - c), step, lr)
    assert np.max(np.abs(x - c)) < 1e-3


# --- the bfloat16 network ----------------------------------------------------
def test_bf16_rounding_matches_torch_and_ties_to_even():
    """bf16() against torch's float32 -> bfloat16 conversion (round to nearest
    even) over many magnitudes, and hand-made ties: with 8 significant bits,
    1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and goes to the even 1;
    1 + 3 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6 and goes to
    1 + 2^-6."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    x = (rng.normal(size=20000) * 10.0 ** rng.uniform(-30, 30, size=20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2.0 ** 10 * (1 + 2.0 ** -8)])
    assert np.array_equal(S.bf16(ties), [1.0, 1 + 2.0 ** -6, -1.0, 2.0 ** 10])
    assert np.array_equal(S.bf16(1 + 2.0 ** -8 + 2.0 ** -20), 1 + 2.0 ** -7)   # just above the tie


def test_bias_split_is_exact_to_two_to_minus_sixteen():
    rng = np.random.default_rng(13)
    b = rng.normal(size=5000).astype(np.float32).astype(np.float64)
    hi, lo = S.bias_split(b)
    assert np.array_equal(S.bf16(hi), hi) and np.array_equal(S.bf16(lo), lo)
    assert np.all(np.abs(hi + lo - b) <= 2.0 ** -16 * np.abs(b))
    exact = S.bf16(b)                                # representable biases: lo = 0
    assert np.all(S.bias_split(exact)[1] == 0.0)


def _representable_net(seed):
    """Weights, biases and features on coarse dyadic grids, so every
    product and sum of the network is exact in bfloat16: the rounded network
    is then the plain one."""
    rng = np.random.default_rng(seed)
    W1 = rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], size=(64, 8))
    W2 = rng.choice([-0.25, 0.0, 0.125, 0.25], size=(64, 64)) * (rng.random((64, 64)) < 0.1)
    b1 = rng.choice([-1.0, 0.0, 0.5, 2.0], size=64)
    b2 = rng.choice([-0.5, 0.0, 0.25], size=64)
    w3 = rng.normal(size=64)
    p = S.pack(W1, b1, W2, b2, w3.astype(np.float32), np.float32(0.3))
    X = rng.integers(-3, 4, size=(200, 8)).astype(np.float64)
    return p, X


def test_bf16_network_reduces_to_the_plain_one_on_representable_values():
    p, X = _representable_net(14)
    y, c = S.forward(p, X)
    yb, cb = S.forward_bf16(p, X)
    assert np.array_equal(cb["h1"], c["h1"])         # every activation exact
    assert np.allclose(yb, y, rtol=1e-14, atol=1e-14)
    rng = np.random.default_rng(15)
    t = rng.normal(size=200)
    w = rng.uniform(0.1, 1.0, size=200)
    L, g = S.loss_and_grad(p, X, t, w)
    Lb, gb, gabs = S.loss_and_grad_bf16(p, X, t, w, abs_bound=True)
    assert abs(Lb - L) <= 1e-13 * L
    assert np.allclose(gb, g, rtol=1e-12, atol=1e-14)
    assert np.all(gabs >= np.abs(gb) - 1e-12)


def test_bf16_network_rounds_where_stated():
    """Generic parameters: the rounded network differs from the plain one by
    no more than its roundings allow (W1, x, W2 and h1 at 2^-8 relative each,
    first order), and its gradient equals the plain gradient evaluated with
    the rounded operands: bf16 weights and features give the same network as
    the rounded parameters fed to the plain forward, up to the h1 rounding."""
    rng = np.random.default_rng(16)
    p = _random_params(4)
    X = rng.normal(size=(300, 8))
    y, c = S.forward(p, X)
    yb, cb = S.forward_bf16(p, X)
    W1, b1, W2, b2, w3, b3 = S.unpack(p)
    e1 = 2.0 ** -7 * (np.abs(X) @ np.abs(W1).T) + 2.0 ** -16 * np.abs(b1)
    e2 = (e1 + 2.0 ** -8 * np.abs(c["h1"])) @ np.abs(W2).T + 2.0 ** -8 * (np.abs(c["h1"]) @ np.abs(W2).T)
    bound = 1.1 * (e2 @ np.abs(w3)) + 1e-12
    assert np.all(np.abs(yb - y) <= bound)
    assert np.any(yb != y)                          # the roundings do act
    # with X and the weights already rounded, only h1 and the biases still round
    W1r, W2r = S.bf16(W1), S.bf16(W2)
    pr = S.pack(W1r, np.float32(b1), W2r, np.float32(b2), np.float32(w3), np.float32(b3))
    yr, cr = S.forward_bf16(pr, S.bf16(X))
    assert np.array_equal(yr, yb)


def test_targets_reduce_to_definitions():
    """ln M and the emission-share weights (Sec. IV.B, Eq. (dotne-mix)):
    tallies spread exactly like n_1s give M = 1 (y = 0) in every cell; one
    cell holding twice its full-mixing share (the others scaled to keep the
    total) gives y = ln 2 there; a cell that absorbed nothing gets weight 0;
    the weights are S_c / sum(S)."""
    import workloads as W
    from oracle import physics as P
    spec = W.make_box("c2", n=6, n_packets=1000)
    n1s = P.n1s_field(spec)
    S_w = P.emission_weights(spec)
    A_fm = n1s / n1s.sum() * 1e12
    y, w = S.targets(spec, A_fm, 0, spec.n_packets)
    assert np.abs(y).max() < 1e-12
    assert np.allclose(w, S_w / S_w.sum(), rtol=1e-14)
    A2 = A_fm.copy()
    A2[5] *= 2.0
    y2, _ = S.targets(spec, A2, 0, spec.n_packets)
    tot = A2.sum()
    expect5 = np.log(A2[5] / (tot * n1s[5] / n1s.sum()))
    assert y2[5] == pytest.approx(expect5, rel=1e-12)
    assert y2[5] == pytest.approx(np.log(2.0) + np.log(A_fm.sum() / tot), rel=1e-12)
    A3 = A_fm.copy()
    A3[7] = 0.0
    y3, w3 = S.targets(spec, A3, 0, spec.n_packets)
    assert y3[7] == 0.0 and w3[7] == 0.0 and (w3[np.arange(w3.size) != 7] > 0).all()
