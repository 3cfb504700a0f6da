"""FP64 oracle of the per-cell surrogate for the Lyman-alpha mixing correction.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. It is written independently of the HIP
library.

What is approximated. The Monte Carlo gives, per cell, the absorbed weight A_c
and from it the mixing correction M_c = A_c / A_c^fm, with A_c^fm the
absorption the cell would receive under full mixing (absorptions spread like
n_1s, Sec. IV.B, Eq. (dotne-mix)). M = 1 everywhere is full mixing; local
absorption (short mixing length, Sec. III.B, Fig. MCtravel) makes M follow the
local emission. The surrogate regresses y = ln M_c on eight local features of
the cell with a small multilayer perceptron, so that the correction can be
evaluated without the transport.

Features, per cell c of a periodic box (all plain definitions):
  0  ln Delta_c
  1  mean of Delta over the 3x3x3 cells centred on c
  2  variance of Delta over the same 27 cells (mean of squared deviations)
  3  div U at c by central differences, (U_x[i+1] - U_x[i-1]) / 2 + (y) + (z),
     in thermal velocities per cell (0 without a flow)
  4  ln(T / 3000 K)
  5  x_e at c
  6  z / 1000 - 1.1
  7  ln(<Delta^2> / <Delta>^2) over the whole box, ln(1 + b) with b the
     clumping factor of Sec. II.C, Eq. (clumpingfactor)

Network: 8 -> 64 -> 64 -> 1 with ReLU activations, relu(z) = max(z, 0) (its
derivative taken as 0 at z = 0).
Parameters are one flat vector of 4801 numbers:
  W1 [64][8] at 0, b1 [64] at 512, W2 [64][64] at 576, b2 [64] at 4672,
  w3 [64] at 4736, b3 at 4800;  row-major [out][in].
Loss: weighted mean squared error sum_i w_i (y_i - t_i)^2 / sum_i w_i.
Optimiser: Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.

The network as the matrix cores evaluate it ("bf16" below): the features, W1,
W2 and the layer-1 activations rounded to bfloat16 (8 significant bits, ties
to even), each of b1 and b2 as the two bfloat16 terms hi = bf16(b),
lo = bf16(b - hi) (their sum is b to 2^-16 relative), w3, b3 and the last
layer exact. Its gradient with respect to the unrounded parameters passes
every rounding through unchanged (the straight-through derivative).
"""
import numpy as np

N_FEAT = 8
HIDDEN = 64
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 512, 576, 4672, 4736, 4800
N_PARAMS = 4801


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# --- features ----------------------------------------------------------------
def features(overdensity, velocity=None, x_e=0.1, temp_K=3000.0, z=1100.0):
    """[cells, 8] features of a box; arrays are [z][y][x] (velocity [3][z][y][x])."""
    od = _f64(overdensity)
    nz, ny, nx = od.shape
    s = np.zeros_like(od)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s += np.roll(od, (dz, dy, dx), axis=(0, 1, 2))
    mean = s / 27.0
    ss = np.zeros_like(od)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = np.roll(od, (dz, dy, dx), axis=(0, 1, 2)) - mean
                ss += d * d
    var = ss / 27.0
    div = np.zeros_like(od)
    if velocity is not None:
        v = _f64(velocity)
        # component a varies along array axis 2 - a (x is the last axis);
        # roll by -1 brings cell i+1 to position i
        for a in range(3):
            ax = 2 - a
            div += 0.5 * (np.roll(v[a], -1, axis=ax) - np.roll(v[a], 1, axis=ax))
    xe = _f64(x_e) * np.ones_like(od) if np.ndim(x_e) == 0 else _f64(x_e).reshape(od.shape)
    f = np.zeros((od.size, N_FEAT))
    f[:, 0] = np.log(od).reshape(-1)
    f[:, 1] = mean.reshape(-1)
    f[:, 2] = var.reshape(-1)
    f[:, 3] = div.reshape(-1)
    f[:, 4] = np.log(temp_K / 3000.0)
    f[:, 5] = xe.reshape(-1)
    f[:, 6] = z / 1000.0 - 1.1
    f[:, 7] = np.log(np.mean(od * od) / np.mean(od) ** 2)
    return f


# --- network -----------------------------------------------------------------
def targets(spec, A, E, n_packets, wing=0):
    """Regression data of the surrogate from a box's tallies: y = ln M_c
    (M_c = A_c / A_c^fm, the mixing correction of Sec. IV.B, Eq. (dotne-mix),
    as the feed forms it) and the loss weight of the cell, its share
    S_c / sum(S) of the box's recombination source. Cells with M_c = 0 have no
    logarithm: y = 0, weight 0."""
    from . import physics as P
    mix = P.feed(spec, A, E, n_packets, wing)["mix_corr"]
    S = P.emission_weights(spec)
    ok = mix > 0
    y = np.where(ok, np.log(np.where(ok, mix, 1.0)), 0.0)
    w = np.where(ok, S / S.sum(), 0.0)
    return y, w


def unpack(params):
    p = _f64(params)
    W1 = p[OFF_W1:OFF_B1].reshape(HIDDEN, N_FEAT)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(HIDDEN, HIDDEN)
    b2 = p[OFF_B2:OFF_W3]
    w3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([_f64(W1).reshape(-1), _f64(b1), _f64(W2).reshape(-1), _f64(b2), _f64(w3),
                           [float(b3)]])


def relu(z):
    return np.maximum(z, 0.0)


def relu_grad(z):
    return (z > 0.0).astype(np.float64)


def forward(params, X):
    """y [n] and the intermediate values of the network on features X [n, 8]."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    X = _f64(X)
    z1 = X @ W1.T + b1
    h1 = relu(z1)
    z2 = h1 @ W2.T + b2
    h2 = relu(z2)
    y = h2 @ w3 + b3
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(params, X, t, w):
    """Weighted MSE and its gradient with respect to the 4801 parameters
    (the chain rule written out layer by layer)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    y, c = forward(params, X)
    w = _f64(w)
    sw = w.sum()
    r = y - _f64(t)
    L = float((w * r * r).sum() / sw)
    gy = 2.0 * w * r / sw                       # dL/dy
    gw3 = c["h2"].T @ gy
    gb3 = gy.sum()
    gz2 = np.outer(gy, w3) * relu_grad(c["z2"])
    gW2 = gz2.T @ c["h1"]
    gb2 = gz2.sum(axis=0)
    gz1 = (gz2 @ W2) * relu_grad(c["z1"])
    gW1 = gz1.T @ c["X"]
    gb1 = gz1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(params, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * _f64(m) + (1.0 - beta1) * _f64(g)
    v = beta2 * _f64(v) + (1.0 - beta2) * _f64(g) * _f64(g)
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return _f64(params) - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --- the bfloat16 network ----------------------------------------------------
def bf16(a):
    """Round to bfloat16, ties to even, after rounding to binary32 (returned
    as float64): on the binary32 bit pattern, add 0x7FFF plus the lowest kept
    bit (bit 16), then clear the 16 low bits. Finite inputs only."""
    a = np.asarray(a, dtype=np.float64)
    f = np.ascontiguousarray(a.astype(np.float32)).reshape(-1)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(a.shape)


def bias_split(b):
    """b as hi + lo, hi = bf16(b), lo = bf16(b - hi) (b - hi is exact in
    binary32 and in float64)."""
    b32 = _f64(np.asarray(b, dtype=np.float64).astype(np.float32))
    hi = bf16(b32)
    return hi, bf16(b32 - hi)


def forward_bf16(params, X):
    """y [n] and the intermediate values of the bfloat16 network."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    Xb, W1b, W2b = bf16(X), bf16(W1), bf16(W2)
    b1e, b2e = sum(bias_split(b1)), sum(bias_split(b2))
    z1 = Xb @ W1b.T + b1e
    h1 = bf16(relu(z1))
    z2 = h1 @ W2b.T + b2e
    h2 = relu(z2)
    w3 = _f64(np.asarray(w3).astype(np.float32))
    y = h2 @ w3 + float(np.float32(b3))
    return y, dict(X=Xb, W2=W2b, w3=w3, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad_bf16(params, X, t, w, abs_bound=False):
    """Weighted MSE of the bfloat16 network and its straight-through gradient
    (the chain rule of loss_and_grad with the rounded operands). With
    abs_bound, also the same chain taken with absolute values of every factor
    (and of dL/dy), the scale of the rounding errors of each gradient entry."""
    y, c = forward_bf16(params, X)
    w = _f64(w)
    sw = w.sum()
    r = y - _f64(t)
    L = float((w * r * r).sum() / sw)
    gy = 2.0 * w * r / sw

    def chain(gy, w3, W2, h1, h2, X, m1, m2):
        gz2 = np.outer(gy, w3) * m2
        gz1 = (gz2 @ W2) * m1
        return pack(gz1.T @ X, gz1.sum(axis=0), gz2.T @ h1, gz2.sum(axis=0), h2.T @ gy, gy.sum())

    m1 = (c["z1"] > 0.0).astype(np.float64)
    m2 = (c["z2"] > 0.0).astype(np.float64)
    g = chain(gy, c["w3"], c["W2"], c["h1"], c["h2"], c["X"], m1, m2)
    if not abs_bound:
        return L, g
    gabs = chain(np.abs(gy), np.abs(c["w3"]), np.abs(c["W2"]), c["h1"], c["h2"], np.abs(c["X"]), m1, m2)
    return L, g, gabs
