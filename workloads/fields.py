"""Synthetic overdensity and peculiar-velocity fields.

Stand-ins for the MHD snapshots the paper ran its Monte Carlo on (Sec. III.B):
those snapshots are not available, so the fields below reproduce their shape,
size and statistics instead. Arrays are C-ordered ``[z][y][x]`` (x fastest);
velocities are structure-of-arrays ``[3][z][y][x]`` in units of the thermal
Doppler velocity. Every generator is driven by numpy's Philox bit generator with
an explicit seed, so the same seed always gives the same bytes.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.Philox(int(seed)))


def lognormal_white(n, ln_sigma, seed):
    """White (uncorrelated) lognormal overdensity with unit mean.

    Delta = exp(ln_sigma * g - ln_sigma**2 / 2), g ~ N(0, 1) per cell.
    """
    g = _rng(seed).standard_normal((n, n, n))
    d = np.exp(ln_sigma * g - 0.5 * ln_sigma * ln_sigma)
    return d.astype(np.float32)


def _kgrid(n):
    k1 = np.fft.fftfreq(n, d=1.0 / n)           # integer wavenumbers
    kz = k1[:, None, None]
    ky = k1[None, :, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, None, :]
    return kx, ky, kz


def grf_k2(n, rms, kmax, seed, clip=(1e-2, 1e2), vel_rms=0.1, device=None):
    """Gaussian random field with a k^2 power spectrum and a matching flow.

    The spectrum P(k) ~ k^2 on integer wavenumbers 1 <= |k| <= kmax mirrors the
    Batchelor-type magnetic spectrum the paper excites (Sec. II.C); the
    overdensity is 1 + delta, clipped to ``clip`` and renormalised to unit mean.
    The velocity is the curl-free flow v_k = i k delta_k / k^2 (infall into
    overdensities, div v = -delta), scaled to a 3-D rms of ``vel_rms``.
    Returns (overdensity float32 [n,n,n], velocity float32 [3,n,n,n]).
    device: a torch GPU device to take the same steps in float64 on it (the
    same seeded white noise; only the FFTs' rounding differs, far below the
    float32 result's).
    """
    rng = _rng(seed)
    white = rng.standard_normal((n, n, n))
    if device is not None:
        return _grf_k2_torch(white, n, rms, kmax, clip, vel_rms, device)
    wk = np.fft.rfftn(white)
    kx, ky, kz = _kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    kmag = np.sqrt(k2)
    amp = np.where((kmag >= 1.0) & (kmag <= kmax), kmag, 0.0)   # sqrt(P) ~ k
    dk = wk * amp
    delta = np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2))
    scale = rms / np.sqrt(np.mean(delta * delta))
    delta *= scale
    dk *= scale
    od = np.clip(1.0 + delta, clip[0], clip[1])
    od /= od.mean()
    vel = None
    if vel_rms is not None and vel_rms > 0:
        safe = np.where(k2 > 0, k2, 1.0)
        comps = []
        for kc in (kx, ky, kz):
            vk = 1j * np.broadcast_to(kc, dk.shape) * dk / safe
            comps.append(np.fft.irfftn(vk, s=(n, n, n), axes=(0, 1, 2)))
        v = np.stack(comps)
        v *= vel_rms / np.sqrt(np.mean(np.sum(v * v, axis=0)))
        vel = v.astype(np.float32)
    return od.astype(np.float32), vel


def _grf_k2_torch(white, n, rms, kmax, clip, vel_rms, device):
    import torch
    w = torch.from_numpy(white).to(device)
    wk = torch.fft.rfftn(w)
    kx, ky, kz = (torch.from_numpy(np.ascontiguousarray(k)).to(device) for k in _kgrid(n))
    k2 = kx * kx + ky * ky + kz * kz
    kmag = torch.sqrt(k2)
    amp = torch.where((kmag >= 1.0) & (kmag <= kmax), kmag, torch.zeros_like(kmag))
    dk = wk * amp
    delta = torch.fft.irfftn(dk, s=(n, n, n), dim=(0, 1, 2))
    scale = rms / torch.sqrt(torch.mean(delta * delta))
    delta = delta * scale
    dk = dk * scale
    od = torch.clamp(1.0 + delta, clip[0], clip[1])
    od = od / od.mean()
    vel = None
    if vel_rms is not None and vel_rms > 0:
        safe = torch.where(k2 > 0, k2, torch.ones_like(k2))
        comps = [torch.fft.irfftn(1j * kc * dk / safe, s=(n, n, n), dim=(0, 1, 2)) for kc in (kx, ky, kz)]
        v = torch.stack(comps)
        v = v * (vel_rms / torch.sqrt(torch.mean(torch.sum(v * v, dim=0))))
        vel = v.to(torch.float32).cpu().numpy()
    return od.to(torch.float32).cpu().numpy(), vel


def uniform_box(n, value=1.0):
    """Homogeneous overdensity (every cell equal to ``value``)."""
    return np.full((n, n, n), value, dtype=np.float32)


def sinusoidal_profile(n, amplitude, periods=1):
    """amplitude * sin(2 pi periods x / L) at the n cell centres, float64."""
    x = (np.arange(n) + 0.5) / n
    return amplitude * np.sin(2.0 * np.pi * periods * x)


def sinusoidal_flow(n, amplitude, periods=1, axis=0):
    """Bulk flow v = amplitude * sin(2 pi periods x / L) along one axis.

    The flow family of the paper's escape test (Fig. MCescape caption), on the
    grid. Returns float32 [3,n,n,n] with only component ``axis`` non-zero.
    """
    prof = sinusoidal_profile(n, amplitude, periods)
    v = np.zeros((3, n, n, n), dtype=np.float64)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    v[axis] = prof.reshape(shape)
    return v.astype(np.float32)
