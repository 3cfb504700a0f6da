"""Host logic of the experiment drivers (CPU only): the fraction beyond a
distance, its diffusive counterpart against a sampled 3-D Gaussian, the grid
of the flow test, and the media the drivers build."""
import math

import numpy as np
import pytest

from paper_2312_11448_amd import experiments as X
import workloads as W


def test_fraction_beyond():
    d = np.array([0.1, 0.5, 0.5, 2.0])
    assert X.fraction_beyond(d, [0.0, 0.1, 0.5, 1.0, 2.0]).tolist() == [1.0, 0.75, 0.25, 0.25, 0.0]
    assert X.fraction_beyond([], [1.0]).tolist() == [1.0]


def test_diffusion_beyond_is_the_gaussian_law():
    """The closed form against 10^6 draws of a 3-D Gaussian with the same
    mean square distance, and its limits."""
    rng = np.random.default_rng(3)
    r = np.linalg.norm(rng.normal(0.0, 0.7, size=(1_000_000, 3)), axis=1)
    D = np.array([0.1, 0.5, 1.0, 1.5, 2.5])
    f = X.diffusion_beyond(r, D)
    emp = X.fraction_beyond(r, D)
    assert np.all(np.abs(f - emp) <= 4.0 * np.sqrt(emp * (1.0 - emp) / r.size) + 1e-6)
    assert X.diffusion_beyond(r, [0.0])[0] == pytest.approx(1.0)
    assert X.diffusion_beyond(r, [100.0])[0] < 1e-300


def test_cells_per_wavelength():
    assert X.cells_per_wavelength(0.1) == 16 and X.cells_per_wavelength(1.0) == 16
    assert X.cells_per_wavelength(10.0) == 128 and X.cells_per_wavelength(1000.0) == 16384
    for lam in (0.05, 3.0, 77.0, 1e4):
        n = X.cells_per_wavelength(lam)
        assert n >= 16 and lam * 1e3 / n <= 100.0 and (n == 16 or lam * 1e3 / (n // 2) > 100.0)


def test_media():
    s = W.escape_slab(64, 0.25, 1e19, 100)
    assert s.n == (64, 1, 1) and s.source.sum() == 2.0 and s.source[0, 0, 0] == s.source[0, 0, 63] == 1.0
    u = s.velocity[0, 0, 0]
    assert u[0] == pytest.approx(0.25 * math.sin(math.pi / 64)) and u[63] == pytest.approx(-u[0])
    assert np.all(s.velocity[1:] == 0.0) and np.all(s.overdensity == 1.0)
    t = X.travel_box(1200.0, 0.33, 10)
    assert t.profile == "voigt" and t.zeta == 1.0 and t.temp_K == pytest.approx(2.7255 * 1201.0)
    assert t.x_e_uniform == pytest.approx(0.33) and t.cell_cm == pytest.approx(X.KPC_CM)
