"""Seeded acquisition inputs: source/receiver points, source wavelet, time step, sampling,
measurement noise.  Seeded-input side only (no finite-element arithmetic).
"""
from __future__ import annotations

import numpy as np

ORBIT_RADIUS = 1.4

# Courant numbers: dt = COURANT[d] * h * sqrt(eps_min).  They put dt at about half of the
# leap-frog stability limit 2 / sqrt(lambda_max(M^-1 K)) of the uniform Kuhn meshes used
# here (lumped mass; the limit is checked against a power iteration in the tests).
COURANT = {2: 0.345, 3: 0.283}


def time_step(d: int, h: float, eps_min: float) -> float:
    return COURANT[d] * h * float(np.sqrt(eps_min))


def circle_points(n: int, radius: float = ORBIT_RADIUS) -> np.ndarray:
    """n points evenly spaced on a circle, the first at angle pi/2, i.e. (0, radius)."""
    th = np.pi / 2 + 2 * np.pi * np.arange(n) / n
    return np.stack([radius * np.cos(th), radius * np.sin(th)], axis=1)


def sphere_points(n: int, radius: float = ORBIT_RADIUS) -> np.ndarray:
    """Fibonacci-sphere points, scaled to the orbit radius."""
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(1.0 - z * z)
    golden = np.pi * (3.0 - np.sqrt(5.0))
    phi = golden * k
    return radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def monostatic(src: np.ndarray) -> np.ndarray:
    """Receivers at the source points: shape (n_src, 1, d)."""
    return src[:, None, :].copy()


def bistatic_antipodal(src: np.ndarray) -> np.ndarray:
    """Two receivers per source: the source point and its antipode, shape (n_src, 2, d)."""
    return np.stack([src, -src], axis=1)


def gaussian_sine(t: np.ndarray, f0: float) -> np.ndarray:
    """Gaussian-modulated sinusoid sin(2 pi f0 (t - t0)) exp(-(t - t0)^2 / (2 tau^2)),
    tau = 1 / f0, t0 = 4 tau."""
    tau = 1.0 / f0
    t0 = 4.0 * tau
    s = t - t0
    return np.sin(2 * np.pi * f0 * s) * np.exp(-(s * s) / (2 * tau * tau))


def blackman_harris(t: np.ndarray, length: float = 0.1) -> np.ndarray:
    """The four-term Blackman-Harris window of Sec. III, stretched to the given length
    (0.1 in the paper's units), zero afterwards."""
    x = np.asarray(t, dtype=np.float64) / length
    w = (0.359 - 0.488 * np.cos(2 * np.pi * x) + 0.141 * np.cos(4 * np.pi * x)
         - 0.012 * np.cos(6 * np.pi * x))
    return np.where((x >= 0) & (x <= 1.0), w, 0.0)


def wavelet_f0(h_ref: float = 3.0 / 128) -> float:
    """Centre frequency giving 10 nodes per wavelength at spacing h_ref in eps = 4."""
    return 1.0 / (20.0 * h_ref)


def sample_wavelet(dt: float, n_steps: int, f0: float) -> np.ndarray:
    """w_l = w(l dt), l = 0 .. n_steps - 1."""
    return gaussian_sine(np.arange(n_steps, dtype=np.float64) * dt, f0)


def sample_steps(n_steps: int, n_samples: int) -> np.ndarray:
    """Evenly spread recorded steps: floor((k+1) n_steps / n_samples) - 1."""
    k = np.arange(n_samples, dtype=np.int64)
    return ((k + 1) * n_steps) // n_samples - 1


def add_peak_noise(traces: np.ndarray, level: float, seed: int) -> np.ndarray:
    """Gaussian noise with per-trace std level * max_t |y(t)| (peak-relative, Sec. III)."""
    rng = np.random.default_rng(seed)
    peak = np.max(np.abs(traces), axis=-1, keepdims=True)
    return traces + level * peak * rng.standard_normal(traces.shape)
