"""Pins of the regularised-deconvolution oracle (App. A-2): exact recovery of a decayed
impulse response at delta = 0, the delta -> infinity limit (a scaled cross-correlation),
and the whole route against the reciprocity Jacobian J2 (eq. approx_2) on a lossy mesh
whose responses die out inside the window, with a source function whose spectrum has no
zeros."""
import numpy as np

from oracle import Oracle, deconv
from synth import configs


def test_delta_zero_recovers_decayed_response():
    rng = np.random.default_rng(1)
    N = 600
    lam = np.exp(-np.arange(N) / 12.0) * rng.normal(size=N)       # e^-50 at the end
    f = 0.6 ** np.arange(N)                                        # F has no zeros
    p = np.convolve(lam, f)[:N]
    g = deconv.tikhonov_deconvolve(p, f, 0.0)
    assert np.abs(g - lam).max() <= 1e-10 * np.abs(lam).max()


def test_large_delta_is_scaled_cross_correlation():
    rng = np.random.default_rng(2)
    N = 300
    f = rng.normal(size=N) * np.exp(-np.arange(N) / 30.0)
    p = rng.normal(size=N)
    delta = 1e12
    F = np.fft.rfft(f, n=deconv.pad_length(N))
    g = deconv.tikhonov_deconvolve(p, f, delta) * delta * (np.abs(F) ** 2).max()
    # sum_m f(m) p(l + m), l = 0..N-1 (p zero beyond the window)
    xc = np.array([np.dot(f[:N - l], p[l:]) for l in range(N)])
    assert np.abs(g - xc).max() <= 1e-9 * np.abs(xc).max()


def test_route_equals_reciprocity_jacobian_when_responses_decay():
    p = configs.make("c3", N=16, L=1, n_src=2, n_steps=700, n_samples=30)
    sigma = np.full(p.mesh.m, 8.0)
    f = 0.6 ** np.arange(p.n_steps)
    o = Oracle(p.mesh.d, p.mesh.coords, p.mesh.elems, p.eps, sigma=sigma,
               bfacets=p.mesh.bfacets, coarse_of_elem=p.mesh.coarse_of_elem,
               coarse_verts=p.mesh.coarse_verts)
    ss = p.sample_steps
    J2 = o.jacobian_mg(p.src, p.rec, f, p.dt, p.n_steps, ss)
    Jd = deconv.jacobian_deconv(o, p.src, p.rec, f, p.dt, p.n_steps, ss, 0.0)
    err = np.linalg.norm(Jd - J2) / np.linalg.norm(J2)
    print(f"deconvolution route vs J2 at delta = 0: {err:.2e}")
    assert err <= 1e-9
    # regularisation moves it away
    Jr = deconv.jacobian_deconv(o, p.src, p.rec, f, p.dt, p.n_steps, ss, 1e-2)
    assert np.linalg.norm(Jr - J2) / np.linalg.norm(J2) > 1e-4
