"""Pins of the projected-data oracle (Sec. II-F): quadrature against closed-form
integrals within the rectangle rule's error bound, the travel-time ratio the paper
states, and the Jacobian of the projection against complex-step derivatives of the
projected simulated data."""
import numpy as np

from oracle import Oracle, projected as pj
from synth import acquisition as acq
from synth import configs


def test_quadrature_against_closed_forms():
    N, dt = 16000, 2e-3
    ss = acq.sample_steps(N, 512)
    q, t = pj.quadrature(ss, dt, N)
    T = N * dt
    # rectangle widths tile [0, T]
    assert abs(q[0].sum() - T) < 1e-12 * T
    assert abs(t[-1] - T) < 1e-12
    # int_0^T sin^2(w t) dt and (1/T) int t sin^2(w t) dt, right-endpoint rule: error
    # <= h/2 * total variation of the integrand
    w = 2 * np.pi * 3.3 / T
    u = np.sin(w * t)
    I1 = T / 2 - np.sin(2 * w * T) / (4 * w)
    I2 = (T ** 2 / 4 - (T * np.sin(2 * w * T) / (4 * w) + (np.cos(2 * w * T) - 1) / (8 * w ** 2))) / T
    h = T / 512
    y = pj.inner(u, u, q)
    tv1 = 2 * 3.3 * 2          # sin^2 rises and falls 2 x 3.3 times per period count
    assert abs(y[0] - I1) <= h / 2 * tv1 * 1.01
    assert abs(y[1] - I2) <= h / 2 * tv1 * 1.01
    # polynomial check: <1, t>_1 = T^2 / 2 up to the rule's O(h) bias, exactly computable
    one = np.ones_like(t)
    assert abs(pj.inner(one, t, q)[0] - np.sum(t * q[0])) == 0
    assert abs(pj.inner(one, t, q)[0] - T ** 2 / 2) <= h * T / 2 * 1.01


def test_travel_time_ratio():
    """y^(2) / y^(1) = int t u^2 / (T int u^2): the relative integrated travel time of a
    pulse, i.e. t0 / T for a narrow pulse centred at t0."""
    N, dt = 16000, 2e-3
    ss = acq.sample_steps(N, 512)
    q, t = pj.quadrature(ss, dt, N)
    T = N * dt
    for t0 in (0.25 * T, 0.5 * T, 0.8 * T):
        u = np.exp(-((t - t0) / (0.01 * T)) ** 2) * np.cos(40 * t)
        y = pj.inner(u, u, q)
        assert abs(y[1] / y[0] - t0 / T) < 2e-3


def test_projected_jacobian_is_derivative_of_projected_data():
    """d/dc_j <u, u0(c)>_k = <u, d u0/dc_j>_k: the projected J1 columns against
    complex-step derivatives of the projected simulated data (the forward run in complex
    arithmetic)."""
    p = configs.make("c3", N=16, L=1, n_src=2, n_steps=400, n_samples=40)
    o = Oracle.from_problem(p)
    ss = p.sample_steps
    q, _ = pj.quadrature(ss, p.dt, p.n_steps)
    u = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)[..., ss] * 1.1 + 0.01
    u = u.reshape(-1, ss.size)
    cols = [3, 40, 71]
    J = o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, cols, ss)
    P = pj.projected_jacobian(J, u, q)
    for k, j in enumerate(cols):
        d = np.stack([o.complex_step_column(p.src[s], p.rec[s], p.wavelet, p.dt, p.n_steps,
                                            o.coarse_direction(j))[..., ss]
                      for s in range(p.src.shape[0])])
        ref = pj.inner(u, d.reshape(-1, ss.size), q).reshape(-1)
        err = np.linalg.norm(P[:, k] - ref) / np.linalg.norm(ref)
        assert err < 1e-12, (j, err)
