"""Pins of the oracle's leap-frog forward run (App. A, eqs. leap-frog1/2).

Each check is fixed by the mathematics rather than by the oracle's own formulas:
discrete energy conservation, source-receiver reciprocity, convergence to the analytic
homogeneous-medium Green's functions, an exact standing wave built from a dense
generalised eigenvector, brute-force dense propagation, and an exact time-scaling
symmetry.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import Oracle
from synth import acquisition as acq
from synth import configs
from synth.mesh import kuhn_mesh
from tests import dense_fe


def _jitter(mesh, amount, seed):
    rng = np.random.default_rng(seed)
    x = mesh.coords.copy()
    interior = np.all(np.abs(np.abs(x) - 1.5) > 1e-9, axis=1)
    x[interior] += rng.uniform(-amount, amount, size=x[interior].shape) * mesh.h
    return x


@pytest.mark.parametrize("d,N", [(2, 12), (3, 5)])
def test_energy_conserved_closed_lossless(d, N):
    """No absorbing boundary, sigma = 0, no source: the leap-frog energy
    E = 1/2 sum_T |T| |q_{l+1/2}|^2 + 1/2 p_{l+1}^T M p_l is constant."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.15, 11)
    rng = np.random.default_rng(12)
    eps = rng.uniform(1.0, 6.0, ms.m)
    o = Oracle(d, x, ms.elems, eps)
    p0 = np.exp(-8.0 * np.sum(x ** 2, axis=1)) * rng.uniform(0.5, 1.5, ms.n)
    dt = acq.time_step(d, ms.h, 1.0)
    rec = np.zeros((1, 1, d))
    energies = []
    for k in (1, 300, 1500, 3000):
        _, pl, pp, ql = o.forward(None, rec, None, dt, k, p0=p0, want_state=True)
        energies.append(0.5 * np.sum(o.vol[:, None] * ql ** 2) + 0.5 * pl @ (o.M * pp))
    e = np.array(energies)
    assert e[0] > 0
    assert np.abs(e / e[0] - 1).max() < 1e-12


@pytest.mark.parametrize("d,N", [(2, 24), (3, 8)])
def test_reciprocity(d, N):
    """Swapping source and receiver leaves the trace unchanged (heterogeneous eps,
    conductivity and absorbing boundary)."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.1, 21)
    rng = np.random.default_rng(22)
    eps = rng.uniform(1.0, 6.0, ms.m)
    sig = rng.uniform(0.0, 1.0, ms.m)
    o = Oracle(d, x, ms.elems, eps, sigma=sig, bfacets=ms.bfacets)
    a = np.array([0.31, -0.52, 0.17][:d])
    b = np.array([-0.77, 0.44, -0.09][:d])
    dt = acq.time_step(d, ms.h, 1.0)
    w = acq.gaussian_sine(np.arange(600) * dt, 1.5)
    ab = o.forward(a[None], b[None, None], w, dt, 600)[0, 0]
    ba = o.forward(b[None], a[None, None], w, dt, 600)[0, 0]
    assert np.abs(ab).max() > 1e-6
    assert np.abs(ab - ba).max() <= 1e-12 * np.abs(ab).max()


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_matches_brute_force_dense_propagation(d, N):
    """Traces equal eqs. leap-frog1/2 stepped with independently assembled dense
    matrices (distorted mesh, eps, sigma, absorbing boundary, off-node source)."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 31)
    rng = np.random.default_rng(32)
    eps, sig = rng.uniform(1, 5, ms.m), rng.uniform(0, 2, ms.m)
    o = Oracle(d, x, ms.elems, eps, sigma=sig, bfacets=ms.bfacets)
    A, B, Ml, r, K = dense_fe.assemble(x, ms.elems, eps, sig, ms.bfacets)
    src = np.array([0.23, -0.41, 0.12][:d])
    recs = np.array([[0.7, 0.3, -0.2][:d], [-1.1, 0.05, 0.9][:d]])
    dt = 0.3 * ms.h
    nst = 400
    w = acq.gaussian_sine(np.arange(nst) * dt, 0.8)
    fs = w[:, None] * dense_fe.point_weights(x, ms.elems, src)[None, :]
    rw = np.stack([dense_fe.point_weights(x, ms.elems, rr) for rr in recs])
    ref, _, _ = dense_fe.leapfrog_dense(A, B, Ml, r, dt, nst, fs, rw)
    got = o.forward(src[None], recs[None], w, dt, nst)[0]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d,N", [(2, 4), (3, 2)])
def test_standing_wave_from_dense_eigenvector(d, N):
    """Closed mesh: with K v = lambda M v, p_0 = v and q_{-1/2} = -(dt/2) grad v, the
    scheme gives p_l = cos(omega l dt) v exactly, sin(omega dt/2) = (dt/2) sqrt(lambda)."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 41)
    eps = np.random.default_rng(42).uniform(1, 4, ms.m)
    o = Oracle(d, x, ms.elems, eps)
    A, B, Ml, r, K = dense_fe.assemble(x, ms.elems, eps)
    Mh = 1.0 / np.sqrt(Ml)
    lam, W = np.linalg.eigh(Mh[:, None] * K * Mh[None, :])
    dt = 0.25 * 2.0 / np.sqrt(lam.max())
    for k in (1, len(lam) // 2, len(lam) - 1):
        v = Mh * W[:, k]
        q0 = np.stack([-(dt / 2) * (B[c] @ v) / A for c in range(d)], axis=1)
        omega = 2.0 / dt * np.arcsin(dt / 2 * np.sqrt(lam[k]))
        for steps in (1, 7, 250):
            _, pl, _, _ = o.forward(None, np.zeros((1, 1, d)), None, dt, steps, p0=v, q0=q0,
                                    want_state=True)
            assert np.abs(pl - np.cos(omega * steps * dt) * v).max() < 1e-11 * np.abs(v).max()


def test_time_scaling_symmetry_is_exact():
    """eps -> 4 eps, dt -> 2 dt, w -> 2 w, sigma -> 2 sigma, boundary admittance -> 2
    maps the discrete solution onto itself; with powers of two it is bit-exact."""
    p = configs.make("c1", N=24, L=0, n_steps=300)
    ms = p.mesh
    sig = np.where(p.eps > 1.5, 0.5, 0.0)
    o1 = Oracle(2, ms.coords, ms.elems, p.eps, sigma=sig, bfacets=ms.bfacets)
    o2 = Oracle(2, ms.coords, ms.elems, 4 * p.eps, sigma=2 * sig, bfacets=ms.bfacets,
                admittance=np.full(ms.bfacets.shape[0], 2.0))
    t1 = o1.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    t2 = o2.forward(p.src, p.rec, 2 * p.wavelet, 2 * p.dt, p.n_steps)
    assert np.array_equal(t1, t2)


def _gauss(t0, tau):
    f = lambda t: np.exp(-(t - t0) ** 2 / (2 * tau ** 2))          # noqa: E731
    df = lambda t: -(t - t0) / tau ** 2 * f(t)                      # noqa: E731
    return f, df


def test_green_function_3d_second_order():
    """eps = 1, sigma = 0: eps u_tt - Lap u = delta_p f'(t) has u = f'(t - r)/(4 pi r)
    (Sec. II-A with the first-order system's source).  The scheme injects f_l at
    t_l and advances to t_{l+1}, so p_{l+1} approximates u((l + 1/2) dt); compared
    there, before any boundary reflection arrives, the error falls as h^2."""
    f, df = _gauss(0.8, 0.2)
    xs, xr = -0.375, 0.375
    r0 = xr - xs
    errs = []
    for N in (16, 32, 64):
        ms = kuhn_mesh(3, N, 0)
        o = Oracle(3, ms.coords, ms.elems, np.ones(ms.m))
        dt = acq.time_step(3, ms.h, 1.0)
        ns = int(2.9 / dt)
        tr = o.forward(np.array([[xs, 0, 0]]), np.array([[[xr, 0, 0]]]),
                       f(np.arange(ns) * dt), dt, ns)[0, 0]
        ex = df((np.arange(ns) + 0.5) * dt - r0) / (4 * np.pi * r0)
        errs.append(np.abs(tr - ex).max() / np.abs(ex).max())
    rates = np.array(errs[:-1]) / np.array(errs[1:])
    assert errs[-1] < 0.05
    assert np.all(rates > 3.2) and np.all(rates < 5.0), (errs, rates)


def test_green_function_2d_second_order():
    """2D: u(r, t) = (1/2pi) int_0^{acosh(t/r)} f'(t - r cosh a) da (the 2D Green's
    function H(t - r)/(2 pi sqrt(t^2 - r^2)) convolved with f', singularity removed by
    t - s = r cosh a); h^2 convergence against it."""
    f, df = _gauss(0.8, 0.2)
    xs, xr = -0.375, 0.375
    r0 = xr - xs

    def exact(t):
        if t <= r0:
            return 0.0
        return quad(lambda a: df(t - r0 * np.cosh(a)), 0, np.arccosh(t / r0), limit=200,
                    epsabs=1e-13)[0] / (2 * np.pi)

    errs = []
    for N in (32, 64, 128):
        ms = kuhn_mesh(2, N, 0)
        o = Oracle(2, ms.coords, ms.elems, np.ones(ms.m))
        dt = acq.time_step(2, ms.h, 1.0)
        ns = int(2.9 / dt)
        tr = o.forward(np.array([[xs, 0]]), np.array([[[xr, 0]]]), f(np.arange(ns) * dt), dt,
                       ns)[0, 0]
        ex = np.array([exact(t) for t in (np.arange(ns) + 0.5) * dt])
        errs.append(np.abs(tr - ex).max() / np.abs(ex).max())
    rates = np.array(errs[:-1]) / np.array(errs[1:])
    assert errs[-1] < 0.01
    assert np.all(rates > 3.2) and np.all(rates < 5.0), (errs, rates)


def test_thread_count_does_not_change_results():
    """The oracle's OpenMP loops split independent rows only, so one thread and every
    thread give the same traces bit for bit (the one-core baseline times the same
    arithmetic)."""
    p = configs.make("c2", N=24, L=1, n_src=3, n_steps=200)
    o = Oracle.from_problem(p)
    threads = o.threads
    a = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    o.set_threads(1)
    try:
        assert o.threads == 1
        b = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    finally:
        o.set_threads(threads)
    assert o.threads == threads
    assert np.array_equal(a, b)
