"""Pins of the oracle's linearisation (Sec. II-B eqs. approx_1/approx_2, App. A-1/A-3).

J1 (exact restricted Jacobian) is checked against two routes that share none of its
tangent-linear code: a complex-step forward run and central finite differences of the
forward run.  J2 (multigrid Jacobian) must coincide with J1 when the coarse level is the
fine mesh itself.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs


@pytest.fixture(scope="module")
def small():
    p = configs.make("c1", N=24, L=2, n_steps=500, n_src=2, n_samples=25)
    o = Oracle.from_problem(p)
    return p, o


def test_tangent_matches_complex_step(small):
    p, o = small
    for j in (3, 17):
        tl = o.tangent(p.src[:1], p.rec[:1], p.wavelet, p.dt, p.n_steps,
                       [o.coarse_direction(j)])[0, 0]
        cs = o.complex_step_column(p.src[0], p.rec[0], p.wavelet, p.dt, p.n_steps,
                                   o.coarse_direction(j))
        assert np.abs(tl).max() > 0
        assert np.abs(tl - cs).max() <= 1e-12 * np.abs(cs).max()


def test_tangent_matches_central_differences(small):
    p, o = small
    h = 1e-5
    for j in (5, 30):
        dirv = o.coarse_direction(j)
        tl = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, [dirv])[:, 0]
        op = Oracle.from_problem(p, eps=p.eps + h * dirv)
        om = Oracle.from_problem(p, eps=p.eps - h * dirv)
        fd = (op.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
              - om.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)) / (2 * h)
        assert np.linalg.norm(tl - fd) <= 1e-7 * np.linalg.norm(tl)


def test_multigrid_jacobian_equals_exact_at_depth_zero():
    """With T' = T (no refinement between levels) the d+1 coarse vertices are all the
    nodes of the element, so approx_2 reduces to approx_1."""
    p = configs.make("c1", N=6, L=0, n_steps=200, n_src=2, n_samples=10)
    o = Oracle.from_problem(p)
    ss = p.sample_steps
    M = p.mesh.n_coarse
    J1 = o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, np.arange(M), ss)
    J2 = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)
    assert J1.shape == J2.shape == (2 * 1 * 10, M)
    assert np.abs(J1 - J2).max() <= 1e-12 * np.abs(J1).max()


def test_multigrid_jacobian_is_an_approximation_at_depth_one():
    """At depth >= 1 J2 only approximates J1 (its quality is the paper's approximation
    and is not pinned): same scale, not equal."""
    p = configs.make("c1", N=32, L=2, n_steps=400, n_src=1, n_samples=20)
    o = Oracle.from_problem(p)
    ss = p.sample_steps
    M = p.mesh.n_coarse
    J1 = o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, np.arange(M), ss)
    J2 = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)
    rel = np.linalg.norm(J1 - J2) / np.linalg.norm(J1)
    assert 1e-6 < rel < 3.0


def test_gradient_is_transpose_of_tangent(small):
    """<J1 v, rho> = <v, J1^T rho> with J1^T rho from the oracle's gradient routine."""
    p, o = small
    rng = np.random.default_rng(9)
    rho = rng.normal(size=(p.src.shape[0], 1, p.n_steps))
    g = o.gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)
    v = rng.normal(size=p.mesh.n_coarse)
    dv = v[p.mesh.coarse_of_elem]
    jv = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, [dv])[:, 0]
    assert np.sum(jv * rho) == pytest.approx(g @ v, rel=1e-12)
