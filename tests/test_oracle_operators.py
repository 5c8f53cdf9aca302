"""Pins of the oracle's operators (App. A matrices) against closed forms and invariants."""
import numpy as np
import pytest

from oracle import Oracle
from synth import acquisition as acq
from synth.mesh import kuhn_mesh
from tests import dense_fe


def _jitter(mesh, amount, seed):
    """Move interior nodes randomly (keeps the mesh valid for amount < 0.25 h)."""
    rng = np.random.default_rng(seed)
    x = mesh.coords.copy()
    interior = np.all(np.abs(np.abs(x) - 1.5) > 1e-9, axis=1)
    x[interior] += rng.uniform(-amount, amount, size=x[interior].shape) * mesh.h
    return x


@pytest.mark.parametrize("d,N", [(2, 8), (3, 4)])
def test_volumes_and_boundary_measure(d, N):
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 1)
    o = Oracle(d, x, ms.elems, np.ones(ms.m), bfacets=ms.bfacets)
    assert o.vol.min() > 0
    assert o.vol.sum() == pytest.approx(3.0 ** d, rel=1e-13)
    # lumped boundary term with Y = 1 sums to the box surface measure
    assert o.r.sum() == pytest.approx(2 * d * 3.0 ** (d - 1), rel=1e-13)


def test_lumped_mass_closed_form_2d():
    """Uniform "/" mesh, eps = 1: M = h^2 inside, h^2/2 on edges, h^2/3 and h^2/6 at the
    corners (the two corners on the cut diagonal own two triangles)."""
    N = 8
    ms = kuhn_mesh(2, N, 0)
    o = Oracle(2, ms.coords, ms.elems, np.ones(ms.m))
    h2 = ms.h ** 2
    Mg = o.M.reshape(N + 1, N + 1)
    assert np.allclose(Mg[1:-1, 1:-1], h2, rtol=1e-14)
    assert np.allclose(Mg[0, 1:-1], h2 / 2, rtol=1e-14)
    assert np.allclose(Mg[1:-1, 0], h2 / 2, rtol=1e-14)
    corners = np.array([Mg[0, 0], Mg[-1, -1], Mg[0, -1], Mg[-1, 0]]) / h2
    assert np.allclose(np.sort(corners), [1 / 6, 1 / 6, 1 / 3, 1 / 3], rtol=1e-13)


def test_lumped_mass_total_weighted():
    ms = kuhn_mesh(3, 4, 0)
    rng = np.random.default_rng(5)
    eps = rng.uniform(1, 6, ms.m)
    o = Oracle(3, _jitter(ms, 0.2, 2), ms.elems, eps)
    assert o.M.sum() == pytest.approx(np.sum(eps * o.vol), rel=1e-13)
    # interior nodes of the uniform cube mesh, eps = 1: M = h^3
    o1 = Oracle(3, ms.coords, ms.elems, np.ones(ms.m))
    Mg = o1.M.reshape(5, 5, 5)
    assert np.allclose(Mg[1:-1, 1:-1, 1:-1], ms.h ** 3, rtol=1e-14)


def test_stiffness_is_five_point_laplacian_2d():
    """On the "/" mesh K is the textbook 5-point stencil (4, -1, -1, -1, -1) inside."""
    N = 10
    ms = kuhn_mesh(2, N, 0)
    o = Oracle(2, ms.coords, ms.elems, np.ones(ms.m))
    p = np.random.default_rng(0).normal(size=ms.n)
    P = p.reshape(N + 1, N + 1)
    lap = 4 * P[1:-1, 1:-1] - P[2:, 1:-1] - P[:-2, 1:-1] - P[1:-1, 2:] - P[1:-1, :-2]
    Kp = o.apply_stiffness(p).reshape(N + 1, N + 1)
    assert np.allclose(Kp[1:-1, 1:-1], lap, rtol=0, atol=1e-12)


def test_stiffness_is_seven_point_laplacian_3d():
    """On the Kuhn cube mesh K/h is the textbook 7-point stencil (6, -1 x 6) inside."""
    N = 6
    ms = kuhn_mesh(3, N, 0)
    o = Oracle(3, ms.coords, ms.elems, np.ones(ms.m))
    p = np.random.default_rng(1).normal(size=ms.n)
    P = p.reshape(N + 1, N + 1, N + 1)
    c = P[1:-1, 1:-1, 1:-1]
    lap = (6 * c - P[2:, 1:-1, 1:-1] - P[:-2, 1:-1, 1:-1] - P[1:-1, 2:, 1:-1]
           - P[1:-1, :-2, 1:-1] - P[1:-1, 1:-1, 2:] - P[1:-1, 1:-1, :-2])
    Kp = o.apply_stiffness(p).reshape(N + 1, N + 1, N + 1)
    assert np.allclose(Kp[1:-1, 1:-1, 1:-1], ms.h * lap, rtol=0, atol=1e-12)


@pytest.mark.parametrize("d,N", [(2, 7), (3, 4)])
def test_stiffness_invariants_on_distorted_mesh(d, N):
    """K 1 = 0, K symmetric, and K annihilates linear functions at interior nodes."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 3)
    o = Oracle(d, x, ms.elems, np.ones(ms.m))
    assert np.abs(o.apply_stiffness(np.ones(ms.n))).max() < 1e-13
    rng = np.random.default_rng(4)
    u, v = rng.normal(size=ms.n), rng.normal(size=ms.n)
    assert u @ o.apply_stiffness(v) == pytest.approx(v @ o.apply_stiffness(u), rel=1e-12)
    lin = x @ np.array([0.3, -1.1, 0.7][:d]) + 0.25
    interior = np.all(np.abs(np.abs(ms.coords) - 1.5) > 1e-9, axis=1)
    assert np.abs(o.apply_stiffness(lin)[interior]).max() < 1e-12


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_operators_match_dense_assembly(d, N):
    """Oracle mass, damping and stiffness equal an independent dense assembly."""
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 7)
    rng = np.random.default_rng(8)
    eps, sig = rng.uniform(1, 5, ms.m), rng.uniform(0, 2, ms.m)
    o = Oracle(d, x, ms.elems, eps, sigma=sig, bfacets=ms.bfacets)
    A, B, Ml, r, K = dense_fe.assemble(x, ms.elems, eps, sig, ms.bfacets)
    assert np.allclose(o.vol, A, rtol=1e-13)
    assert np.allclose(o.M, Ml, rtol=1e-13)
    assert np.allclose(o.r, r, rtol=1e-13)
    Ko = np.stack([o.apply_stiffness(e) for e in np.eye(ms.n)], axis=1)
    assert np.allclose(Ko, K, rtol=0, atol=1e-12 * np.abs(K).max())


def test_locate_reproduces_point():
    ms = kuhn_mesh(2, 16, 0)
    o = Oracle(2, ms.coords, ms.elems, np.ones(ms.m))
    pts = acq.circle_points(7)
    nodes, w = o.locate(pts)
    assert np.all(w >= -1e-12)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(np.einsum("pa,pak->pk", w, ms.coords[nodes]), pts, atol=1e-13)


@pytest.mark.parametrize("d,Ns", [(2, (8, 24)), (3, (8, 16))])
def test_time_step_recipe_is_half_cfl(d, Ns):
    """dt = COURANT h sqrt(eps_min) lies at (just under) half the leap-frog limit
    2 / sqrt(lambda_max(M^-1 K)) -- checked by power iteration, and the power
    iteration itself against a dense eigen-solve of an independent assembly."""
    for N in Ns:
        ms = kuhn_mesh(d, N, 0)
        o = Oracle(d, ms.coords, ms.elems, np.ones(ms.m))
        lam = o.lambda_max(3000)
        ratio = acq.time_step(d, ms.h, 1.0) / (2.0 / np.sqrt(lam))
        assert 0.47 < ratio <= 0.5
    ms = kuhn_mesh(d, Ns[0] if d == 2 else 3, 0)
    o = Oracle(d, ms.coords, ms.elems, np.ones(ms.m))
    _, _, Ml, _, K = dense_fe.assemble(ms.coords, ms.elems, np.ones(ms.m))
    ev = np.linalg.eigvalsh(K / np.sqrt(np.outer(Ml, Ml)))
    assert o.lambda_max(5000) == pytest.approx(ev.max(), rel=1e-4)
