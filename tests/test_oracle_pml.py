"""Pins of the oracle's split-field PML (App. A, matrices S and T^(k)) and the lossy
target: brute-force dense propagation with the T^(k) term, exact discrete reciprocity
(which the PML keeps: eliminating q leaves a symmetric operator at every frequency),
zero coefficients reduce to the closed domain, and the layer absorbs what reaches the
box surface (against a run in a domain so large that no reflection arrives)."""
import numpy as np
import pytest

from tests import dense_fe
from oracle import Oracle
from synth import acquisition as acq
from synth import configs, pml
from synth.mesh import kuhn_mesh


def _jitter(mesh, amount, seed):
    rng = np.random.default_rng(seed)
    x = mesh.coords.copy()
    interior = np.all(np.abs(x) < 1.5 - 1e-9, axis=1)
    x[interior] += amount * mesh.h * rng.uniform(-1, 1, size=(interior.sum(), mesh.d))
    return x


@pytest.mark.parametrize("d,N", [(2, 4), (3, 2)])
def test_pml_matches_brute_force_dense_propagation(d, N):
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.2, 41)
    rng = np.random.default_rng(42)
    eps, sig = rng.uniform(1, 5, ms.m), rng.uniform(0, 2, ms.m)
    xi = rng.uniform(0, 3, ms.m)
    zeta = rng.uniform(0, 3, (ms.m, d)) * (rng.uniform(size=(ms.m, d)) < 0.6)
    o = Oracle(d, x, ms.elems, eps, sigma=sig, pml=(xi, zeta))
    A, B, Ml, r, K = dense_fe.assemble(x, ms.elems, eps, sig + xi)   # S lumped like R
    T = np.stack([np.diag(zeta[:, k] * A) for k in range(d)])
    src = np.array([0.23, -0.41, 0.12][:d])
    recs = np.array([[0.7, 0.3, -0.2][:d], [-1.1, 0.05, 0.9][:d]])
    dt = 0.3 * ms.h
    nst = 400
    w = acq.gaussian_sine(np.arange(nst) * dt, 0.8)
    fs = w[:, None] * dense_fe.point_weights(x, ms.elems, src)[None, :]
    rw = np.stack([dense_fe.point_weights(x, ms.elems, rr) for rr in recs])
    ref, _, _ = dense_fe.leapfrog_dense(A, B, Ml, r, dt, nst, fs, rw, T=T)
    got = o.forward(src[None], recs[None], w, dt, nst)[0]
    assert np.abs(ref).max() > 1e-6
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the T term matters: without it the traces differ
    no_t, _, _ = dense_fe.leapfrog_dense(A, B, Ml, r, dt, nst, fs, rw)
    assert np.abs(no_t - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("d,N", [(2, 24), (3, 8)])
def test_pml_reciprocity(d, N):
    ms = kuhn_mesh(d, N, 0)
    x = _jitter(ms, 0.1, 43)
    rng = np.random.default_rng(44)
    eps = rng.uniform(1.0, 6.0, ms.m)
    cen = x[ms.elems].mean(axis=1)
    xi, zeta = pml.pml_coefficients(cen, 1.1, 1.5, 5.0)
    o = Oracle(d, x, ms.elems, eps, sigma=rng.uniform(0, 1, ms.m), pml=(xi, zeta))
    a = np.array([0.31, -0.52, 0.17][:d])
    b = np.array([-0.77, 1.24, -0.09][:d])              # b inside the layer
    dt = acq.time_step(d, ms.h, 1.0)
    w = acq.gaussian_sine(np.arange(600) * dt, 1.5)
    ab = o.forward(a[None], b[None, None], w, dt, 600)[0, 0]
    ba = o.forward(b[None], a[None, None], w, dt, 600)[0, 0]
    assert np.abs(ab).max() > 1e-6
    assert np.abs(ab - ba).max() <= 1e-12 * np.abs(ab).max()


def test_zero_coefficients_are_the_closed_domain():
    ms = kuhn_mesh(2, 16, 0)
    eps = np.full(ms.m, 2.0)
    dt = acq.time_step(2, ms.h, 2.0)
    w = acq.gaussian_sine(np.arange(300) * dt, 1.5)
    a = Oracle(2, ms.coords, ms.elems, eps).forward([[0.2, 0.1]], [[[0.5, -0.3]]], w, dt, 300)
    b = Oracle(2, ms.coords, ms.elems, eps, pml=(np.zeros(ms.m), np.zeros((ms.m, 2)))).forward(
        [[0.2, 0.1]], [[[0.5, -0.3]]], w, dt, 300)
    assert np.array_equal(a, b)


def test_layer_absorbs_the_outgoing_wave():
    """Vacuum box [-1.5, 1.5]^2 with the layer at its surface, against the same source
    and receiver in a box three times larger (no reflection arrives in the window): the
    PML run stays close to it, the closed box does not."""
    N, T_steps = 64, 700
    ms = kuhn_mesh(2, N, 0)
    eps = np.ones(ms.m)
    dt = acq.time_step(2, ms.h, 1.0)
    f0 = 4.0
    w = acq.gaussian_sine(np.arange(T_steps) * dt, f0)
    src, rec = np.array([[0.9, 0.3]]), np.array([[[1.1, -0.2]]])
    big = kuhn_mesh(2, 3 * N, 0)
    bx = big.coords * 3.0                                # [-4.5, 4.5]^2, same spacing
    ref = Oracle(2, bx, big.elems, np.ones(big.m)).forward(src, rec, w, dt, T_steps)[0, 0]
    closed = Oracle(2, ms.coords, ms.elems, eps).forward(src, rec, w, dt, T_steps)[0, 0]
    xi, zeta = pml.pml_coefficients(ms.centroids, 1.25, 1.5, 40.0)
    lay = Oracle(2, ms.coords, ms.elems, eps, pml=(xi, zeta)).forward(src, rec, w, dt,
                                                                      T_steps)[0, 0]
    e_closed = np.linalg.norm(closed - ref) / np.linalg.norm(ref)
    e_pml = np.linalg.norm(lay - ref) / np.linalg.norm(ref)
    print(f"reflection: closed box {e_closed:.3f}, PML {e_pml:.3f}")
    assert e_closed > 0.3 and e_pml < 0.25 * e_closed


def test_pml_workload_inputs():
    p = configs.make("c1", pml=True, N=32, L=1, n_steps=10)
    xi, zeta = p.pml
    assert p.sigma is not None and p.sigma.max() > 0
    inside = p.body.inside(p.mesh.centroids)
    np.testing.assert_array_equal(p.sigma[inside], 5 * p.eps[inside])
    assert not p.sigma[~inside].any()
    a = np.abs(p.mesh.centroids)
    assert np.all(xi[a.max(axis=1) >= pml.RHO1] == pml.VARSIGMA)
    assert not xi[a.max(axis=1) < pml.RHO1].any()
    # the layer is outside the sources
    assert np.all(np.abs(p.src).max(axis=1) < pml.RHO1)
    # the explicit q damping factor 1 - dt zeta stays in (0.5, 1) at every full-size
    # workload's time step (vacuum, the smallest permittivity)
    for name, spec in configs.SPECS.items():
        dt = acq.time_step(spec["d"], 3.0 / spec["N"], 1.0)
        assert pml.VARSIGMA * dt < 0.5, name
