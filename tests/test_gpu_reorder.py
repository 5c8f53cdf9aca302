"""Arbitrarily numbered meshes: the library steps in its own node order (reverse
Cuthill-McKee when the input numbering scatters neighbours) while every input and
output keeps the caller's numbering.  Checked against the oracle on a randomly
renumbered mesh for every entry point."""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def shuffled():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = configs.make("c3", N=24, L=2, n_src=2, n_steps=400, n_samples=16)
    ms = p.mesh
    perm = np.random.default_rng(7).permutation(ms.n).astype(np.int32)   # old id -> new id
    coords = np.empty_like(ms.coords)
    coords[perm] = ms.coords
    elems, bf, cv = perm[ms.elems], perm[ms.bfacets], perm[ms.coarse_verts]
    from paper_1707_04605_amd import Context
    ctx = Context(0)
    ctx.upload_mesh(2, coords, elems, bf, None, ms.coarse_of_elem, cv)
    ctx.upload_permittivity(p.eps)
    o = Oracle(2, coords, elems, p.eps, bfacets=bf, coarse_of_elem=ms.coarse_of_elem,
               coarse_verts=cv)
    return p, ctx, o


def test_forward_on_renumbered_mesh(shuffled):
    p, ctx, o = shuffled
    ref = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    for prec, tol in ((64, 1e-11), (32, 1e-4)):
        g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
        assert _rel(g, ref) <= tol


def test_jacobians_and_gradient_on_renumbered_mesh(shuffled):
    p, ctx, o = shuffled
    ss = p.sample_steps
    J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss, mode="mg", precision=64)
    assert _rel(J2, o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)) <= 1e-10
    cols = np.array([3, 40, 71])
    J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss, mode="exact",
                             cols=cols, precision=64)
    assert _rel(J1, o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, cols, ss)) <= 1e-10
    rho = np.random.default_rng(2).normal(size=(2, 1, p.n_steps))
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64)
    assert _rel(g, o.gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)) <= 1e-10
