"""3D (Kuhn tetrahedra) checks against the oracle at large sizes.

* The 128^3-cell batched forward (2,146,689 nodes, 32 sources, FP32) in the launch
  configuration the benchmark times, source 0 compared over all 6,000 steps.
* The 256^3-cell gradient over all 12,000 steps: FP32 against FP64, and against the
  forward tangent columns.
* The misfit gradient on a 32^3 mesh with an 8^3 coarse level and bistatic receivers:
  sampled coarse columns against the oracle's J1^T rho.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def mgrt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_04605_amd as m
    return m


def test_c4_full_size_forward_full_length(mgrt):
    """The 128^3-cell batched forward (2,146,689 nodes, 32 sources, FP32) in the launch
    configuration the benchmark times, source 0 against the oracle over all 6,000 steps."""
    p = configs.make("c4")
    ctx = mgrt.context_for_problem(p)
    nst = p.n_steps
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, nst, precision=32)
    t = ctx.last_timing()
    assert t["batch"] in [b for b in t["tune_b"] if b > 0] and t["graph_steps"] > 0
    ref = Oracle.from_problem(p).forward(p.src[:1], p.rec[:1], p.wavelet, p.dt, nst)
    err = _rel(g[:1], ref)
    print(f"c4 full size, source 0, {nst} steps (batch {t['batch']}): fp32 rel L2 {err:.2e}")
    assert err <= 1e-4


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_3d_bistatic_gradient_sampled_columns(mgrt, prec, tol):
    p = configs.make("c5", N=32, L=2, n_src=2, n_steps=300)
    ctx = mgrt.context_for_problem(p)
    rho = np.random.default_rng(11).normal(size=(2, 2, p.n_steps))
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=prec)
    o = Oracle.from_problem(p)
    cols = np.array([5, 777, 1500, 2222, 3000])
    dirs = [o.coarse_direction(j) for j in cols]
    tl = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, dirs)
    ref = np.einsum("scrn,srn->c", tl, rho)
    err = _rel(g[cols], ref)
    print(f"3d gradient prec={prec}, sampled columns: {err:.2e}")
    assert err <= tol


@pytest.fixture(scope="module")
def morton3d():
    """65^3 nodes: the lexicographic numbering puts z neighbours a 4,225-node plane apart,
    so the library steps in its Morton order (a far fraction of stiffness references
    about 0.06 against 0.57); every input and output keeps the caller's numbering."""
    p = configs.make("c5", N=64, L=3, n_src=1, n_steps=60, n_samples=4)
    return p, Oracle.from_problem(p)


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_3d_morton_order_forward(mgrt, morton3d, prec, tol):
    p, o = morton3d
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    ref = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    err = _rel(g, ref)
    print(f"3d 65^3 nodes forward prec={prec}: {err:.2e}")
    assert err <= tol


def test_3d_morton_order_gradient_and_jacobian(mgrt, morton3d):
    """Sampled coarse columns (the oracle runs one tangent or auxiliary solve per column
    or vertex): the gradient against J1^T rho, J2 against the oracle's J2."""
    p, o = morton3d
    ctx = mgrt.context_for_problem(p)
    rho = np.random.default_rng(29).normal(size=(1, 2, p.n_steps))
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64)
    cols = np.array([5, 1500, 3000])
    tl = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, [o.coarse_direction(j) for j in cols])
    ref = np.einsum("scrn,srn->c", tl, rho)
    err = _rel(g[cols], ref)
    print(f"3d 65^3 nodes gradient, sampled columns: {err:.2e}")
    assert err <= 1e-10
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=64)
    # the two coarse elements nearest the source (the field reaches them within the run)
    cent = p.mesh.coords[p.mesh.coarse_verts].mean(axis=1)
    jc = np.sort(np.argsort(np.linalg.norm(cent - p.src[0], axis=1))[:2])
    Jr = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps, cols=jc)
    assert np.linalg.norm(Jr) > 0
    err = _rel(J[:, jc], Jr)
    print(f"3d 65^3 nodes J2, sampled columns: {err:.2e}")
    assert err <= 1e-10


@pytest.fixture(scope="module")
def c5_fp32(mgrt):
    """The 256^3-cell bistatic gradient (16,974,593 nodes, 16 sources x 2 receivers, 32^3
    coarse level, all 12,000 steps) in the benchmark's FP32 configuration."""
    p = configs.make("c5")
    ctx = mgrt.context_for_problem(p)
    rho = np.random.default_rng(5).normal(size=(p.src.shape[0], 2, p.n_steps)) * 1e-3
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, level="coarse",
                            precision=32)
    return p, ctx, rho, g, ctx.last_timing()["batch"]


def test_c5_full_size_gradient_plan(c5_fp32):
    """The checkpointed adjoint's memory plan takes the 16 sources in several passes."""
    p, _, _, g, b32 = c5_fp32
    print(f"c5 full size: fp32 gradient with batch {b32}")
    assert b32 < p.src.shape[0] and np.isfinite(g).all() and np.abs(g).max() > 0


def test_c5_full_size_gradient_fp32_vs_fp64(c5_fp32):
    """Too large for the oracle: the FP32 gradient against the same call with FP64 fields
    (its own memory plan, FP64 sums) bounds the FP32 error over all 12,000 steps."""
    p, ctx, rho, g, b32 = c5_fp32
    g64 = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, level="coarse",
                              precision=64)
    e64 = _rel(g, g64)
    print(f"c5 full size, {p.n_steps} steps: fp32 (batch {b32}) vs fp64 (batch "
          f"{ctx.last_timing()['batch']}) gradient {e64:.2e}")
    assert e64 <= 1e-4


def test_c5_full_size_gradient_matches_tangent_columns(c5_fp32):
    """A property that holds at any size: for a coarse column j the adjoint gradient equals
    sum_{s,r,l} rho[s,r,l] J1[(s,r,l), j], with J1 from the forward tangent system (EXACT
    mode, an independent code path), on the three columns next to the first source."""
    p, ctx, rho, g, _ = c5_fp32
    N = p.n_steps
    cent = p.mesh.coords[p.mesh.coarse_verts].mean(axis=1)
    cols = np.sort(np.argsort(np.linalg.norm(cent - p.src[0], axis=1))[:3])
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, N, np.arange(N), mode="exact",
                            cols=cols, precision=32)
    ref = np.einsum("rc,r->c", J, rho.reshape(-1))
    err = _rel(g[cols], ref)
    print(f"c5 full size: adjoint gradient vs tangent columns {cols.tolist()}: {err:.2e}")
    assert np.abs(ref).max() > 0
    assert err <= 1e-4
