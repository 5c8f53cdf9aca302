"""GPU parity with the split-field PML and the lossy target (App. A S and T^(k), Sec. III
sigma = 5 eps_r) against the mixed-form oracle: forward traces in 2D and 3D, both
precisions, batched with a ragged last batch; J2 and J1; the checkpointed misfit
gradient (its q state is checkpointed with p); upload order; the plain stepper's error.

Tolerances as without a layer: FP64 traces 1e-11, Jacobians and gradients 1e-10; FP32
traces 1e-4."""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs, pml

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


def _p2d(**over):
    # 64^2 cells: the default layer [1.42, 1.5] is about two cells thick, dt zeta = 0.65
    kw = dict(N=64, L=2, n_src=5, n_steps=900)
    kw.update(over)
    return configs.make("c1", pml=True, **kw)


def _p3d(**over):
    kw = dict(N=12, L=1, n_src=3, n_steps=250)
    kw.update(over)
    p = configs.make("c5", pml=True, **kw)
    # a thicker, weaker layer resolved by the coarse 3D test mesh (dt zeta = 0.35)
    p.pml = pml.pml_coefficients(p.mesh.centroids, 1.0, 1.5, 5.0)
    return p


@pytest.mark.parametrize("prec,tol,batch", [(64, 1e-11, 4), (32, 1e-4, 4), (64, 1e-11, 0)])
def test_pml_forward_2d(mgrt, prec, tol, batch):
    p = _p2d()
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec, batch=batch)
    err = _rel(g, ref)
    print(f"PML 2D forward fp{prec} batch {batch}: {err:.2e}")
    assert err <= tol
    # the layer and the losses matter: the same run without them differs
    noabs = Oracle(p.mesh.d, p.mesh.coords, p.mesh.elems, p.eps).forward(
        p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    assert _rel(noabs, ref) > 1e-2


def test_pml_launch_variants(mgrt):
    """The layer load and the adjoint correlation in the XCD-ordered non-temporal launch
    and the linear plain one (forced): the same traces and gradient."""
    p = _p2d(n_src=3, n_steps=300)
    ctx = mgrt.context_for_problem(p)
    a = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64, launch=1)
    for v in (4, 6, 8, 14, 16):
        b = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64, launch=v)
        assert np.array_equal(a, b), v
    rho = np.random.default_rng(3).normal(size=a.shape)
    ref = Oracle.from_problem(p).gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)
    ga = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64,
                             launch=1)
    assert _rel(ga, ref) <= 1e-10
    for v in (4, 8, 16):
        gb = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64,
                                 launch=v)
        assert np.array_equal(ga, gb), v
    # FP32 packed records in linear and XCD-contiguous order
    a32 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32, launch=6)
    b32 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32, launch=8)
    assert np.array_equal(a32, b32)


def test_pml_forward_3d_bistatic(mgrt):
    p = _p3d()
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    err = _rel(g, ref)
    print(f"PML 3D forward fp64: {err:.2e}")
    assert err <= 1e-11


def test_pml_upload_order_and_removal(mgrt):
    p = _p2d(n_src=2, n_steps=400)
    ctx = mgrt.context_for_problem(p)
    a = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    # layer first, permittivity afterwards
    ms = p.mesh
    c2 = mgrt.Context(0)
    c2.upload_mesh(ms.d, ms.coords, ms.elems, None, None, ms.coarse_of_elem, ms.coarse_verts)
    c2.upload_pml(*p.pml)
    c2.upload_permittivity(p.eps, p.sigma)
    b = c2.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    assert _rel(b, a) <= 1e-14
    # removing the layer gives the closed lossy domain
    c2.upload_pml(None, None)
    c = c2.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    ref = Oracle(ms.d, ms.coords, ms.elems, p.eps, sigma=p.sigma).forward(
        p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    assert _rel(c, ref) <= 1e-11 and _rel(c, a) > 1e-3


def test_pml_plain_stepper_rejected(mgrt):
    from paper_1707_04605_amd import MgrtError
    p = _p2d(n_src=1, n_steps=10)
    ctx = mgrt.context_for_problem(p)
    with pytest.raises(MgrtError) as ei:
        ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64,
                           variant="plain")
    assert ei.value.name == "MGRT_E_ARG"


def test_pml_jacobians_2d(mgrt):
    p = configs.make("c3", pml=True, N=64, L=3, n_src=2, n_steps=500, n_samples=20)
    o = Oracle.from_problem(p)
    ss = p.sample_steps
    ctx = mgrt.context_for_problem(p)
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)
    J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss, mode="mg",
                             precision=64)
    e2 = _rel(J2, ref)
    cols = np.array([0, 17, 63, 100, 127])
    ref1 = o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, cols, ss)
    J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss, mode="exact",
                             cols=cols, precision=64)
    e1 = _rel(J1, ref1)
    print(f"PML J2 {e2:.2e}, J1 {e1:.2e}")
    assert e2 <= 1e-10 and e1 <= 1e-10


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_pml_misfit_gradient(mgrt, case):
    p = _p2d(n_src=2, n_steps=400) if case == "2d" else _p3d(n_steps=200)
    o = Oracle.from_problem(p)
    rho = np.random.default_rng(9).normal(size=(p.src.shape[0], p.rec.shape[1], p.n_steps))
    ref = o.gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)
    ctx = mgrt.context_for_problem(p)
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64)
    b_full = ctx.last_timing()["batch"]
    err = _rel(g, ref)
    # fewer sources per sweep under a small budget (q checkpoints included in the plan):
    # the same gradient
    g1 = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64,
                             mem_budget_gb=0.003)
    b_small = ctx.last_timing()["batch"]
    print(f"PML gradient {case}: {err:.2e}; budget plan {_rel(g1, g):.1e} "
          f"(batch {b_full} -> {b_small})")
    assert err <= 1e-10 and _rel(g1, g) <= 1e-13
    assert b_small < b_full
