"""GPU parity of mgrt_project_rows (projected data and projected Jacobian rows, Sec. II-F)
against the FP64 oracle: random row blocks in both precisions, host and device input,
one to eight projections, a ragged column count; projected data through the same call;
the projection of a GPU multigrid Jacobian against the oracle's projection of the oracle
Jacobian."""
import numpy as np
import pytest

from oracle import Oracle, projected as pj
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


# M = 1000: 16-byte loads over 4 (FP32) or 8 (FP64) column tiles with a ragged last tile;
# M = 999: rows too short for 16-byte alignment, the scalar kernel; ns = 1100: three chunks
# of staged weights, the last one ragged
@pytest.mark.parametrize("prec,n_proj,on_dev,M,ns", [
    (64, 2, False, 1000, 37), (32, 2, False, 1000, 37), (64, 5, True, 1000, 37),
    (32, 1, True, 1000, 37), (64, 8, False, 1000, 37), (32, 2, False, 999, 37),
    (64, 3, True, 999, 37), (32, 2, True, 1000, 1100), (64, 8, False, 1000, 1100)])
def test_project_rows_random(mgrt, prec, n_proj, on_dev, M, ns):
    rng = np.random.default_rng(11)
    nt = 5
    J = rng.normal(size=(nt * ns, M))
    if prec == 32:
        J = J.astype(np.float32)
    u = rng.normal(size=(nt, ns))
    q = rng.uniform(0.1, 1.0, size=(n_proj, ns))
    ref = pj.projected_jacobian(J.astype(np.float64), u, q)
    ctx = mgrt.Context(0)
    Jin = J
    if on_dev:
        import torch
        Jin = torch.from_numpy(J).cuda()
    P = ctx.project_rows(Jin, u, q)
    err = _rel(P, ref)
    print(f"project_rows fp{prec} n_proj={n_proj} device={on_dev} M={M} ns={ns}: {err:.2e}")
    assert P.shape == ref.shape and err <= 1e-13


def test_projected_data_and_weights(mgrt):
    p = configs.make("c3", N=16, L=1, n_src=3, n_steps=600, n_samples=50)
    ss = p.sample_steps
    q, _ = pj.quadrature(ss, p.dt, p.n_steps)
    # the library's weights (mgrt_projection_weights) against the oracle's quadrature
    np.testing.assert_allclose(mgrt.projection_weights(ss, p.dt, p.n_steps), q, rtol=1e-15)
    from paper_1707_04605_amd import MgrtError
    for bad in ((ss[::-1], p.dt, p.n_steps), (ss, -p.dt, p.n_steps), (ss, p.dt, int(ss[-1])),
                (np.array([-1]), p.dt, p.n_steps)):
        with pytest.raises(MgrtError):
            mgrt.projection_weights(*bad)
    o = Oracle.from_problem(p)
    u0 = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)[..., ss].reshape(-1, ss.size)
    rng = np.random.default_rng(2)
    u = 1.05 * u0 + 0.01 * np.abs(u0).max() * rng.normal(size=u0.shape)
    y_ref, y0_ref = pj.projected_data(u, u0, q)
    ctx = mgrt.Context(0)
    y0 = ctx.project_rows(u0.reshape(-1, 1), u, q).reshape(-1, 2)
    y = ctx.project_rows(u.reshape(-1, 1), u, q).reshape(-1, 2)
    assert _rel(y0, y0_ref) <= 1e-14 and _rel(y, y_ref) <= 1e-14


def test_projected_multigrid_jacobian(mgrt):
    p = configs.make("c3", N=32, L=2, n_src=3, n_steps=700, n_samples=24)
    ss = p.sample_steps
    o = Oracle.from_problem(p)
    Jref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)
    u = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)[..., ss].reshape(-1, ss.size)
    q = mgrt.projection_weights(ss, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss, mode="mg",
                            precision=64)
    P = ctx.project_rows(J, u, q)
    err = _rel(P, pj.projected_jacobian(Jref, u, q))
    print(f"projected J2 (FP64 fields): {err:.2e}")
    assert err <= 1e-10


def test_project_rows_rejects_bad_sizes(mgrt):
    from paper_1707_04605_amd import MgrtError
    ctx = mgrt.Context(0)
    with pytest.raises(MgrtError) as ei:
        ctx.project_rows(np.zeros((6, 3)), np.zeros((2, 3)), np.ones((9, 3)))
    assert ei.value.name == "MGRT_E_ARG"


def test_projected_tv_step(mgrt):
    """The TV step on projected data (alpha = 1e-7, beta = 1; 6 rows, 128 columns: the
    low-rank preconditioned path) against the dense oracle, per step, to
    max(1e-9, 10 cond(A) cg_rtol): CG stops on the residual, so the error bound scales
    with the condition number of that step's matrix A."""
    from oracle import tv
    from synth import regularizer
    p = configs.make("c3", N=32, L=2, n_src=3, n_steps=700, n_samples=24)
    ss = p.sample_steps
    o = Oracle.from_problem(p)
    J = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, ss)
    u0 = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)[..., ss].reshape(-1, ss.size)
    rng = np.random.default_rng(6)
    u = 1.05 * u0 + 0.01 * np.abs(u0).max() * rng.normal(size=u0.shape)
    q = mgrt.projection_weights(ss, p.dt, p.n_steps)
    P = pj.projected_jacobian(J, u, q)
    y, y0 = pj.projected_data(u, u0, q)
    r = (y - y0).reshape(-1)
    M = P.shape[1]
    rp, col, val = regularizer.tv_matrix(p.mesh.coords, p.mesh.coarse_verts, 1.0)
    D = regularizer.csr_to_dense(rp, col, val, M)
    alpha, rtol = 1e-7, 1e-12
    ref = tv.tv_iterates(P, r, D, alpha, 3)
    ctx = mgrt.Context(0)
    z, its = ctx.tv_invert_level(P, r, rp, col, val, alpha, iters=3, cg_rtol=rtol,
                                 cg_maxit=5000)
    for l in range(3):
        if l == 0:
            g = np.ones(M)
        else:
            a = np.abs(D @ ref[l - 1]); g = 1 / np.maximum(a, 1e-8 * a.max())
        A = P.T @ P + alpha * D.T @ (g[:, None] * D)
        tol = max(1e-9, 10 * np.linalg.cond(A) * rtol)
        err = _rel(z[l], ref[l])
        print(f"projected TV step {l}: {err:.2e} (tol {tol:.1e}), CG {its[l]}")
        assert err <= tol and its[l] < 5000
