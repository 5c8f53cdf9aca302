"""GPU parity of the linearisation entry points against the FP64 oracle:
mgrt_jacobian_coarse (MG = eq. approx_2, EXACT = eq. approx_1), mgrt_misfit_gradient
(J1^T rho) and mgrt_tv_invert_level (eq. tv_iteration).

Tolerances: FP64 wave fields <= 1e-10 relative Frobenius, FP32 <= 1e-4.
"""
import numpy as np
import pytest

from oracle import Oracle, tv
from synth import configs, regularizer

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


@pytest.fixture(scope="module")
def small2d():
    p = configs.make("c3", N=32, L=2, n_src=3, n_steps=700, n_samples=24)
    return p, Oracle.from_problem(p)


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_multigrid_jacobian_2d(mgrt, small2d, prec, tol):
    p, o = small2d
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=prec)
    err = _rel(J, ref)
    print(f"J2 2D prec={prec}: {err:.2e}")
    assert J.shape == ref.shape == (3 * 24, p.mesh.n_coarse)
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
@pytest.mark.parametrize("pairing", ["split", "direct"])
def test_multigrid_jacobian_pairings(mgrt, small2d, prec, tol, pairing):
    """Both pairings of the reciprocity route give the oracle's J2: the physical source
    runs with unit-impulse receiver runs, and the wavelet split exactly between the two
    (w = w1 * w2).  The library reports which one ran.  On this coarse mesh the wavelet
    reaches the grid scale, so the automatic choice pairs directly in both precisions."""
    p, o = small2d
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=prec, pairing=pairing)
    assert ctx.last_timing()["jac_split"] == (pairing == "split")
    err = _rel(J, ref)
    print(f"J2 2D prec={prec} {pairing}: {err:.2e}")
    assert err <= tol
    ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps, mode="mg",
                        precision=prec)
    assert ctx.last_timing()["jac_split"] == 0


@pytest.mark.parametrize("prec,tol,batch", [(64, 1e-10, 2), (32, 1e-4, 1), (32, 1e-4, 0)])
def test_multigrid_jacobian_one_run_per_monostatic_pair(mgrt, small2d, prec, tol, batch):
    """With the wavelet split and every receiver at its own source point, one run with w1
    gives both factors (the field, and the velocity filtered by w1^-1 * w2): the oracle's
    J2, the same J2 as the two-run pairing to rounding, over full and ragged batches."""
    p, o = small2d
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mode="mg", precision=prec, pairing="split", batch=batch)
    t = ctx.last_timing()
    assert t["jac_split"] == 1 and t["jac_runs"] == 1
    # several batches: the filter and sums of one overlap the run of the next
    assert t["jac_sets"] == (2 if -(-p.src.shape[0] // t["batch"]) > 1 else 1)
    J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mode="mg", precision=prec, pairing="split", batch=batch,
                             one_run=False)
    assert ctx.last_timing()["jac_sets"] == 0
    assert ctx.last_timing()["jac_runs"] == 2
    e1, e2, e12 = _rel(J1, ref), _rel(J2, ref), _rel(J1, J2)
    print(f"J2 one run prec={prec} batch={batch}: {e1:.2e} (two runs {e2:.2e}, between {e12:.2e})")
    assert e1 <= tol and e2 <= tol
    assert e12 <= (1e-12 if prec == 64 else 2e-5)


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_one_run_pipeline_ragged_last_batch(mgrt, prec, tol):
    """14 sources at width 8: two runs, the second with 6 live columns, its filter and
    sums after the first batch's on the second stream: the oracle's J2 and the two-run
    pairing's."""
    p = configs.make("c3", N=32, L=2, n_src=14, n_steps=700, n_samples=24)
    ref = Oracle.from_problem(p).jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps,
                                             p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    kw = dict(mode="mg", precision=prec, pairing="split", batch=8)
    J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps, **kw)
    t = ctx.last_timing()
    assert t["jac_runs"] == 1 and t["batch"] == 8 and t["jac_sets"] == 2
    assert t["step_launches"] == 2 * p.n_steps
    J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             one_run=False, **kw)
    e1, e12 = _rel(J1, ref), _rel(J1, J2)
    print(f"J2 one run, 8 + 6 columns, prec={prec}: {e1:.2e} (vs two runs {e12:.2e})")
    assert e1 <= tol
    assert e12 <= (1e-12 if prec == 64 else 2e-5)


@pytest.mark.parametrize("prec", [64, 32])
def test_one_run_pipeline_with_one_history_set(mgrt, small2d, prec):
    """Three batches of one source: with two history sets each run overlaps the previous
    batch's filter and sums; under a memory budget with room for one set only, each run
    waits for them.  The arithmetic is the same, so is J, bit for bit."""
    p, _ = small2d
    ctx = mgrt.context_for_problem(p)
    kw = dict(mode="mg", precision=prec, pairing="split", batch=1)
    Ja = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps, **kw)
    assert ctx.last_timing()["jac_sets"] == 2
    # the library's plan for B = 1 source per batch: correlations, J, the field and velocity
    # histories of one set, two state vectors, the transform scratch (at least 128 MiB);
    # the budget leaves room for half of a second set
    esz, N, K = prec // 8, p.n_steps, len(p.sample_steps)
    ncn = len(np.unique(p.mesh.coarse_verts))
    S, M, n = p.src.shape[0], p.mesh.n_coarse, p.mesh.coords.shape[0]
    need = S * K * ncn * 8 + S * K * M * 8 + ncn * N * esz * 2 + n * esz * 2 + (128 << 20)
    set_bytes = ncn * N * esz * 2
    Jb = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mem_budget_gb=(need + set_bytes // 2) / 2**30, **kw)
    t = ctx.last_timing()
    assert t["batch"] == 1 and t["jac_sets"] == 1
    assert np.array_equal(Ja, Jb)


def test_one_run_jacobians_of_several_lengths_in_one_context(mgrt, small2d):
    """The velocity filter's FFT plans are kept in the context per (length, batch): calls
    of different lengths each equal the two-run pairing, in FP64 with the wavelet split.
    The filter's kernel (198 samples above 2^-60 of its peak here) sets the transform
    length N + 197 rounded up to a power of two or three times one: 1,024 points for 700
    and 600 steps, 768 for 500, one length twice."""
    p, _ = small2d
    ctx = mgrt.context_for_problem(p)
    for nst in (700, 500, 600, 700):
        ss = np.arange(nst // 24 - 1, nst, nst // 24)[:24]
        J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, nst, ss, mode="mg",
                                 precision=64, pairing="split")
        assert ctx.last_timing()["jac_runs"] == 1
        J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, nst, ss, mode="mg",
                                 precision=64, pairing="split", one_run=False)
        e = _rel(J1, J2)
        print(f"{nst} steps: one run vs two runs {e:.2e}")
        assert e <= 1e-12


def test_multigrid_jacobian_pairing_flags_rejected(mgrt, small2d):
    from paper_1707_04605_amd import MgrtError, native
    p, _ = small2d
    ctx = mgrt.context_for_problem(p)
    with pytest.raises(MgrtError) as ei:
        ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="deconv", pairing="split", deconv_delta=1e-2)
    assert ei.value.name == "MGRT_E_ARG"
    # both flags at once
    with pytest.raises(MgrtError):
        ctx._check(ctx.lib.mgrt_jacobian_coarse(
            ctx._h, 1, np.ascontiguousarray(p.src[:1]).ctypes.data, 1,
            np.ascontiguousarray(p.rec[:1]).ctypes.data,
            np.ascontiguousarray(p.wavelet).ctypes.data, float(p.dt), int(p.n_steps), 1,
            np.array([p.n_steps - 1], dtype=np.int64).ctypes.data, native.JAC_MG, 0, None,
            ctx._opts(32, "batched", 0, False, native.F_JAC_SPLIT | native.F_JAC_DIRECT),
            np.empty((1, p.mesh.n_coarse)).ctypes.data), "jacobian")


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_multigrid_jacobian_depth4_all_columns(mgrt, prec, tol):
    """J2 at the differentiation workload's coarse depth (each coarse cell 16 x 16 fine
    cells: 128^2 fine, 8^2 coarse), every column, two sources over 2,000 steps (the
    physical duration of the 1024^2 run), against the oracle's brute-force J2."""
    p = configs.make("c3", N=128, L=4, n_src=2, n_steps=2000, n_samples=64)
    o = Oracle.from_problem(p)
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=prec)
    # the wavelet's band lies well below this mesh's grid scale: FP32 splits it by default,
    # and the monostatic pairs then take one run each
    assert ctx.last_timing()["jac_split"] == (prec == 32)
    assert ctx.last_timing()["jac_runs"] == (1 if prec == 32 else 2)
    err = _rel(J, ref)
    print(f"J2 depth 4, all {p.mesh.n_coarse} columns, prec={prec}: {err:.2e}")
    assert J.shape == ref.shape == (2 * 64, 128)
    assert err <= tol
    if prec == 64:
        Js = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                                 mode="mg", precision=64, pairing="split")
        assert ctx.last_timing()["jac_runs"] == 1
        print(f"  FP64 with the wavelet split (one run per pair): {_rel(Js, ref):.2e}")
        assert _rel(Js, ref) <= tol


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_multigrid_jacobian_3d_bistatic(mgrt, prec, tol):
    p = configs.make("c5", N=8, L=1, n_src=2, n_steps=240, n_samples=12)
    o = Oracle.from_problem(p)
    ref = o.jacobian_mg(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=prec, batch=2 if prec == 64 else 4)
    err = _rel(J, ref)
    print(f"J2 3D bistatic prec={prec}: {err:.2e}")
    assert err <= tol
    assert ctx.last_timing()["jac_runs"] == 2          # the antipodal receivers need their own runs


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_exact_jacobian_columns(mgrt, small2d, prec, tol):
    p, o = small2d
    cols = np.array([0, 7, 40, 77, 127])
    ref = o.jacobian_exact(p.src, p.rec, p.wavelet, p.dt, p.n_steps, cols, p.sample_steps)
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="exact", cols=cols, precision=prec)
    err = _rel(J, ref)
    print(f"J1 columns prec={prec}: {err:.2e}")
    assert err <= tol


def test_multigrid_equals_exact_at_depth_zero(mgrt):
    p = configs.make("c1", N=8, L=0, n_src=2, n_steps=200, n_samples=10)
    ctx = mgrt.context_for_problem(p)
    J2 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mode="mg", precision=64)
    J1 = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mode="exact", cols=np.arange(p.mesh.n_coarse), precision=64)
    assert _rel(J2, J1) <= 1e-11


@pytest.mark.parametrize("prec,tol", [(64, 1e-10), (32, 1e-4)])
def test_misfit_gradient_coarse_and_fine(mgrt, prec, tol):
    p = configs.make("c3", N=16, L=1, n_src=2, n_steps=300)
    o = Oracle.from_problem(p)
    rho = np.random.default_rng(17).normal(size=(2, 1, p.n_steps))
    ref = o.gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)
    ctx = mgrt.context_for_problem(p)
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, level="coarse",
                            precision=prec)
    err = _rel(g, ref)
    print(f"gradient coarse prec={prec}: {err:.2e}")
    assert err <= tol
    # fine level: d/d eps_T for a sample of fine elements
    elems = np.arange(0, p.mesh.m, 37)
    dirs = [np.eye(1, p.mesh.m, t).ravel() for t in elems]
    tl = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, dirs)
    reff = np.einsum("scrn,srn->c", tl, rho)
    gf = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, level="fine",
                             precision=prec)
    assert _rel(gf[elems], reff) <= tol
    # the coarse gradient is the sum of its fine children
    assert np.allclose(np.bincount(p.mesh.coarse_of_elem, weights=gf), g, rtol=1e-12,
                       atol=1e-14 * np.abs(g).max())


def test_misfit_gradient_3d_bistatic_and_small_budget(mgrt):
    p = configs.make("c5", N=8, L=1, n_src=3, n_steps=200)
    o = Oracle.from_problem(p)
    rho = np.random.default_rng(5).normal(size=(3, 2, p.n_steps))
    ref = o.gradient_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho)
    ctx = mgrt.context_for_problem(p)
    g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64)
    assert _rel(g, ref) <= 1e-10
    # a tiny memory budget forces one source per sweep: same gradient
    g1 = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=64,
                             mem_budget_gb=0.0004)
    assert _rel(g1, g) <= 1e-13
    assert ctx.last_timing()["batch"] == 1


def test_gradient_memory_plan_failure(mgrt):
    from paper_1707_04605_amd import MgrtError
    p = configs.make("c3", N=32, L=1, n_src=1, n_steps=100)
    ctx = mgrt.context_for_problem(p)
    with pytest.raises(MgrtError) as ei:
        ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps,
                            np.zeros((1, 1, 100)), mem_budget_gb=1e-6)
    assert ei.value.name == "MGRT_E_OOM_PLAN"


# (mesh cells per side, rows of L): rows > M forms the normal matrix L^T L on the matrix
# cores (72 and 288 columns: 2 and 5 tiles of 64 with a ragged tail, ragged row panels);
# rows < M / 2 streams L in every CG product
@pytest.mark.parametrize("N,rows", [(6, 300), (6, 30), (12, 700)])
@pytest.mark.parametrize("lprec", [64, 32])
@pytest.mark.parametrize("solver", ["auto", "cg"])
def test_tv_invert_level(mgrt, lprec, N, rows, solver):
    """auto: the formed normal matrix (M = 72, 288: ragged 64-blocks) is factorised
    (dense Cholesky, 0 iterations reported); rows = 30 streams L through CG."""
    from synth.mesh import kuhn_mesh
    ms = kuhn_mesh(2, N, 0)
    M = ms.m
    rp, col, val = regularizer.tv_matrix(ms.coords, ms.elems, 0.01)
    D = regularizer.csr_to_dense(rp, col, val, M)
    rng = np.random.default_rng(4)
    L = rng.normal(size=(rows, M))
    if lprec == 32:
        L = L.astype(np.float32)
    r = L.astype(np.float64) @ np.where(np.arange(M) % 7 == 0, 1.0, 0.0) + 0.01 * rng.normal(size=rows)
    ref = tv.tv_iterates(L.astype(np.float64), r, D, 0.05, 3)
    ctx = mgrt.Context(0)
    z, its = ctx.tv_invert_level(L, r, rp, col, val, 0.05, iters=3, cg_rtol=1e-13, cg_maxit=2000,
                                 solver=solver)
    for k in range(3):
        err = _rel(z[k], ref[k])
        print(f"TV iterate {k} (L fp{lprec}, {solver}): {err:.2e}, CG iterations {its[k]}")
        assert err <= 1e-9
    formed = M * 8 < 2 * rows * (4 if lprec == 32 else 8)
    assert (not its.any()) == (solver == "auto" and formed)
    # L resident on the device (torch tensor)
    import torch
    Ld = torch.from_numpy(np.ascontiguousarray(L)).cuda()
    zd, _ = ctx.tv_invert_level(Ld, r, rp, col, val, 0.05, iters=3, cg_rtol=1e-13, cg_maxit=2000,
                                solver=solver)
    assert _rel(zd[-1], ref[-1]) <= 1e-9


def test_tv_direct_solve_falls_back_on_a_singular_system(mgrt):
    """alpha = 0 with fewer rows than unknowns but the normal matrix formed (FP64 L, rows >
    M / 2): G is singular, the factorisation meets a pivot below its tolerance and the
    step falls back to CG, whose iterate still satisfies the normal equations."""
    from synth.mesh import kuhn_mesh
    ms = kuhn_mesh(2, 6, 0)
    M = ms.m
    rp, col, val = regularizer.tv_matrix(ms.coords, ms.elems, 0.01)
    rng = np.random.default_rng(8)
    rows = 50
    L = rng.normal(size=(rows, M))
    r = rng.normal(size=rows)
    ctx = mgrt.Context(0)
    z, its = ctx.tv_invert_level(L, r, rp, col, val, 0.0, iters=1, cg_rtol=1e-12, cg_maxit=5000)
    assert its[0] > 0
    res = L.T @ (L @ z[0]) - L.T @ r
    assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(L.T @ r)
    with pytest.raises(ValueError):
        ctx.tv_invert_level(L, r, rp, col, val, 0.0, iters=1, solver="direct")


def test_autograd_gradient_matches_oracle_and_finite_difference(mgrt):
    """torch.autograd through the traces: backward = J1^T (dLoss/dtraces) via the adjoint,
    against the oracle's tangent columns and against central differences of the loss
    evaluated through traces() itself (FP64, a few fine elements)."""
    import torch
    from paper_1707_04605_amd.autograd import Acquisition, traces
    p = configs.make("c3", N=16, L=1, n_src=2, n_steps=300)
    ctx = mgrt.context_for_problem(p)
    acq = Acquisition(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    target = torch.from_numpy(Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt,
                                                             p.n_steps) * 0.9)
    eps = torch.tensor(p.eps, dtype=torch.float64, requires_grad=True)
    loss = 0.5 * ((traces(eps, ctx, acq) - target) ** 2).sum()
    loss.backward()
    # oracle: d loss / d eps_T = J1^T (y - target) on sampled fine elements
    o = Oracle.from_problem(p)
    y = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    elems = np.arange(3, p.mesh.m, 41)
    dirs = [np.eye(1, p.mesh.m, t).ravel() for t in elems]
    tl = o.tangent(p.src, p.rec, p.wavelet, p.dt, p.n_steps, dirs)
    ref = np.einsum("scrn,srn->c", tl, y - target.numpy())
    assert _rel(eps.grad.numpy()[elems], ref) <= 1e-10
    # central differences of the same loss through traces(), h = 1e-5 of eps_T
    g = eps.grad.numpy()
    fd = []
    for t in elems[::3]:
        h = 1e-5 * float(p.eps[t])
        vals = []
        for sgn in (1.0, -1.0):
            e = torch.tensor(p.eps, dtype=torch.float64)
            e[t] += sgn * h
            with torch.no_grad():
                vals.append(float(0.5 * ((traces(e, ctx, acq) - target) ** 2).sum()))
        fd.append((vals[0] - vals[1]) / (2 * h))
    err = _rel(g[elems[::3]], np.array(fd))
    print(f"autograd gradient vs central differences on {len(fd)} elements: {err:.2e}")
    assert err <= 1e-6


def test_device_outputs_match_host_outputs(mgrt, small2d):
    """MGRT_F_DEVICE_OUT: J and traces written to caller-owned device memory are the
    host results bit for bit; a tensor of the wrong shape, dtype or device is rejected."""
    import torch
    p, _ = small2d
    ctx = mgrt.context_for_problem(p)
    J = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                            mode="mg", precision=32)
    Jd = torch.empty(J.shape, dtype=torch.float64, device="cuda")
    out = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                              mode="mg", precision=32, out=Jd)
    assert out is Jd
    assert np.array_equal(Jd.cpu().numpy(), J)
    y = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32)
    yd = torch.empty(y.shape, dtype=torch.float64, device="cuda")
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32, out=yd)
    assert np.array_equal(yd.cpu().numpy(), y)
    for bad in (torch.empty(J.shape, dtype=torch.float32, device="cuda"),
                torch.empty((J.shape[0] + 1, J.shape[1]), dtype=torch.float64, device="cuda"),
                torch.empty(J.shape, dtype=torch.float64),
                torch.empty(J.shape[::-1], dtype=torch.float64, device="cuda").t()):
        with pytest.raises(ValueError):
            ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                                mode="mg", precision=32, out=bad)


@pytest.mark.parametrize("prec", [32, 64])
def test_launch_variants_on_linearisation_paths(mgrt, small2d, prec):
    """The coarse-node histories (J2) and the adjoint correlation with the velocity
    output (gradient) in the packed-record launches (linear and XCD-contiguous order) and
    the plain linear one: bit-identical Jacobians and gradients."""
    p, _ = small2d
    ctx = mgrt.context_for_problem(p)
    J = [ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                             mode="mg", precision=prec, launch=v) for v in (1, 6, 8, 14, 16)]
    for Jv in J[1:]:
        assert np.array_equal(Jv, J[0])
    n_rec = np.asarray(p.rec).reshape(p.src.shape[0], -1, p.mesh.d).shape[1]
    rho = np.random.default_rng(23).normal(size=(p.src.shape[0], n_rec, p.n_steps))
    g = [ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=prec,
                             launch=v) for v in (1, 6, 8, 14, 16)]
    for gv in g[1:]:
        assert np.array_equal(gv, g[0])
