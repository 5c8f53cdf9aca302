"""GPU parity of mgrt_forward_traces against the FP64 oracle (same seeded inputs).

Tolerances (relative L2 over all traces): FP64 wave fields <= 1e-11, FP32 <= 1e-4.
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs
from synth.mesh import kuhn_mesh

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
FP32_TOL = 1e-4


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def mgrt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_04605_amd as m
    return m


def test_c1_full_fp64_fp32_plain(mgrt):
    """128^2 cells, one monostatic source, 4,000 steps (the FP64 single-source case)."""
    p = configs.make("c1")
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g64 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    gpl = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64,
                             variant="plain")
    g32 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32)
    print(f"c1: fp64 {_rel(g64, ref):.2e} plain {_rel(gpl, ref):.2e} fp32 {_rel(g32, ref):.2e}")
    assert _rel(g64, ref) <= FP64_TOL
    assert _rel(gpl, ref) <= FP64_TOL
    assert _rel(g32, ref) <= FP32_TOL


@pytest.mark.parametrize("prec,batch", [(64, 2), (64, 4), (64, 8), (32, 4), (32, 8), (32, 16)])
def test_ragged_batches(mgrt, prec, batch):
    """5 sources over batches of 2..16 columns: full and partly empty batches, several
    tiles and a ragged last tile (n = 65^2 nodes)."""
    p = configs.make("c2", N=64, L=2, n_src=5, n_steps=1500)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec, batch=batch)
    err = _rel(g, ref)
    print(f"ragged prec={prec} batch={batch}: {err:.2e}")
    assert err <= (FP64_TOL if prec == 64 else FP32_TOL)


@pytest.mark.parametrize("prec,batch,cfg", [(32, 4, "c2"), (32, 8, "c2"), (64, 8, "c2"),
                                            (32, 64, "c2"), (64, 32, "c2"), (32, 8, "c5"),
                                            (32, 16, "c5"), (32, 32, "c5"),
                                            (32, 64, "c2big"), (64, 32, "c2big")])
def test_launch_variants_identical(mgrt, prec, batch, cfg):
    """Every launch variant (non-temporal state, XCD-contiguous tile order, packed per-node
    records shared by cross-lane shuffles, speculative gathers at the dominant neighbour
    offsets; with too few lanes per node for the record the packed launches fall back) on meshes whose tile counts leave a ragged last tile, and
    (c2big: 66,049 nodes, over 2,048 tiles) on more tiles than the device holds resident at
    once: bit-identical traces, equal to the oracle."""
    if cfg == "c2":
        p = configs.make("c2", N=64, L=2, n_src=5, n_steps=400)
    elif cfg == "c2big":
        p = configs.make("c2", N=256, L=2, n_src=5, n_steps=240)
    else:
        p = configs.make("c5", N=10, L=1, n_src=3, n_steps=200)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    outs = []
    for v in range(1, 17):
        g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                               batch=batch, launch=v)
        assert ctx.last_timing()["variant"] == v - 1
        outs.append(g)
    err = _rel(outs[0], ref)
    print(f"launch variants {cfg} prec={prec} batch={batch}: {err:.2e}")
    assert err <= (FP64_TOL if prec == 64 else FP32_TOL)
    for g in outs[1:]:
        assert np.array_equal(g, outs[0])


@pytest.mark.parametrize("prec", [64, 32])
def test_3d_bistatic(mgrt, prec):
    """3D Kuhn mesh, three sources with two receivers each (source point and antipode)."""
    p = configs.make("c5", N=12, L=1, n_src=3, n_steps=500)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    err = _rel(g, ref)
    print(f"3d bistatic prec={prec}: {err:.2e}")
    assert err <= (FP64_TOL if prec == 64 else FP32_TOL)


def test_conductivity_and_admittance(mgrt):
    """Lossy body (sigma = 5 eps_r inside, Sec. III) and a non-unit boundary admittance."""
    from paper_1707_04605_amd import Context
    p = configs.make("c1", N=48, L=0, n_src=2, n_steps=1200)
    ms = p.mesh
    sig = np.where(p.eps > 1.5, 5.0 * p.eps, 0.0)
    adm = np.full(ms.bfacets.shape[0], 0.7)
    o = Oracle(2, ms.coords, ms.elems, p.eps, sigma=sig, bfacets=ms.bfacets, admittance=adm)
    ref = o.forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = Context(0)
    ctx.upload_mesh(2, ms.coords, ms.elems, ms.bfacets, adm)
    ctx.upload_permittivity(p.eps, sig)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    assert _rel(g, ref) <= FP64_TOL


def test_single_step_and_empty_absorbing_boundary(mgrt):
    """Degenerate sizes: one step; a closed domain (no boundary facets)."""
    from paper_1707_04605_amd import Context
    p = configs.make("c1", N=16, L=0, n_src=1, n_steps=1)
    ms = p.mesh
    o = Oracle(2, ms.coords, ms.elems, p.eps)
    ctx = Context(0)
    ctx.upload_mesh(2, ms.coords, ms.elems)
    ctx.upload_permittivity(p.eps)
    for nst in (1, 2, 300):
        w = np.sin(np.arange(nst) * 0.3) + 1.0
        ref = o.forward(p.src, p.rec, w, p.dt, nst)
        g = ctx.forward_traces(p.src, p.rec, w, p.dt, nst, precision=64)
        assert np.abs(g - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)


def test_empty_inputs_rejected(mgrt):
    """No sources, no receivers, no steps or no samples: MGRT_E_ARG from the C ABI (the
    forward call directly, the Jacobian and gradient through the binding), and the context
    keeps working."""
    import ctypes as C
    from paper_1707_04605_amd import MgrtError
    p = configs.make("c1", N=16, L=1, n_src=1, n_steps=20)
    ctx = mgrt.context_for_problem(p)
    src = np.ascontiguousarray(p.src, np.float64)
    rec = np.ascontiguousarray(p.rec, np.float64)
    w = np.ascontiguousarray(p.wavelet, np.float64)
    out = np.zeros(4096)
    opts = ctx._opts(64, "batched", 0, False)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    for n_src, n_rec, n_steps in ((0, 1, 20), (1, 0, 20), (1, 1, 0), (1, 1, -3), (-1, 1, 20)):
        rc = ctx.lib.mgrt_forward_traces(ctx._h, n_src, ptr(src), n_rec, ptr(rec), ptr(w),
                                         float(p.dt), n_steps, C.byref(opts), ptr(out))
        assert MgrtError(rc, "").name == "MGRT_E_ARG", (n_src, n_rec, n_steps)
    with pytest.raises(MgrtError) as ei:
        ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, 20, np.zeros(0, np.int64),
                            mode="mg", precision=64)
    assert ei.value.name == "MGRT_E_ARG"
    with pytest.raises(MgrtError) as ei:
        ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, 0, np.zeros((1, 1, 0)), precision=64)
    assert ei.value.name == "MGRT_E_ARG"
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, 20, precision=64)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, 20)
    assert _rel(g, ref) <= FP64_TOL


@pytest.mark.parametrize("prec", [32, 64])
def test_widest_batch(mgrt, prec):
    """The widest batch (128 columns per launch, 32 lanes per node in FP32, 64 in FP64) with
    a ragged second batch (130 sources), against the oracle."""
    p = configs.make("c1", N=16, L=0, n_src=130, n_steps=300)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    ctx = mgrt.context_for_problem(p)
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec, batch=128)
    assert ctx.last_timing()["batch"] == 128
    err = _rel(g, ref)
    print(f"batch 128 prec={prec}: {err:.2e}")
    assert err <= (FP64_TOL if prec == 64 else FP32_TOL)


def test_unstable_dt_and_bad_inputs_rejected(mgrt):
    from paper_1707_04605_amd import MgrtError
    p = configs.make("c1", N=16, L=0, n_steps=10)
    ctx = mgrt.context_for_problem(p)
    bound = ctx.stability_bound()
    assert bound > p.dt
    with pytest.raises(MgrtError) as ei:
        ctx.forward_traces(p.src, p.rec, p.wavelet, 1.01 * bound, 10)
    assert ei.value.name == "MGRT_E_UNSTABLE"
    with pytest.raises(MgrtError) as ei:
        ctx.forward_traces(np.array([[5.0, 5.0]]), p.rec, p.wavelet, p.dt, 10)
    assert ei.value.name == "MGRT_E_ARG"
    bad = p.eps.copy()
    bad[3] = np.nan
    with pytest.raises(MgrtError) as ei:
        ctx.upload_permittivity(bad)
    assert ei.value.name == "MGRT_E_NONFINITE"
    for v in (0.0, -1.0):
        bad = p.eps.copy()
        bad[5] = v
        with pytest.raises(MgrtError) as ei:
            ctx.upload_permittivity(bad)
        assert ei.value.name == "MGRT_E_ARG"
    ctx.upload_permittivity(p.eps)               # the context still works afterwards
    w = p.wavelet.copy()
    w[4] = np.nan
    with pytest.raises(MgrtError) as ei:
        ctx.forward_traces(p.src, p.rec, w, p.dt, 10)
    assert ei.value.name == "MGRT_E_NONFINITE"
    rho = np.zeros((1, 1, 10))
    rho[0, 0, 2] = np.inf
    with pytest.raises(MgrtError) as ei:
        ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, 10, rho, level="fine")
    assert ei.value.name == "MGRT_E_NONFINITE"
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, 10)
    assert np.isfinite(g).all()
    ms = kuhn_mesh(2, 4, 1)
    from paper_1707_04605_amd import Context
    c2 = Context(0)
    wrong = ms.coarse_of_elem.copy()
    wrong[0] = (wrong[0] + 1) % ms.n_coarse
    with pytest.raises(MgrtError) as ei:
        c2.upload_mesh(2, ms.coords, ms.elems, ms.bfacets, None, wrong, ms.coarse_verts)
    assert ei.value.name == "MGRT_E_MESH"


def test_c2_full_size_sampled_sources(mgrt):
    """The 1024^2, 64-source FP32 launches the benchmark times; sources 0 and 37 compared
    with the oracle over the first 3,000 steps (a prefix of a run depends only on
    earlier steps)."""
    p = configs.make("c2")
    ctx = mgrt.context_for_problem(p)
    nst = 3000
    g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, nst, precision=32)
    o = Oracle.from_problem(p)
    for s in (0, 37):
        ref = o.forward(p.src[s:s + 1], p.rec[s:s + 1], p.wavelet, p.dt, nst)
        err = _rel(g[s:s + 1], ref)
        print(f"c2 source {s}: fp32 rel L2 {err:.2e}")
        assert err <= FP32_TOL
    t = ctx.last_timing()
    # the batch width the tuner timed fastest among its candidates (16, 32, 64 columns)
    cands = [b for b in t["tune_b"] if b > 0]
    assert cands == [16, 32, 64] and t["batch"] in cands
    assert t["node_updates"] == p.mesh.n * nst * 64


def test_context_in_a_process_that_imports_only_the_package(mgrt):
    """A fresh process that imports the package (not torch) and creates a context: the
    binding must leave one HIP runtime in the process (regression)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import numpy as np, paper_1707_04605_amd as m\n"
            "ctx = m.Context(0)\n"
            "print('context ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "context ok" in r.stdout, r.stderr[-2000:]


def test_launch_variant_out_of_range_is_rejected(mgrt):
    p = configs.make("c2", N=16, L=2, n_src=1, n_steps=50)
    ctx = mgrt.context_for_problem(p)
    for bad in (17, -1):
        with pytest.raises(mgrt.MgrtError):
            ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32,
                               launch=bad)
