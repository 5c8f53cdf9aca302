"""Several leap-frog steps per launch on small meshes: each workgroup advances its tile
and the tile's k-ring in the stiffness graph k steps in LDS.  Every node update is the
one-step launch's, term by term, so the traces agree with one launch per step to
rounding and with the oracle to the usual bounds: 2D and 3D meshes, a step count that
is not a multiple of k, sources and receivers spread over many tiles' rings, replayed
runs of launches.  (Runs that resume from a given state, the gradient's checkpointed
forward sweep at one column, take this path in the gradient tests under a small memory
budget.)"""
import numpy as np
import pytest

from oracle import Oracle
from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mgrt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_04605_amd as m
    return m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 1e-4)])
def test_multistep_2d_equals_one_step_and_oracle(mgrt, prec, tol):
    # 1,089 nodes = 5 tiles of 256; 701 steps is not a multiple of k; five receivers
    # across the mesh, the source near the top edge
    p = configs.make("c1", N=32, L=0, n_src=1, n_steps=701)
    rec = np.array([[[0.0, 1.4], [0.3, -0.2], [-1.0, 0.5], [1.2, -1.2], [-0.05, 0.02]]])
    ctx = mgrt.context_for_problem(p)
    y1 = ctx.forward_traces(p.src, rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                            one_step=True)
    assert ctx.last_timing()["steps_per_launch"] == 1
    ym = ctx.forward_traces(p.src, rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    t = ctx.last_timing()
    k = t["steps_per_launch"]
    assert k in (2, 4, 6, 8)
    assert t["step_launches"] == -(-p.n_steps // k)
    d = float(np.abs(ym - y1).max() / np.abs(y1).max())
    ref = Oracle.from_problem(p).forward(p.src, rec, p.wavelet, p.dt, p.n_steps)
    err = _rel(ym, ref)
    print(f"2D prec={prec}: {k} steps per launch; vs one step per launch {d:.2e}, "
          f"vs oracle {err:.2e}")
    assert d <= (1e-13 if prec == 64 else 1e-6)
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 1e-4)])
def test_multistep_3d_equals_one_step_and_oracle(mgrt, prec, tol):
    # 9^3 = 729 nodes in Morton order: 3 tiles, k-rings of the 14-neighbour stencil
    p = configs.make("c4", N=8, L=1, n_src=1, n_steps=300)
    ctx = mgrt.context_for_problem(p)
    y1 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                            one_step=True)
    ym = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    k = ctx.last_timing()["steps_per_launch"]
    assert k >= 2
    d = float(np.abs(ym - y1).max() / np.abs(y1).max())
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    err = _rel(ym, ref)
    print(f"3D prec={prec}: {k} steps per launch; vs one step per launch {d:.2e}, "
          f"vs oracle {err:.2e}")
    assert d <= (1e-13 if prec == 64 else 1e-6)
    assert err <= tol


def test_multistep_after_permittivity_change(mgrt):
    """The region tables carry the coefficients: a new permittivity rebuilds them."""
    p = configs.make("c1", N=32, L=0, n_src=1, n_steps=400)
    ctx = mgrt.context_for_problem(p)
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    eps2 = np.asarray(p.eps) * 1.3
    ctx.upload_permittivity(eps2)
    ym = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    assert ctx.last_timing()["steps_per_launch"] > 1
    y1 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64,
                            one_step=True)
    ref = Oracle.from_problem(p, eps=eps2).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    assert float(np.abs(ym - y1).max() / np.abs(y1).max()) <= 1e-13
    assert _rel(ym, ref) <= 1e-11


def test_multistep_not_used_for_batches(mgrt):
    """Several columns keep one launch per step (the batched stepper)."""
    p = configs.make("c1", N=32, L=0, n_src=3, n_steps=200)
    ctx = mgrt.context_for_problem(p)
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    t = ctx.last_timing()
    assert t["steps_per_launch"] == 1 and t["step_launches"] == p.n_steps


@pytest.mark.parametrize("prec", [64, 32])
def test_multistep_graph_replay(mgrt, prec):
    """Runs of 64 launches of k steps are captured once and replayed (the series index and
    the trace row read from a device-side step base); 1,100 steps = two replays of 512
    and 76 steps in direct launches.  Replays equal direct launches bit for bit, and one
    step per launch to rounding."""
    p = configs.make("c1", N=32, L=0, n_src=1, n_steps=1100)
    ctx = mgrt.context_for_problem(p)
    yg = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    t = ctx.last_timing()
    assert t["steps_per_launch"] == 8 and t["graph_steps"] == 1024
    assert t["step_launches"] == 128 + 10
    yd = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                            graph=False)
    assert ctx.last_timing()["graph_steps"] == 0
    assert np.array_equal(yg, yd)
    y1 = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                            one_step=True)
    d = float(np.abs(yg - y1).max() / np.abs(y1).max())
    print(f"replayed multi-step prec={prec}: vs one step per launch {d:.2e}")
    assert d <= (1e-13 if prec == 64 else 1e-6)
