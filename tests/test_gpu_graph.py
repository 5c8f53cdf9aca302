"""Replayed step runs: the stepping loop captured once per call into a graph of kernel
nodes (64 steps, or one coarse-node history chunk) and replayed, with the per-step
offsets read from a device-side step base.  Every replay must equal the direct per-step
launches bit for bit, including the steps left over after the last full run, the
history flushes, the PML state and the reversed velocity reads of the adjoint sweep."""
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


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("pml", [False, True])
def test_forward_graph_equals_direct(mgrt, prec, pml):
    # 700 steps = 10 replays of 64 steps + 60 direct steps; 5 sources (ragged batch)
    p = configs.make("c2", N=32, L=2, n_src=5, n_steps=700, pml=pml)
    ctx = mgrt.context_for_problem(p)
    y_d = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                             graph=False)
    assert ctx.last_timing()["graph_steps"] == 0
    for _ in range(2):      # two calls in a row, each capturing and replaying its own graph
        y_g = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
        assert ctx.last_timing()["graph_steps"] == 640
        assert np.array_equal(y_g, y_d)
    ref = Oracle.from_problem(p).forward(p.src, p.rec, p.wavelet, p.dt, p.n_steps)
    err = np.linalg.norm(y_g - ref) / np.linalg.norm(ref)
    print(f"graph forward prec={prec} pml={pml}: vs oracle {err:.2e}")
    assert err <= (1e-11 if prec == 64 else 1e-4)


def test_forward_short_run_takes_direct_launches(mgrt):
    p = configs.make("c1", N=16, L=1, n_src=2, n_steps=127)
    ctx = mgrt.context_for_problem(p)
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=64)
    assert ctx.last_timing()["graph_steps"] == 0


@pytest.mark.parametrize("prec", [32, 64])
def test_jacobian_and_gradient_graph_equal_direct(mgrt, prec):
    """J2 (coarse-node histories flushed at the end of every replay) and the checkpointed
    gradient (velocity segments written forward and read backwards) with and without
    replays."""
    p = configs.make("c3", N=32, L=2, n_src=3, n_steps=700, n_samples=24)
    ctx = mgrt.context_for_problem(p)
    kw = dict(mode="mg", precision=prec)
    J_d = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps,
                              graph=False, **kw)
    J_g = ctx.jacobian_coarse(p.src, p.rec, p.wavelet, p.dt, p.n_steps, p.sample_steps, **kw)
    assert ctx.last_timing()["graph_steps"] > 0
    assert np.array_equal(J_g, J_d)
    rho = np.random.default_rng(31).normal(size=(3, 1, p.n_steps))
    g_d = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=prec,
                              graph=False)
    g_g = ctx.misfit_gradient(p.src, p.rec, p.wavelet, p.dt, p.n_steps, rho, precision=prec)
    assert np.array_equal(g_g, g_d)
