"""The allocation-free forward entry point (mgrt_forward_traces_noalloc) against the
allocating one (mgrt_forward_traces with direct launches), through the C ABI: two calls
in a row, the second with fewer sources and steps, in both precisions, to host and to
device memory; the scratch limit and the missing-operator case are errors."""
import numpy as np
import pytest

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
def test_noalloc_equals_allocating_forward(mgrt, prec, pml):
    import torch
    p = configs.make("c2", N=48, L=2, n_src=6, n_steps=500, pml=pml)
    ctx = mgrt.context_for_problem(p)
    from paper_1707_04605_amd import MgrtError
    with pytest.raises(MgrtError) as ei:      # no operator built for this dt yet
        ctx.forward_traces_noalloc(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    assert ei.value.name == "MGRT_E_STATE"
    for ns, k in ((p.n_steps, 6), (300, 3)):        # second call: smaller input
        ref = ctx.forward_traces(p.src[:k], p.rec[:k], p.wavelet, p.dt, ns, precision=prec,
                                 graph=False)
        y = ctx.forward_traces_noalloc(p.src[:k], p.rec[:k], p.wavelet, p.dt, ns,
                                       precision=prec)
        assert y.shape == ref.shape and np.array_equal(y, ref)
        yd = torch.empty(ref.shape, dtype=torch.float64, device="cuda")
        ctx.forward_traces_noalloc(p.src[:k], p.rec[:k], p.wavelet, p.dt, ns, precision=prec,
                                   out=yd)
        assert np.array_equal(yd.cpu().numpy(), ref)


def test_noalloc_scratch_limit(mgrt):
    from paper_1707_04605_amd import MgrtError
    # 263,169 nodes x 64 columns x 4 B x 2 state fields = 135 MB > 64 MiB of scratch
    p = configs.make("c2", N=512, L=3, n_src=64, n_steps=20)
    ctx = mgrt.context_for_problem(p)
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32, batch=64)
    with pytest.raises(MgrtError) as ei:
        ctx.forward_traces_noalloc(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=32,
                                   batch=64)
    assert ei.value.name == "MGRT_E_OOM_PLAN"
    # a narrower batch of the same mesh fits (2 x 263,169 x 16 x 4 B = 34 MB)
    ctx.forward_traces(p.src[:16], p.rec[:16], p.wavelet, p.dt, p.n_steps, precision=32,
                       batch=16, graph=False)
    ref = ctx.forward_traces(p.src[:16], p.rec[:16], p.wavelet, p.dt, p.n_steps, precision=32,
                             batch=16, graph=False)
    y = ctx.forward_traces_noalloc(p.src[:16], p.rec[:16], p.wavelet, p.dt, p.n_steps,
                                   precision=32, batch=16)
    assert np.array_equal(y, ref)
