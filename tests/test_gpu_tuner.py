"""The batch-width tuner: on a mesh large enough to time, every candidate width is timed
once per context (its fastest launch variant on scratch state) and the width with the
smallest estimated run time is used (the widest within 2% of it); the tuned and every
forced width give the same traces."""
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
def test_tuned_batch_width(mgrt, prec):
    # 513^2 = 263,169 nodes x 16 sources: above the tuning threshold of 2^20 node-columns
    p = configs.make("c2", N=512, L=3, n_src=16, n_steps=200)
    ctx = mgrt.context_for_problem(p)
    y = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    t = ctx.last_timing()
    cands = [b for b in t["tune_b"] if b > 0]
    us = [u for b, u in zip(t["tune_b"], t["tune_b_us"]) if b > 0]
    print(f"prec={prec}: tuned widths {cands}, us per launch {[round(u, 1) for u in us]}, "
          f"picked {t['batch']}")
    assert len(cands) >= 2 and all(u > 0 for u in us)
    assert t["batch"] in cands
    # the widest width whose estimated run time is within 2% of the smallest
    est = [-(-16 // b) * u for b, u in zip(cands, us)]
    assert t["batch"] == cands[max(i for i, e in enumerate(est) if e <= 1.02 * min(est))]
    # cached: the second call does not time again
    ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec)
    assert not any(ctx.last_timing()["tune_b"])
    for b in cands:
        yb = ctx.forward_traces(p.src, p.rec, p.wavelet, p.dt, p.n_steps, precision=prec,
                                batch=b)
        assert ctx.last_timing()["batch"] == b
        if prec == 64:
            assert np.allclose(yb, y, rtol=0, atol=1e-13 * np.abs(y).max())
        else:
            assert np.allclose(yb, y, rtol=0, atol=1e-6 * np.abs(y).max())
    ref = Oracle.from_problem(p).forward(p.src[:1], p.rec[:1], p.wavelet, p.dt, p.n_steps)
    err = np.linalg.norm(y[:1] - ref) / np.linalg.norm(ref)
    assert err <= (1e-11 if prec == 64 else 1e-4)
