"""GPU parity of mgrt_tv_invert_two_level (coarse-to-fine TV inversion, Sec. II-D/E)
against the dense FP64 oracle: x per step on T' and z_c per step on T'' to 1e-9 relative
(CG to 1e-13 on systems with condition numbers up to ~1e4), the kept parent sets exactly.
The fine coordinates themselves depend on the pair basis chosen and are not compared;
the fine field they make is (it is part of x)."""
import numpy as np
import pytest

from oracle import tv, two_level as tl
from synth import levels, regularizer

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def mgrt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_04605_amd as m
    return m


def _problem(d, Nc, rows, seed=5, beta=0.01):
    lv = levels.two_level(d, Nc)
    Dc = regularizer.tv_matrix(lv.coords, lv.verts2, beta)
    Df = regularizer.tv_matrix(lv.coords, lv.verts1, beta)
    rng = np.random.default_rng(seed)
    L = rng.normal(size=(rows, lv.M))
    xt = np.where(np.arange(lv.M) % 5 == 0, 1.0, 0.0)
    r = L @ xt + 0.01 * rng.normal(size=rows)
    return lv, L, r, Dc, Df


def _dense(csr, n):
    return regularizer.csr_to_dense(csr[0], csr[1], csr[2], n)


def _check(out, ref, n_keep, M2):
    for l, o in enumerate(ref):
        ex, ez = _rel(out["x"][l], o["x"]), _rel(out["zc"][l], o["zc"])
        print(f"step {l}: x {ex:.2e}  z_c {ez:.2e}  CG {out['cg_iters'][l].tolist()}")
        assert ex <= 1e-9 and ez <= 1e-9
        if n_keep < M2:
            a = np.sort(np.abs(o["zc"]))[::-1]
            assert a[n_keep - 1] - a[n_keep] > 1e-6 * a[0], "kept set decided by a near tie"
        np.testing.assert_array_equal(out["kept"][l], o["kept"][:min(n_keep, M2)])


# (d, Nc, rows, L precision, compression): 2D with rows > M (normal matrices formed on the
# matrix cores) and rows < M2 / 2 (L streamed in every CG product), 3D (8 children, 7
# pairs per parent), with and without the largest-third compression
CASES = [(2, 12, 700, 64, True), (2, 12, 700, 32, True), (2, 12, 30, 64, True),
         (2, 12, 700, 64, False), (3, 4, 300, 64, True), (3, 4, 300, 32, False)]


@pytest.mark.parametrize("solver", ["auto", "cg"])
@pytest.mark.parametrize("d,Nc,rows,prec,compress", CASES)
def test_two_level_matches_oracle(mgrt, d, Nc, rows, prec, compress, solver):
    lv, L, r, Dc, Df = _problem(d, Nc, rows)
    n_keep = levels.keep_third(lv.M2) if compress else lv.M2
    Lh = L.astype(np.float32) if prec == 32 else L
    ref = tl.two_level_iterates(Lh.astype(np.float64), r, lv.parent, lv.verts1,
                                _dense(Dc, lv.M2), _dense(Df, lv.M), 0.05, 3, n_keep)
    ctx = mgrt.Context(0)
    out = ctx.tv_invert_two_level(Lh, r, lv.verts1, lv.parent, lv.M2, Dc, Df, 0.05, iters=3,
                                  n_keep=n_keep, cg_rtol=1e-13, cg_maxit=5000, solver=solver)
    _check(out, ref, n_keep, lv.M2)


def test_two_level_device_matrix_and_zero_data(mgrt):
    import torch
    lv, L, r, Dc, Df = _problem(2, 12, 700)
    n_keep = levels.keep_third(lv.M2)
    ctx = mgrt.Context(0)
    a = ctx.tv_invert_two_level(L, r, lv.verts1, lv.parent, lv.M2, Dc, Df, 0.05, iters=3,
                                n_keep=n_keep, cg_rtol=1e-13, cg_maxit=5000)
    b = ctx.tv_invert_two_level(torch.from_numpy(L).cuda(), r, lv.verts1, lv.parent, lv.M2,
                                Dc, Df, 0.05, iters=3, n_keep=n_keep, cg_rtol=1e-13,
                                cg_maxit=5000)
    assert _rel(b["x"][-1], a["x"][-1]) <= 1e-12
    z = ctx.tv_invert_two_level(L, 0 * r, lv.verts1, lv.parent, lv.M2, Dc, Df, 0.05,
                                iters=3, n_keep=n_keep)
    assert not z["x"].any()


def test_single_child_levels_equal_one_level(mgrt):
    """T'' = T': no fine fluctuations, the routine is mgrt_tv_invert_level on T''."""
    lv, L, r, Dc, Df = _problem(2, 12, 400)
    ident = np.arange(lv.M, dtype=np.int32)
    ctx = mgrt.Context(0)
    out = ctx.tv_invert_two_level(L, r, lv.verts1, ident, lv.M, Df, Df, 0.05, iters=3,
                                  cg_rtol=1e-13, cg_maxit=5000)
    one, _ = ctx.tv_invert_level(L, r, *Df, 0.05, iters=3, cg_rtol=1e-13, cg_maxit=5000)
    ref = tv.tv_iterates(L, r, _dense(Df, lv.M), 0.05, 3)
    for l in range(3):
        assert _rel(out["x"][l], ref[l]) <= 1e-9
        assert _rel(one[l], ref[l]) <= 1e-9
    assert not out["cg_iters"][:, 1].any()


def test_two_level_rejects_disconnected_children(mgrt):
    from paper_1707_04605_amd import MgrtError
    lv, L, r, Dc, Df = _problem(2, 4, 50)
    bad = lv.parent.copy()
    # swap two corner children of different parents: each parent then has a child that
    # shares no facet with its siblings
    kids0 = np.flatnonzero(lv.parent == 0)
    kids5 = np.flatnonzero(lv.parent == 5)
    bad[kids0[0]], bad[kids5[0]] = 5, 0
    ctx = mgrt.Context(0)
    with pytest.raises(MgrtError) as ei:
        ctx.tv_invert_two_level(L, r, lv.verts1, bad, lv.M2, Dc, Df, 0.05)
    assert ei.value.name == "MGRT_E_MESH"
