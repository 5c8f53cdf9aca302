"""Pins of the coarse-to-fine TV oracle (Sec. II-D/E) against facts fixed by the paper and
by linear algebra: the pair basis of Fig. 3, the unique decomposition, the single-level
special case, least squares at alpha = 0, brute-force minimisation, the compression size
rule, and independence of the pair basis chosen."""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import tv, two_level as tl
from synth import levels, regularizer


def _problem(d, Nc, rows, seed=5, beta=0.01):
    lv = levels.two_level(d, Nc)
    rp, cl, vl = regularizer.tv_matrix(lv.coords, lv.verts1, beta)
    Df = regularizer.csr_to_dense(rp, cl, vl, lv.M)
    rp, cl, vl = regularizer.tv_matrix(lv.coords, lv.verts2, beta)
    Dc = regularizer.csr_to_dense(rp, cl, vl, lv.M2)
    rng = np.random.default_rng(seed)
    L = rng.normal(size=(rows, lv.M))
    xt = np.where(np.arange(lv.M) % 5 == 0, 1.0, 0.0)
    r = L @ xt + 0.01 * rng.normal(size=rows)
    return lv, L, r, Dc, Df


@pytest.mark.parametrize("d,Nc", [(2, 4), (3, 2)])
def test_pair_basis_structure(d, Nc):
    lv = levels.two_level(d, Nc)
    Rf, owner = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    Rc = tl.coarse_basis(lv.parent, lv.M2)
    # 2^d children per parent, 2^d - 1 pair functions each
    assert np.all(np.bincount(lv.parent, minlength=lv.M2) == 2 ** d)
    assert Rf.shape[1] == (2 ** d - 1) * lv.M2
    for k in range(Rf.shape[1]):
        pos, neg = np.flatnonzero(Rf[:, k] == 1), np.flatnonzero(Rf[:, k] == -1)
        assert pos.size == 1 and neg.size == 1 and np.count_nonzero(Rf[:, k]) == 2
        a, b = pos[0], neg[0]
        assert lv.parent[a] == lv.parent[b] == owner[k]
        assert len(set(lv.verts1[a]) & set(lv.verts1[b])) == d     # adjacent: shared facet
    # [R_c R_f] square and nonsingular: the decomposition of eq. decomposition is unique
    B = np.hstack([Rc, Rf])
    assert B.shape == (lv.M, lv.M)
    assert np.linalg.matrix_rank(B) == lv.M


def test_pair_basis_2d_is_corner_middle():
    """Fig. 3: each T'' triangle holds a middle triangle (vertices at the parent's edge
    midpoints) and three corner ones; every pair is corner/middle."""
    lv = levels.two_level(2, 6)
    Rf, owner = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    for P in range(lv.M2):
        pv = lv.coords[lv.verts2[P]]
        mids = {tuple(np.round((pv[i] + pv[j]) / 2, 12)) for i in range(3) for j in range(i + 1, 3)}
        kids = np.flatnonzero(lv.parent == P)
        middle = [e for e in kids
                  if {tuple(np.round(lv.coords[v], 12)) for v in lv.verts1[e]} == mids]
        assert len(middle) == 1
        cols = np.flatnonzero(owner == P)
        assert cols.size == 3
        for k in cols:
            assert Rf[middle[0], k] == -1.0
            assert set(np.flatnonzero(Rf[:, k])) - {middle[0]} <= set(kids)


@pytest.mark.parametrize("d,Nc", [(2, 6), (3, 2)])
def test_decomposition_closed_form(d, Nc):
    """Fine fluctuations sum to zero over the (equal-measure) siblings, so the coarse
    coordinate of x is the mean of x over each parent's children, and
    L x = L_c x_c + L_f x_f (Sec. II-D)."""
    lv = levels.two_level(d, Nc)
    Rf, _ = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    Rc = tl.coarse_basis(lv.parent, lv.M2)
    rng = np.random.default_rng(1)
    x = rng.normal(size=lv.M)
    coef = np.linalg.solve(np.hstack([Rc, Rf]), x)
    xc, xf = coef[:lv.M2], coef[lv.M2:]
    mean = np.bincount(lv.parent, weights=x, minlength=lv.M2) / np.bincount(lv.parent)
    np.testing.assert_allclose(xc, mean, rtol=0, atol=1e-12)
    L = rng.normal(size=(7, lv.M))
    np.testing.assert_allclose(L @ x, (L @ Rc) @ xc + (L @ Rf) @ xf, rtol=0, atol=1e-11)


def test_single_child_levels_reduce_to_one_level():
    """With T'' = T' (every parent has one child) there are no fine fluctuations and the
    routine is the one-level iteration eq. tv_iteration on T''."""
    lv, L, r, Dc, Df = _problem(2, 4, 60)
    ident = np.arange(lv.M, dtype=np.int32)
    out = tl.two_level_iterates(L, r, ident, lv.verts1, Df, Df, 0.05, 3, lv.M)
    ref = tv.tv_iterates(L, r, Df, 0.05, 3)
    for o, z in zip(out, ref):
        np.testing.assert_allclose(o["x"], z, rtol=0, atol=1e-12 * np.abs(z).max())
        assert not o["f"].any()


def test_alpha_zero_first_step_is_two_least_squares_solves():
    lv, L, r, Dc, Df = _problem(2, 4, 200)
    out = tl.two_level_iterates(L, r, lv.parent, lv.verts1, Dc, Df, 0.0, 1, lv.M2)
    Rc = tl.coarse_basis(lv.parent, lv.M2)
    Rf, _ = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    zc = np.linalg.lstsq(L @ Rc, r, rcond=None)[0]
    zf = np.linalg.lstsq(L @ Rf, r - L @ Rc @ zc, rcond=None)[0]
    np.testing.assert_allclose(out[0]["zc"], zc, rtol=0, atol=1e-10)
    np.testing.assert_allclose(out[0]["x"], Rc @ zc + Rf @ zf, rtol=0, atol=1e-10)


def test_steps_minimise_their_objectives_brute_force():
    """Each level step is the minimiser of its penalised least-squares objective, with
    Gamma taken from the previous iterate of the same level; checked with a generic
    minimiser on a tiny problem (T': 8 triangles, T'': 2)."""
    lv, L, r, Dc, Df = _problem(2, 2, 12, seed=8)
    alpha = 0.3
    out = tl.two_level_iterates(L, r, lv.parent, lv.verts1, Dc, Df, alpha, 3, lv.M2)
    Rc = tl.coarse_basis(lv.parent, lv.M2)
    Rf, _ = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    for l in range(3):
        if l == 0:
            gc, gf = np.ones(lv.M2), np.ones(lv.M)
        else:
            a = np.abs(Dc @ out[l - 1]["zc"]); gc = 1 / np.maximum(a, 1e-8 * a.max())
            a = np.abs(Df @ out[l - 1]["f"]); gf = 1 / np.maximum(a, 1e-8 * a.max())
        fc = lambda z: np.sum((L @ Rc @ z - r) ** 2) + alpha * np.sum(gc * (Dc @ z) ** 2)
        zc = so.minimize(fc, np.zeros(lv.M2), method="BFGS", options={"gtol": 1e-12}).x
        np.testing.assert_allclose(out[l]["zc"], zc, rtol=0, atol=1e-6)
        rr = r - L @ Rc @ out[l]["zc"]
        ff = lambda z: np.sum((L @ Rf @ z - rr) ** 2) + alpha * np.sum(gf * (Df @ Rf @ z) ** 2)
        zf = so.minimize(ff, np.zeros(Rf.shape[1]), method="BFGS", options={"gtol": 1e-12}).x
        np.testing.assert_allclose(out[l]["f"], Rf @ zf, rtol=0, atol=1e-6)


def test_compression_keeps_largest_third_and_matches_coarse_size():
    """Sec. II-E: the fine basis of the parents with the largest third of |z_c| is kept;
    in 2D (3 fluctuations per parent) L_f then has as many columns as L_c."""
    lv, L, r, Dc, Df = _problem(2, 6, 300)       # M2 = 18, divisible by 3
    n_keep = levels.keep_third(lv.M2)
    assert 3 * n_keep == lv.M2
    out = tl.two_level_iterates(L, r, lv.parent, lv.verts1, Dc, Df, 0.05, 3, n_keep)
    Rf, owner = tl.pair_basis(lv.parent, lv.verts1, lv.M2)
    for o in out:
        k = o["kept"]
        assert k.size == n_keep
        assert np.isin(owner, k).sum() == lv.M2
        a = np.abs(o["zc"])
        assert a[k].min() >= np.delete(a, k).max()
        # the fine field lives on the kept parents only and sums to zero on each
        outside = ~np.isin(lv.parent, k)
        assert not o["f"][outside].any()
        np.testing.assert_allclose(np.bincount(lv.parent, weights=o["f"], minlength=lv.M2),
                                   0, atol=1e-12)


@pytest.mark.parametrize("d,Nc,rows", [(2, 6, 300), (3, 2, 200)])
def test_result_does_not_depend_on_pair_basis(d, Nc, rows):
    lv, L, r, Dc, Df = _problem(d, Nc, rows)
    n_keep = levels.keep_third(lv.M2)
    a = tl.two_level_iterates(L, r, lv.parent, lv.verts1, Dc, Df, 0.05, 3, n_keep)
    b = tl.two_level_iterates(L, r, lv.parent, lv.verts1, Dc, Df, 0.05, 3, n_keep,
                              root_rule="lowest_id")
    for oa, ob in zip(a, b):
        np.testing.assert_allclose(oa["x"], ob["x"], rtol=0, atol=1e-10 * np.abs(oa["x"]).max())


def test_zero_data_gives_zero_iterates():
    lv, L, r, Dc, Df = _problem(2, 4, 60)
    out = tl.two_level_iterates(L, 0 * r, lv.parent, lv.verts1, Dc, Df, 0.05, 3, lv.M2)
    for o in out:
        assert not o["x"].any()
    for z in tv.tv_iterates(L, 0 * r, Df, 0.05, 3):
        assert not z.any()


def test_levels_match_the_jacobian_coarse_ids():
    """T' of the two-level inputs is the coarse level of the fine mesh (same element ids
    and vertices, up to the grid scaling)."""
    from synth.mesh import kuhn_mesh
    for d, N, Lr in [(2, 16, 2), (3, 8, 1)]:
        ms = kuhn_mesh(d, N, Lr)
        lv = levels.two_level(d, N >> Lr)
        np.testing.assert_allclose(ms.coords[ms.coarse_verts], lv.coords[lv.verts1], atol=1e-12)
