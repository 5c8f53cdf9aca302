"""Pins of the TV-regularised iteration reference (Sec. II-C, eqs. tv_iteration, d_mat)."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import minimize

from oracle import tv
from synth import regularizer
from synth.mesh import kuhn_mesh


def _problem(M=6, rows=9, seed=0):
    rng = np.random.default_rng(seed)
    L = rng.normal(size=(rows, M))
    z_true = np.zeros(M)
    z_true[1] = 1.0
    z_true[4] = -0.7
    r = L @ z_true + 0.05 * rng.normal(size=rows)
    D = np.eye(M) * 1.3 - 0.4 * (np.eye(M, k=1) + np.eye(M, k=-1))
    return L, r, D


def test_first_iterate_is_generalised_tikhonov():
    """Gamma_0 = I: z_1 minimises ||L z - r||^2 + alpha ||D z||^2, i.e. the least-squares
    solution of the stacked system [L; sqrt(alpha) D] z = [r; 0]."""
    L, r, D = _problem()
    alpha = 0.3
    z1 = tv.tv_iterates(L, r, D, alpha, 1)[0]
    A = np.vstack([L, np.sqrt(alpha) * D])
    b = np.concatenate([r, np.zeros(D.shape[0])])
    ref = sla.lstsq(A, b)[0]
    assert np.allclose(z1, ref, rtol=1e-12, atol=1e-13)


def test_small_alpha_gives_least_squares():
    L, r, D = _problem(rows=12)
    z = tv.tv_iterates(L, r, D, 1e-12, 1)[0]
    assert np.allclose(z, np.linalg.lstsq(L, r, rcond=None)[0], rtol=1e-8, atol=1e-9)


def test_fixed_point_minimises_l1_objective():
    """The iteration's fixed point minimises ||L z - r||^2 + 2 alpha ||D z||_1; compared
    with a brute-force constrained minimisation of the epigraph form."""
    L, r, D = _problem()
    alpha = 0.2
    z = tv.tv_iterates(L, r, D, alpha, 400)[-1]
    M = L.shape[1]

    def F(zz):
        return np.sum((L @ zz - r) ** 2) + 2 * alpha * np.sum(np.abs(D @ zz))

    # epigraph: min ||Lz - r||^2 + 2 alpha sum t  s.t.  -t <= D z <= t
    def obj(v):
        return np.sum((L @ v[:M] - r) ** 2) + 2 * alpha * np.sum(v[M:])

    cons = [{"type": "ineq", "fun": lambda v: v[M:] - D @ v[:M]},
            {"type": "ineq", "fun": lambda v: v[M:] + D @ v[:M]}]
    best = None
    for s in range(4):
        x0 = np.concatenate([np.random.default_rng(s).normal(size=M), np.ones(M)])
        res = minimize(obj, x0, constraints=cons, method="SLSQP",
                       options={"ftol": 1e-14, "maxiter": 2000})
        if best is None or res.fun < best.fun:
            best = res
    assert F(z) <= best.fun + 1e-7
    assert np.allclose(z, best.x[:M], atol=2e-4)


def test_regulariser_closed_form_on_uniform_mesh():
    """D on the uniform "/" coarse mesh: interior diagonal beta + 1 + sqrt(2), legs
    -1/sqrt(2), hypotenuse -1; rows of interior elements sum to beta."""
    ms = kuhn_mesh(2, 8, 0)
    beta = 0.01
    rp, col, val = regularizer.tv_matrix(ms.coords, ms.elems, beta)
    Dm = regularizer.csr_to_dense(rp, col, val, ms.m)
    assert np.allclose(Dm, Dm.T)
    # element of cell (3, 3), local 0: fully interior
    e = (3 * 8 + 3) * 2
    assert Dm[e, e] == pytest.approx(beta + 1 + np.sqrt(2), rel=1e-14)
    offs = np.sort(Dm[e][Dm[e] < 0])
    assert np.allclose(offs, [-1.0, -1 / np.sqrt(2), -1 / np.sqrt(2)], rtol=1e-14)
    interior = [(cy * 8 + cx) * 2 + q for cy in range(1, 7) for cx in range(1, 7) for q in (0, 1)]
    assert np.allclose(Dm[interior].sum(axis=1), beta, atol=1e-13)
