"""Dense FP64 reference of the coarse-to-fine TV inversion (Sec. II-D, eqs.
decomposition, tv_iteration_0, tv_iteration_2; Sec. II-E, compression of coefficients).

Test infrastructure only.

Levels: T' (M simplices, the level of the Jacobian L) nested in T'' (M2 simplices).
R_c maps a T'' coordinate vector to the piecewise constant T' function (each T' simplex
takes its parent's value).  R_f holds the fine-fluctuation basis: one column per adjacent
pair of sibling simplices (sharing a facet), +1 on one and -1 on the other; per parent the
pairs are the edges of a spanning tree of the siblings' facet adjacency, rooted at the
sibling with most sibling neighbours (in 2D the middle triangle, so every pair is
corner/middle as in Fig. 3).  Every column sums to zero over the siblings, and
[R_c R_f] is square and nonsingular, so the decomposition is unique.

With z = x - x0 = 0 initially and r = y - y0, for l = 0 .. iters-1:
  (2)  z_c = (L_c^T L_c + alpha D_c^T G_c D_c)^{-1} L_c^T r,   L_c = L R_c,
       G_c = I for l = 0, else diag(1 / max(|D_c z_c,prev|, tau))
  compression: keep the fine basis functions of the n_keep parents with the largest
       |z_c| (ties: lower id first); R_f restricted to them, L_f = L R_f
  (3)  z_f = (L_f^T L_f + alpha (D_f R_f)^T G_f (D_f R_f))^{-1} L_f^T (r - L_c z_c),
       G_f = I for l = 0, else diag(1 / max(|D_f f_prev|, tau)) with f_prev the previous
       fine field R_f z_f on T'
  (4)  x_{l+1} - x0 = R_c z_c + R_f z_f
Readings: the paper leaves D_f undefined; here the fine penalty is the T' regularisation
matrix D_f (eq. d_mat on T') applied to the fine field R_f z_f, so it does not depend on
which pair basis spans the kept fluctuations, and G_f lives on the T' rows, which stay
the same when the kept set changes between steps.  tau = 1e-8 max|.| as on one level, and
G = I when the vector it is built from vanishes.
"""
from __future__ import annotations

from collections import deque

import numpy as np
import scipy.linalg as sla


def _siblings(parent, M2):
    kids = [[] for _ in range(M2)]
    for e, p in enumerate(parent):
        kids[int(p)].append(e)
    return kids


def _share_facet(verts, a, b):
    d = verts.shape[1] - 1
    return len(set(verts[a].tolist()) & set(verts[b].tolist())) == d


def pair_basis(parent, verts, M2, root_rule="most_neighbours"):
    """Dense R_f (M x K) and the parent of every column.

    root_rule "most_neighbours" is the basis described above; "lowest_id" roots every
    spanning tree at the lowest sibling id (another valid pair basis, for checking that
    results do not depend on the choice)."""
    parent = np.asarray(parent)
    verts = np.asarray(verts)
    M = parent.size
    cols, owners = [], []
    for P, kids in enumerate(_siblings(parent, M2)):
        if len(kids) <= 1:
            continue
        adj = {a: [b for b in kids if b != a and _share_facet(verts, a, b)] for a in kids}
        if root_rule == "most_neighbours":
            root = min(kids, key=lambda a: (-len(adj[a]), a))
        else:
            root = min(kids)
        seen = {root}
        queue = deque([root])
        while queue:
            a = queue.popleft()
            for b in sorted(adj[a]):
                if b in seen:
                    continue
                seen.add(b)
                queue.append(b)
                col = np.zeros(M)
                col[b] = 1.0
                col[a] = -1.0
                cols.append(col)
                owners.append(P)
        if len(seen) != len(kids):
            raise ValueError(f"siblings of parent {P} are not facet-connected")
    Rf = np.stack(cols, axis=1) if cols else np.zeros((M, 0))
    return Rf, np.asarray(owners, dtype=np.int64)


def coarse_basis(parent, M2):
    """Dense R_c (M x M2): R_c[e, parent[e]] = 1."""
    parent = np.asarray(parent)
    Rc = np.zeros((parent.size, M2))
    Rc[np.arange(parent.size), parent] = 1.0
    return Rc


def kept_parents(zc, n_keep):
    """The n_keep parents with the largest |z_c|, ties to the lower id, ascending ids."""
    order = np.lexsort((np.arange(zc.size), -np.abs(zc)))
    return np.sort(order[:n_keep])


def _solve(L, rhs, D, g, alpha):
    A = L.T @ L + alpha * (D.T @ (g[:, None] * D))
    return sla.cho_solve(sla.cho_factor(A, lower=True), L.T @ rhs)


def _gamma(v, tau_rel):
    """diag(1 / max(|v|, tau)); the identity when v vanishes (no jump information)."""
    a = np.abs(v)
    if a.max() == 0.0:
        return np.ones_like(a)
    return 1.0 / np.maximum(a, tau_rel * a.max())


def two_level_iterates(L, r, parent, verts, Dc, Df, alpha, iters, n_keep, tau_rel=1e-8,
                       root_rule="most_neighbours"):
    """Returns a list of dicts per step: x (M, = x_{l+1} - x0 on T'), zc (M2), f (M, the
    fine field R_f z_f) and kept (parent ids)."""
    L = np.asarray(L, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    Dc = np.asarray(Dc, dtype=np.float64)
    Df = np.asarray(Df, dtype=np.float64)
    M2 = Dc.shape[0]
    Rc = coarse_basis(parent, M2)
    Rf_all, owner = pair_basis(parent, verts, M2, root_rule)
    Lc = L @ Rc
    zc = np.zeros(M2)
    f = np.zeros(L.shape[1])
    out = []
    for l in range(iters):
        gc = np.ones(M2) if l == 0 else _gamma(Dc @ zc, tau_rel)
        zc = _solve(Lc, r, Dc, gc, alpha)
        kept = kept_parents(zc, min(n_keep, M2))
        Rf = Rf_all[:, np.isin(owner, kept)]
        if Rf.shape[1]:
            gf = np.ones(Df.shape[0]) if l == 0 else _gamma(Df @ f, tau_rel)
            zf = _solve(L @ Rf, r - Lc @ zc, Df @ Rf, gf, alpha)
            f = Rf @ zf
        else:
            f = np.zeros(L.shape[1])
        out.append({"x": Rc @ zc + f, "zc": zc.copy(), "f": f.copy(), "kept": kept})
    return out
