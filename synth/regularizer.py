"""The TV regularisation matrix D on a coarse simplex level, as an input (CSR).

Eq. (d_mat): D = beta I + G / l_max with, for the facet-adjacency of the coarse simplices,
G_ij = -|shared facet| (i != j neighbours) and G_ii = total facet measure of T'_i
(perimeter in 2D, surface area in 3D, boundary facets included); l_max is the largest
shared-facet measure.  The paper's diagonal entry is garbled (an intersection of an
element with itself); taking the element's boundary measure makes every row of G sum to
its boundary-facet measure, so D (without beta) annihilates constants away from the box
surface, which is the total-variation reading the paper states.
"""
from __future__ import annotations

import numpy as np


def _facet_measure(pts: np.ndarray) -> np.ndarray:
    """pts (k, d, d): k facets of d vertices in R^d -> (d-1)-measure."""
    d = pts.shape[1]
    if d == 2:
        return np.linalg.norm(pts[:, 1] - pts[:, 0], axis=1)
    a = pts[:, 1] - pts[:, 0]
    b = pts[:, 2] - pts[:, 0]
    return 0.5 * np.linalg.norm(np.cross(a, b), axis=1)


def tv_matrix(coords: np.ndarray, coarse_verts: np.ndarray, beta: float):
    """Return (rowptr int64, col int32, val float64) of D on the coarse elements."""
    M, dp1 = coarse_verts.shape
    d = dp1 - 1
    # all facets: drop one vertex at a time
    fac = np.concatenate([np.delete(coarse_verts, k, axis=1) for k in range(dp1)], axis=0)
    owner = np.tile(np.arange(M, dtype=np.int64), dp1)
    key = np.sort(fac, axis=1).astype(np.int64)
    meas = _facet_measure(coords[fac])
    order = np.lexsort(key.T[::-1])
    key, owner, meas = key[order], owner[order], meas[order]
    same = np.all(key[1:] == key[:-1], axis=1)
    i = owner[:-1][same]
    j = owner[1:][same]
    w = meas[:-1][same]
    lmax = w.max()
    perim = np.bincount(owner, weights=meas, minlength=M)
    rows = np.concatenate([np.arange(M), i, j])
    cols = np.concatenate([np.arange(M), j, i])
    vals = np.concatenate([beta + perim / lmax, -w / lmax, -w / lmax])
    o = np.lexsort((cols, rows))
    rows, cols, vals = rows[o], cols[o], vals[o]
    rowptr = np.zeros(M + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def csr_to_dense(rowptr, col, val, M):
    Dm = np.zeros((M, M))
    for r in range(M):
        Dm[r, col[rowptr[r]:rowptr[r + 1]]] = val[rowptr[r]:rowptr[r + 1]]
    return Dm
