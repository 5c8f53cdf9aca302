"""Nested Kuhn simplex meshes of the square [-1.5, 1.5]^2 and the cube [-1.5, 1.5]^3.

Seeded-input side only: this module builds mesh connectivity and index maps.  It holds
no finite-element arithmetic (no volumes, gradients, mass or stiffness).

Construction (the mesh hierarchy of Sec. II-B and Fig. 2, and the regular edge-halving
refinement of Sec. III):

* The box is cut into N^d cells; every cell is cut into d! Kuhn simplices, one per
  permutation pi of the axes (lexicographic order of the permutations).  Simplex pi
  has vertices v0 = cell min corner, v_k = v_{k-1} + e_{pi(k-1)}.  In 2D this is the
  "/" split of every square into two triangles.
* Nodes are numbered lexicographically, x fastest: id = sum_a idx_a (N+1)^a.
* Fine element id = cell_lin * d! + perm_index.
* Halving every edge of a Kuhn simplex gives Kuhn simplices of the grid with half the
  spacing, so the mesh with N cells per axis is nested inside the one with N / 2^L
  cells (the coarse inversion level T').  A fine simplex lies in the coarse simplex
  whose axis ordering equals the ordering of (sub-cell index, centroid offset).
* Coarse element id = coarse_cell_lin * d! + coarse_perm_index (same numbering rule).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

BOX_LO = -1.5
BOX_HI = 1.5


def permutations(d: int) -> np.ndarray:
    """All permutations of range(d), lexicographic order, shape (d!, d)."""
    return np.array(list(itertools.permutations(range(d))), dtype=np.int64)


@dataclass
class Mesh:
    d: int
    N: int                      # cells per axis of the fine mesh T
    L: int                      # refinement depth between the coarse level T' and T
    coords: np.ndarray          # (n, d) float64
    elems: np.ndarray           # (m, d+1) int32, fine simplices
    bfacets: np.ndarray         # (nb, d) int32, facets on the box surface
    coarse_of_elem: np.ndarray  # (m,) int32, nesting map T -> T'
    coarse_verts: np.ndarray    # (M, d+1) int32, fine-node ids of coarse vertices
    centroids: np.ndarray       # (m, d) float64 element centroids (classification only)

    @property
    def n(self) -> int:
        return self.coords.shape[0]

    @property
    def m(self) -> int:
        return self.elems.shape[0]

    @property
    def Nc(self) -> int:
        return self.N >> self.L

    @property
    def n_coarse(self) -> int:
        return self.coarse_verts.shape[0]

    @property
    def h(self) -> float:
        return (BOX_HI - BOX_LO) / self.N


def _node_id(idx: np.ndarray, N: int) -> np.ndarray:
    """idx (..., d) integer grid indices -> lexicographic node id (x fastest)."""
    d = idx.shape[-1]
    out = np.zeros(idx.shape[:-1], dtype=np.int64)
    stride = 1
    for a in range(d):
        out += idx[..., a] * stride
        stride *= (N + 1)
    return out


def _lex_cells(N: int, d: int) -> np.ndarray:
    """(N^d, d) integer cell indices in lexicographic order (x fastest)."""
    lin = np.arange(N ** d, dtype=np.int64)
    idx = np.empty((lin.size, d), dtype=np.int64)
    rem = lin
    for a in range(d):
        idx[:, a] = rem % N
        rem = rem // N
    return idx


def kuhn_mesh(d: int, N: int, L: int = 0) -> Mesh:
    """Kuhn mesh with N cells per axis; coarse level has N >> L cells per axis."""
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    if N % (1 << L):
        raise ValueError("N must be divisible by 2^L")
    perms = permutations(d)
    nperm = perms.shape[0]
    h = (BOX_HI - BOX_LO) / N

    # nodes
    nidx = _lex_cells(N + 1, d)
    coords = BOX_LO + nidx.astype(np.float64) * h

    # fine elements
    cells = _lex_cells(N, d)                       # (C, d)
    eye = np.eye(d, dtype=np.int64)
    verts = np.empty((cells.shape[0], nperm, d + 1, d), dtype=np.int64)
    for q, pi in enumerate(perms):
        v = cells.copy()
        verts[:, q, 0, :] = v
        for k in range(d):
            v = v + eye[pi[k]]
            verts[:, q, k + 1, :] = v
    elems = _node_id(verts, N).reshape(-1, d + 1).astype(np.int32)
    centroids = (BOX_LO + (verts.astype(np.float64).mean(axis=2)) * h).reshape(-1, d)

    # nesting map: coarse cell and coarse permutation of each fine simplex
    Lm = (1 << L) - 1
    ccell = cells >> L                             # (C, d)
    local = cells & Lm                             # (C, d)
    Nc = N >> L
    clin = np.zeros(cells.shape[0], dtype=np.int64)
    stride = 1
    for a in range(d):
        clin += ccell[:, a] * stride
        stride *= Nc
    perm_lookup = {tuple(p): i for i, p in enumerate(perms)}
    coarse = np.empty((cells.shape[0], nperm), dtype=np.int64)
    for q, pi in enumerate(perms):
        pos = np.empty(d, dtype=np.int64)
        pos[pi] = np.arange(d)
        # key_a = local_a*(d+1) + (d - pos(a)); the coarse simplex orders axes by key descending
        key = local * (d + 1) + (d - pos)[None, :]
        order = np.argsort(-key, axis=1, kind="stable")
        # map each row's order to its permutation index
        code = np.zeros(cells.shape[0], dtype=np.int64)
        for a in range(d):
            code = code * d + order[:, a]
        lut = np.full(d ** d, -1, dtype=np.int64)
        for p, i in perm_lookup.items():
            c = 0
            for a in range(d):
                c = c * d + p[a]
            lut[c] = i
        cperm = lut[code]
        assert (cperm >= 0).all()
        coarse[:, q] = clin * nperm + cperm
    coarse_of_elem = coarse.reshape(-1).astype(np.int32)

    # coarse vertices (fine-node ids)
    ccells = _lex_cells(Nc, d)
    cverts = np.empty((ccells.shape[0], nperm, d + 1, d), dtype=np.int64)
    for q, pi in enumerate(perms):
        v = ccells << L
        cverts[:, q, 0, :] = v
        for k in range(d):
            v = v + (eye[pi[k]] << L)
            cverts[:, q, k + 1, :] = v
    coarse_verts = _node_id(cverts, N).reshape(-1, d + 1).astype(np.int32)

    bfacets = _box_facets(d, N, cells, perms, elems.reshape(cells.shape[0], nperm, d + 1))
    return Mesh(d=d, N=N, L=L, coords=coords, elems=elems, bfacets=bfacets,
                coarse_of_elem=coarse_of_elem, coarse_verts=coarse_verts,
                centroids=centroids)


def _box_facets(d, N, cells, perms, el):
    """Facets on the box surface.

    On the face x_a = min, the simplices with pi(d-1) = a have the facet opposite their
    last vertex there; on x_a = max, those with pi(0) = a have the facet opposite v0.
    """
    out = []
    for a in range(d):
        lo = cells[:, a] == 0
        hi = cells[:, a] == N - 1
        for q, pi in enumerate(perms):
            if pi[d - 1] == a:
                out.append(el[lo, q, :d])
            if pi[0] == a:
                out.append(el[hi, q, 1:])
    return np.concatenate(out, axis=0).astype(np.int32)
