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


def kuhn_mesh(d: int, N: int, L: int = 0, chunk: int = 1 << 20) -> Mesh:
    """Kuhn mesh with N cells per axis; coarse level has N >> L cells per axis.

    Elements are generated in chunks of cells so that 3D meshes with ~1e8 simplices stay
    within a few GB of temporaries."""
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    if N % (1 << L):
        raise ValueError("N must be divisible by 2^L")
    perms = permutations(d)
    nperm = perms.shape[0]
    h = (BOX_HI - BOX_LO) / N
    Nc = N >> L
    Lm = (1 << L) - 1
    eye = np.eye(d, dtype=np.int64)

    coords = BOX_LO + _lex_cells(N + 1, d).astype(np.float64) * h

    # permutation lookup: code(order) -> permutation index
    lut = np.full(d ** d, -1, dtype=np.int64)
    for i, p in enumerate(perms):
        c = 0
        for a in range(d):
            c = c * d + int(p[a])
        lut[c] = i
    pos_of = []
    for pi in perms:
        pos = np.empty(d, dtype=np.int64)
        pos[pi] = np.arange(d)
        pos_of.append(pos)

    C = N ** d
    elems = np.empty((C * nperm, d + 1), dtype=np.int32)
    centroids = np.empty((C * nperm, d), dtype=np.float64)
    coarse_of_elem = np.empty(C * nperm, dtype=np.int32)
    for c0 in range(0, C, chunk):
        c1 = min(C, c0 + chunk)
        cells = _lex_range(N, d, c0, c1)                       # (k, d)
        k = c1 - c0
        el = np.empty((k, nperm, d + 1), dtype=np.int64)
        cen = np.zeros((k, nperm, d), dtype=np.float64)
        for q, pi in enumerate(perms):
            v = cells.copy()
            el[:, q, 0] = _node_id(v, N)
            cen[:, q, :] += v
            for j in range(d):
                v = v + eye[pi[j]]
                el[:, q, j + 1] = _node_id(v, N)
                cen[:, q, :] += v
        elems[c0 * nperm:c1 * nperm] = el.reshape(-1, d + 1)
        centroids[c0 * nperm:c1 * nperm] = (BOX_LO + cen / (d + 1) * h).reshape(-1, d)
        # nesting map: coarse cell and coarse permutation of each fine simplex
        local = cells & Lm
        clin = np.zeros(k, dtype=np.int64)
        stride = 1
        for a in range(d):
            clin += (cells[:, a] >> L) * stride
            stride *= Nc
        co = np.empty((k, nperm), dtype=np.int64)
        for q in range(nperm):
            # key_a = local_a*(d+1) + (d - pos(a)); the coarse simplex orders axes by key
            key = local * (d + 1) + (d - pos_of[q])[None, :]
            order = np.argsort(-key, axis=1, kind="stable")
            code = np.zeros(k, dtype=np.int64)
            for a in range(d):
                code = code * d + order[:, a]
            cperm = lut[code]
            assert (cperm >= 0).all()
            co[:, q] = clin * nperm + cperm
        coarse_of_elem[c0 * nperm:c1 * nperm] = co.reshape(-1)

    # coarse vertices (fine-node ids)
    ccells = _lex_cells(Nc, d)
    cverts = np.empty((ccells.shape[0], nperm, d + 1), dtype=np.int64)
    for q, pi in enumerate(perms):
        v = ccells << L
        cverts[:, q, 0] = _node_id(v, N)
        for j in range(d):
            v = v + (eye[pi[j]] << L)
            cverts[:, q, j + 1] = _node_id(v, N)
    coarse_verts = cverts.reshape(-1, d + 1).astype(np.int32)

    bfacets = _box_facets(d, N, perms)
    return Mesh(d=d, N=N, L=L, coords=coords, elems=elems, bfacets=bfacets,
                coarse_of_elem=coarse_of_elem, coarse_verts=coarse_verts,
                centroids=centroids)


def _lex_range(N: int, d: int, c0: int, c1: int) -> np.ndarray:
    lin = np.arange(c0, c1, dtype=np.int64)
    idx = np.empty((lin.size, d), dtype=np.int64)
    rem = lin
    for a in range(d):
        idx[:, a] = rem % N
        rem = rem // N
    return idx


def _simplex_nodes(cells, pi, N, d):
    eye = np.eye(d, dtype=np.int64)
    out = np.empty((cells.shape[0], d + 1), dtype=np.int64)
    v = cells.copy()
    out[:, 0] = _node_id(v, N)
    for j in range(d):
        v = v + eye[pi[j]]
        out[:, j + 1] = _node_id(v, N)
    return out


def _box_facets(d, N, perms):
    """Facets on the box surface.

    On the face x_a = min, the simplices with pi(d-1) = a have the facet opposite their
    last vertex there; on x_a = max, those with pi(0) = a have the facet opposite v0.
    """
    out = []
    face = _lex_cells(N, d - 1)                      # cells of one face, (N^{d-1}, d-1)
    for a in range(d):
        for side in (0, N - 1):
            cells = np.empty((face.shape[0], d), dtype=np.int64)
            others = [b for b in range(d) if b != a]
            for j, b in enumerate(others):
                cells[:, b] = face[:, j]
            cells[:, a] = side
            for pi in perms:
                if side == 0 and pi[d - 1] == a:
                    out.append(_simplex_nodes(cells, pi, N, d)[:, :d])
                if side == N - 1 and pi[0] == a:
                    out.append(_simplex_nodes(cells, pi, N, d)[:, 1:])
    return np.concatenate(out, axis=0).astype(np.int32)
