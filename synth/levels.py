"""Two nested inversion levels T' and T'' (Sec. II-D, Fig. 3), as inputs.

Seeded-input side only: connectivity and index maps, no method arithmetic.  T' is a Kuhn
mesh with Nc cells per axis (the inversion level of the multigrid Jacobian) and T'' the
same box with Nc / 2 cells per axis: every T'' simplex is the union of 2^d T' simplices
(4 triangles in 2D, 8 tetrahedra in 3D), the regular edge-halving refinement.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mesh import kuhn_mesh


@dataclass
class TwoLevel:
    d: int
    coords: np.ndarray    # (n, d) vertices of the T' grid
    verts1: np.ndarray    # (M, d+1) int32 vertex ids of the T' simplices
    verts2: np.ndarray    # (M2, d+1) int32 vertex ids of the T'' simplices
    parent: np.ndarray    # (M,) int32 nesting map T' -> T''

    @property
    def M(self) -> int:
        return self.verts1.shape[0]

    @property
    def M2(self) -> int:
        return self.verts2.shape[0]


def two_level(d: int, Nc: int) -> TwoLevel:
    """T' with Nc cells per axis (element ids as the coarse ids of kuhn_mesh(d, N, L) with
    N >> L == Nc) and T'' with Nc / 2."""
    t = kuhn_mesh(d, Nc, 1)
    return TwoLevel(d=d, coords=t.coords, verts1=t.elems, verts2=t.coarse_verts,
                    parent=t.coarse_of_elem)


def keep_third(M2: int) -> int:
    """Number of T'' elements whose fine fluctuations are kept: the largest third."""
    return (M2 + 2) // 3
