"""Split-field PML coefficients and the lossy target of Sec. III, as inputs.

Seeded-input side only (element classification by centroid, no method arithmetic).

App. A: the layer {rho1 <= max_k |x_k| <= rho2}; xi = varsigma in the layer (weight of the
mass matrix S in the p-equation), zeta^(k) = varsigma where rho1 <= |x_k| <= rho2 (the
diagonal T^(k) = zeta^(k) A in the q-equations), zero elsewhere.  Elements are classified
by their centroid.  The paper gives no values for rho1, rho2, varsigma: the defaults put
the layer outside the source circle (r = 1.4) up to the box surface (1.5), with
varsigma * dt well below 1 at every workload's time step.
Sec. III: conductivity sigma = 5 eps_r inside the target, 0 outside.
"""
from __future__ import annotations

import numpy as np

RHO1 = 1.42
RHO2 = 1.5
VARSIGMA = 40.0


def pml_coefficients(centroids: np.ndarray, rho1: float = RHO1, rho2: float = RHO2,
                     varsigma: float = VARSIGMA):
    """xi (m,) and zeta (m, d) for elements with the given centroids."""
    a = np.abs(np.asarray(centroids, dtype=np.float64))
    zeta = np.where((a >= rho1) & (a <= rho2), varsigma, 0.0)
    mx = a.max(axis=1)
    xi = np.where((mx >= rho1) & (mx <= rho2), varsigma, 0.0)
    return xi, zeta


def lossy_sigma(eps: np.ndarray, inside: np.ndarray, factor: float = 5.0) -> np.ndarray:
    """sigma = factor * eps_r on the target's elements, 0 elsewhere."""
    return np.where(inside, factor * np.asarray(eps, dtype=np.float64), 0.0)
