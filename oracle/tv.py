"""Dense FP64 reference of the TV-regularised iteration (Sec. II-C, eq. tv_iteration).

Test infrastructure only.

    z_{l+1} = (L^T L + alpha D^T Gamma_l D)^{-1} L^T r,   z = x - x0,  r = y - y0,
    Gamma_0 = I,  Gamma_l = diag(1 / max(|D z_l|, tau)),  tau = tau_rel * max|D z_l|.

The paper writes D Gamma D; D^T is used so that a non-symmetric D is also handled (they
agree for the symmetric D of eq. d_mat).  Zero entries of |D z| would make Gamma
infinite, hence the floor tau; when D z vanishes altogether (r = 0) Gamma = I.  Each linear system is solved by a dense Cholesky
factorisation of the normal matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def tv_iterates(L, r, D, alpha, iters, tau_rel=1e-8):
    L = np.asarray(L, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    LtL = L.T @ L
    Ltr = L.T @ r
    z = np.zeros(L.shape[1])
    out = []
    for l in range(iters):
        a = np.abs(D @ z)
        if l == 0 or a.max() == 0.0:
            g = np.ones(D.shape[0])
        else:
            g = 1.0 / np.maximum(a, tau_rel * a.max())
        A = LtL + alpha * (D.T @ (g[:, None] * D))
        z = sla.cho_solve(sla.cho_factor(A, lower=True), Ltr)
        out.append(z.copy())
    return out
