"""Tiny dense finite-element assembly for brute-force checks of the oracle.

Built from the definitions of App. A directly and by different means than the oracle:
P1 basis gradients by solving the Vandermonde system [1 x] c = e_a, consistent mass by
the exact quadrature rule int phi_a phi_b = |T| (1 + delta_ab) / ((d+1)(d+2)), row-sum
lumped afterwards, and the matrices A, B^(k), C, R as dense arrays.  Only for meshes of a
few dozen nodes.
"""
from __future__ import annotations

import math

import numpy as np


def element_data(coords, elems):
    d = coords.shape[1]
    vols, grads = [], []
    for e in elems:
        X = coords[e]                                  # (d+1, d)
        V = np.hstack([np.ones((d + 1, 1)), X])        # rows: [1, x_a]
        Cf = np.linalg.solve(V, np.eye(d + 1))         # column a: coefficients of phi_a
        grads.append(Cf[1:, :].T)                      # (d+1, d)
        vols.append(abs(np.linalg.det(V)) / math.factorial(d))
    return np.array(vols), np.array(grads)


def assemble(coords, elems, eps, sigma=None, bfacets=None, admittance=None):
    """Dense A (m), B (d, m, n), lumped C (n), lumped R+boundary (n), stiffness K."""
    n, d = coords.shape
    m = elems.shape[0]
    vol, grad = element_data(coords, elems)
    A = vol.copy()
    B = np.zeros((d, m, n))
    Cc = np.zeros((n, n))
    Rc = np.zeros((n, n))
    for t, e in enumerate(elems):
        for a in range(d + 1):
            B[:, t, e[a]] += vol[t] * grad[t, a]
        loc = vol[t] * (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
        Cc[np.ix_(e, e)] += eps[t] * loc
        if sigma is not None:
            Rc[np.ix_(e, e)] += sigma[t] * loc
    Ml = Cc.sum(axis=1)
    r = Rc.sum(axis=1)
    if bfacets is not None:
        for f, fac in enumerate(bfacets):
            X = coords[fac]
            if d == 2:
                meas = np.linalg.norm(X[1] - X[0])
            else:
                meas = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
            # consistent boundary mass over F, then row-sum lumping
            locb = meas * (np.ones((d, d)) + np.eye(d)) / (d * (d + 1))
            y = 1.0 if admittance is None else admittance[f]
            r[fac] += y * locb.sum(axis=1)
    K = sum(B[k].T @ np.diag(1.0 / A) @ B[k] for k in range(d))
    return A, B, Ml, r, K


def point_weights(coords, elems, x):
    """Barycentric weights of point x in the first element that contains it."""
    d = coords.shape[1]
    for e in elems:
        V = np.hstack([np.ones((d + 1, 1)), coords[e]])
        lam = np.linalg.solve(V.T, np.concatenate([[1.0], x]))
        if lam.min() >= -1e-12:
            w = np.zeros(coords.shape[0])
            w[e] = lam
            return w
    raise ValueError("point outside mesh")


def leapfrog_dense(A, B, Ml, r, dt, n_steps, f_series, rec_w, p0=None, q0=None, T=None):
    """Eqs. leap-frog1/2 as dense matrix algebra with midpoint damping:
    q <- q + dt A^-1 (B p - T q) ;  (M + dt r/2) p' = (M - dt r/2) p + dt (f - sum B^T q),
    T: (d, m, m) dense T^(k) matrices or None."""
    d, m, n = B.shape
    p = np.zeros(n) if p0 is None else p0.copy()
    q = np.zeros((d, m)) if q0 is None else q0.copy()
    out = np.zeros((rec_w.shape[0], n_steps))
    lo = np.diag(Ml - 0.5 * dt * r)
    hi_inv = np.diag(1.0 / (Ml + 0.5 * dt * r))
    for l in range(n_steps):
        for k in range(d):
            tq = 0.0 if T is None else T[k] @ q[k]
            q[k] = q[k] + dt * (B[k] @ p - tq) / A
        s = sum(B[k].T @ q[k] for k in range(d))
        p = hi_inv @ (lo @ p + dt * (f_series[l] - s))
        out[:, l] = rec_w @ p
    return out, p, q
