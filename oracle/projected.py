"""FP64 reference of the projected data and its Jacobian (Sec. II-F).

Test infrastructure only.

Inner products over the measurement interval [0, T], T = N dt:
    <a, b>_1 = int_0^T a b dt,      <a, b>_2 = (1/T) int_0^T t a b dt,
evaluated on the sampled traces.  Reading: sample k holds the trace at
t_k = (s_k + 1) dt (trace[l] is the field after step l), and the integrals use the
rectangle rule on the sample grid with widths w_k = t_k - t_{k-1}, t_{-1} = 0.  So
<a, b>_j = sum_k q_j[k] a_k b_k with q_1 = w and q_2 = t w / T.

Projected data per trace i: y^(j)_i = <u_i, u_i>_j (measured with itself) and
y0^(j)_i = <u_i, u0_i>_j (measured with simulated); Jacobian rows
d y0^(j)_i / dc = <u_i, d u0_i / dc>_j, i.e. the time-weighted sum of the trace's J rows.
"""
from __future__ import annotations

import numpy as np


def quadrature(sample_steps, dt, n_steps):
    """(q, t): q (2, n_samples) weights of <.,.>_1 and <.,.>_2, t the sample times."""
    t = (np.asarray(sample_steps, dtype=np.float64) + 1.0) * dt
    w = np.diff(np.concatenate([[0.0], t]))
    T = n_steps * dt
    return np.stack([w, t * w / T]), t


def inner(a, b, q):
    """<a, b>_j for every j (rows of q); a, b (..., n_samples) -> (..., n_proj)."""
    return np.einsum("jk,...k,...k->...j", q, np.asarray(a, float), np.asarray(b, float))


def projected_data(u, u0, q):
    """u, u0: (n_traces, n_samples) measured and simulated sampled traces.
    Returns y, y0 of shape (n_traces, n_proj)."""
    return inner(u, u, q), inner(u, u0, q)


def projected_jacobian(J, u, q):
    """J: (n_traces * n_samples, M) rows ordered (trace, sample); u (n_traces, n_samples).
    Returns P (n_traces * n_proj, M), rows ordered (trace, projection)."""
    u = np.asarray(u, dtype=np.float64)
    nt, ns = u.shape
    Jr = np.asarray(J, dtype=np.float64).reshape(nt, ns, -1)
    P = np.einsum("jk,ik,ikm->ijm", q, u, Jr)
    return P.reshape(nt * q.shape[0], -1)
