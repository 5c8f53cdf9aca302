"""FP64 reference of the regularised-deconvolution route to the multigrid Jacobian
(App. A-2, steps (1)-(4), with the coarse-node source of App. A-3).

Test infrastructure only.

Per source s and receiver r:
  (1) source at x_s: record the auxiliary source series h_v(l) = b_v(l) =
      -(p_{l+1,v} - p_{l,v})/dt at every coarse node v;
  (2) the same source function at the receiver x_r: record p~_v(l) = p_{l+1,v} at v;
  (3) Tikhonov-regularised deconvolution p~ = g~ * f~ for the Green's function g~;
  (4) by reciprocity, the receiver's response to the auxiliary source at v is
      d~_v = g~_v * h_v; J[(s, r, k), j] = |T'_j|/(d+1) sum_{v in vert(T'_j)} d~_v(l_k).
Readings (the paper gives neither the discretisation nor delta): (3) is done on the
recorded window of N samples, zero-padded to a length L >= 2N, in the discrete Fourier
domain,  G = conj(F) P / (|F|^2 + delta max|F|^2),  g~ = the first N samples of the
inverse transform; convolutions are causal and truncated to N samples.  With delta = 0
and a source function whose spectrum has no zeros, g~ is the discrete impulse response
wherever the response has died out inside the window, and the route equals the
reciprocity Jacobian J2 of eq. approx_2.
"""
from __future__ import annotations

import numpy as np


def pad_length(N: int) -> int:
    """Transform length: the smallest power of two >= 2N."""
    L = 1
    while L < 2 * N:
        L *= 2
    return L


def tikhonov_deconvolve(p, f, delta, L=None):
    """p: (..., N) responses, f: (N,) source function -> g~ (..., N)."""
    p = np.asarray(p, dtype=np.float64)
    N = p.shape[-1]
    L = pad_length(N) if L is None else L
    F = np.fft.rfft(np.asarray(f, dtype=np.float64)[:N], n=L)
    F2 = np.abs(F) ** 2
    H = np.conj(F) / (F2 + delta * F2.max())
    return np.fft.irfft(np.fft.rfft(p, n=L, axis=-1) * H, n=L, axis=-1)[..., :N]


def causal_convolve(a, b):
    """(a * b)(l) = sum_{m <= l} a(l - m) b(m) for l < N, along the last axis."""
    N = a.shape[-1]
    out = np.empty(np.broadcast_shapes(a.shape, b.shape))
    for idx in np.ndindex(out.shape[:-1]):
        out[idx] = np.convolve(a[idx if a.ndim > 1 else ()], b[idx if b.ndim > 1 else ()])[:N]
    return out


def jacobian_deconv(o, src, rec, wavelet, dt, n_steps, sample_steps, delta, L=None):
    """Rows (s*n_rec + r)*K + k, columns the coarse elements (as mgrt_jacobian_coarse)."""
    d = o.d
    src = np.asarray(src, dtype=np.float64).reshape(-1, d)
    rec = np.asarray(rec, dtype=np.float64).reshape(src.shape[0], -1, d)
    cnodes, cinv = np.unique(o.coarse_verts, return_inverse=True)
    cinv = cinv.reshape(o.coarse_verts.shape)
    wgt = o.coarse_volume() / (d + 1)
    ss = np.asarray(sample_steps)
    f = np.asarray(wavelet, dtype=np.float64)[:n_steps]
    blocks = []
    for s in range(src.shape[0]):
        h = o.record_velocity(src[s], wavelet, dt, n_steps, cnodes).T          # (1): (nc, N)
        for r in range(rec.shape[1]):
            pt = o.record_field(rec[s, r], wavelet, dt, n_steps, cnodes).T     # (2): (nc, N)
            g = tikhonov_deconvolve(pt, f, delta, L)                           # (3)
            dd = causal_convolve(g, h)[:, ss]                                  # (4): (nc, K)
            blocks.append(np.einsum("j,jvk->kj", wgt, dd[cinv]))               # (K, M)
    return np.concatenate(blocks, axis=0)
