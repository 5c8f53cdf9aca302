"""Seeded synthetic asteroid bodies and element permittivities.

Seeded-input side only.  The paper's own target (Sec. III, Fig. 3 left: an irregular
body with a surface layer and voids) exists only as a figure, so a seeded star-shaped
body stands in for it, with the permittivity contrast the paper uses (body 4, voids 1,
vacuum 1 outside) plus a denser core.

Element classification is by centroid, with precedence void > core > body > vacuum.
Optional noise U(-a, a) is added to every element inside the body (core and voids
included) after classification; vacuum stays exactly 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EPS_VACUUM = 1.0
EPS_BODY = 4.0
EPS_CORE = 6.0
EPS_VOID = 1.0
CORE_RADIUS = 0.3


@dataclass
class Body2D:
    a: np.ndarray            # star amplitudes a_k, k = 2..6
    phi: np.ndarray          # phases
    void_c: np.ndarray       # (nv, 2) centres
    void_ax: np.ndarray      # (nv, 2) semi-axes
    void_rot: np.ndarray     # (nv,) orientation angle

    def radius(self, theta):
        k = np.arange(2, 7)[:, None]
        return 1.0 + 0.15 * np.sum(self.a[:, None] * np.cos(k * theta[None, :] + self.phi[:, None]),
                                   axis=0)

    def inside(self, x):
        r = np.hypot(x[:, 0], x[:, 1])
        th = np.arctan2(x[:, 1], x[:, 0])
        return r < self.radius(th)

    def in_void(self, x):
        out = np.zeros(x.shape[0], dtype=bool)
        for c, ax, rot in zip(self.void_c, self.void_ax, self.void_rot):
            y = x - c
            cr, sr = np.cos(rot), np.sin(rot)
            u = cr * y[:, 0] + sr * y[:, 1]
            v = -sr * y[:, 0] + cr * y[:, 1]
            out |= (u / ax[0]) ** 2 + (v / ax[1]) ** 2 < 1.0
        return out


def make_body2d(seed: int, n_voids: int) -> Body2D:
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.3, size=5)
    phi = rng.uniform(0.0, 2 * np.pi, size=5)
    body = Body2D(a=a, phi=phi, void_c=np.zeros((0, 2)), void_ax=np.zeros((0, 2)),
                  void_rot=np.zeros(0))
    cs, axs, rots = [], [], []
    while len(cs) < n_voids:
        ax = rng.uniform(0.05, 0.15, size=2)
        rot = rng.uniform(0.0, np.pi)
        c = rng.uniform(-1.15, 1.15, size=2)
        # accept only if the whole ellipse lies inside the body
        t = np.linspace(0, 2 * np.pi, 64, endpoint=False)
        pts = np.stack([ax[0] * np.cos(t), ax[1] * np.sin(t)], axis=1)
        cr, sr = np.cos(rot), np.sin(rot)
        pts = np.stack([cr * pts[:, 0] - sr * pts[:, 1], sr * pts[:, 0] + cr * pts[:, 1]], axis=1) + c
        if body.inside(pts).all():
            cs.append(c); axs.append(ax); rots.append(rot)
    body.void_c = np.array(cs).reshape(-1, 2)
    body.void_ax = np.array(axs).reshape(-1, 2)
    body.void_rot = np.array(rots)
    return body


def _real_sh_basis(lmax_lo, lmax_hi, theta, phi):
    """Real spherical-harmonic-like basis P_l^m(cos theta) * cos/sin(m phi), l = lo..hi.

    Unnormalised associated Legendre functions are enough: the coefficients are random
    and the sum is rescaled to a fixed maximum afterwards.
    """
    from scipy.special import lpmv
    x = np.cos(theta)
    cols = []
    for l in range(lmax_lo, lmax_hi + 1):
        for mm in range(0, l + 1):
            P = lpmv(mm, l, x)
            cols.append(P * np.cos(mm * phi))
            if mm > 0:
                cols.append(P * np.sin(mm * phi))
    return np.stack(cols, axis=-1)


@dataclass
class Body3D:
    coef: np.ndarray
    scale: float
    void_c: np.ndarray
    void_ax: np.ndarray
    void_R: np.ndarray       # (nv, 3, 3) rotation matrices

    def radius(self, theta, phi):
        return 1.0 + self.scale * (_real_sh_basis(2, 4, theta, phi) @ self.coef)

    def inside(self, x):
        r = np.linalg.norm(x, axis=1)
        # |radius - 1| <= scale * max|sum| = 0.15: only the shell needs the harmonics
        out = r < 1.0 - 0.15
        shell = np.nonzero((r >= 1.0 - 0.15) & (r <= 1.0 + 0.15))[0]
        if shell.size:
            xs, rs = x[shell], r[shell]
            theta = np.arccos(np.clip(xs[:, 2] / np.maximum(rs, 1e-300), -1.0, 1.0))
            phi = np.arctan2(xs[:, 1], xs[:, 0])
            out[shell] = rs < self.radius(theta, phi)
        return out

    def in_void(self, x):
        out = np.zeros(x.shape[0], dtype=bool)
        for c, ax, R in zip(self.void_c, self.void_ax, self.void_R):
            y = (x - c) @ R
            out |= np.sum((y / ax) ** 2, axis=1) < 1.0
        return out


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def make_body3d(seed: int, n_voids: int) -> Body3D:
    rng = np.random.default_rng(seed)
    nb = sum(2 * l + 1 for l in range(2, 5))
    coef = rng.uniform(-1.0, 1.0, size=nb)
    th, ph = np.meshgrid(np.linspace(0, np.pi, 64), np.linspace(0, 2 * np.pi, 128, endpoint=False),
                         indexing="ij")
    s = _real_sh_basis(2, 4, th.ravel(), ph.ravel()) @ coef
    scale = 0.15 / np.max(np.abs(s))
    body = Body3D(coef=coef, scale=scale, void_c=np.zeros((0, 3)), void_ax=np.zeros((0, 3)),
                  void_R=np.zeros((0, 3, 3)))
    cs, axs, Rs = [], [], []
    u = rng.normal(size=(200, 3))
    sphere = u / np.linalg.norm(u, axis=1, keepdims=True)
    while len(cs) < n_voids:
        ax = rng.uniform(0.05, 0.15, size=3)
        R = _random_rotation(rng)
        c = rng.uniform(-1.15, 1.15, size=3)
        pts = (sphere * ax) @ R.T + c
        if body.inside(pts).all():
            cs.append(c); axs.append(ax); Rs.append(R)
    body.void_c = np.array(cs).reshape(-1, 3)
    body.void_ax = np.array(axs).reshape(-1, 3)
    body.void_R = np.array(Rs).reshape(-1, 3, 3)
    return body


def element_permittivity(centroids: np.ndarray, body, noise: float = 0.0,
                         noise_seed: int | None = None, chunk: int = 1 << 22) -> np.ndarray:
    """Relative permittivity per element by centroid class (void > core > body > vacuum)."""
    m = centroids.shape[0]
    eps = np.full(m, EPS_VACUUM, dtype=np.float64)
    inside = np.zeros(m, dtype=bool)
    for s in range(0, m, chunk):
        x = centroids[s:s + chunk]
        ins = body.inside(x)
        core = np.linalg.norm(x, axis=1) < CORE_RADIUS
        void = body.in_void(x)
        e = np.where(ins, EPS_BODY, EPS_VACUUM)
        e = np.where(ins & core, EPS_CORE, e)
        e = np.where(ins & void, EPS_VOID, e)
        eps[s:s + chunk] = e
        inside[s:s + chunk] = ins
    if noise > 0.0:
        rng = np.random.default_rng(noise_seed)
        dn = rng.uniform(-noise, noise, size=m)
        eps = np.where(inside, eps + dn, eps)
    return eps


def prior_permittivity(coarse_centroids: np.ndarray, body) -> np.ndarray:
    """A priori coarse permittivity: 4 in coarse elements whose centroid is in the body."""
    return np.where(body.inside(coarse_centroids), EPS_BODY, EPS_VACUUM).astype(np.float64)
