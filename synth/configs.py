"""Named seeded workloads.

Every array a workload needs (mesh, permittivity, acquisition geometry, wavelet, time
step) comes from here, identically for the GPU library and for the oracle.

Workloads (the paper's target and meshes exist only as figures, so seeded star-shaped
bodies on nested Kuhn meshes stand in for them):

=========  ==  ======  ===========  =====================  ========  =================
name       d   cells   coarse lvl   sources x receivers    steps     notes
=========  ==  ======  ===========  =====================  ========  =================
c1         2   128^2   16^2 (L=3)   1 x 1 monostatic        4,000    FP64, 3 voids
c2         2   1024^2  64^2 (L=4)   64 x 1 monostatic      16,000    8 voids, eps noise
c3         2   1024^2  64^2 (L=4)   64 x 1 monostatic      16,000    Jacobian, 512 samples
c4         3   128^3   16^3 (L=3)   32 x 1 monostatic       6,000    5 voids
c5         3   256^3   32^3 (L=3)   16 x 2 bistatic        12,000    misfit gradient
=========  ==  ======  ===========  =====================  ========  =================

``make(name, **overrides)`` accepts smaller N / n_src / n_steps / L for test-sized
versions with the same construction.  ``pml=True`` gives the paper's boundary and losses
instead: the split-field PML of App. A in a layer at the box surface (no first-order
absorbing boundary: the outer surface is then natural) and sigma = 5 eps_r in the target.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import acquisition as acq
from . import body as bd
from . import pml as pml_in
from .mesh import Mesh, kuhn_mesh

SPECS = {
    "c1": dict(d=2, N=128, L=3, seed=1, n_voids=3, noise=0.0, n_src=1, n_rec=1,
               n_steps=4000, n_samples=512),
    "c2": dict(d=2, N=1024, L=4, seed=2, n_voids=8, noise=0.1, n_src=64, n_rec=1,
               n_steps=16000, n_samples=512),
    "c3": dict(d=2, N=1024, L=4, seed=2, n_voids=8, noise=0.1, n_src=64, n_rec=1,
               n_steps=16000, n_samples=512),
    "c4": dict(d=3, N=128, L=3, seed=4, n_voids=5, noise=0.0, n_src=32, n_rec=1,
               n_steps=6000, n_samples=512),
    "c5": dict(d=3, N=256, L=3, seed=5, n_voids=5, noise=0.0, n_src=16, n_rec=2,
               n_steps=12000, n_samples=512),
}

NOISE_SEED = 3          # data noise and random column choices of the differentiation workload
DATA_NOISE = 0.01       # 1% peak-relative Gaussian noise
TV_ALPHA = 0.01         # Sec. III: alpha = beta = 0.01 for full-wave data
TV_BETA = 0.01


@dataclass
class Problem:
    name: str
    mesh: Mesh
    eps: np.ndarray              # (m,) relative permittivity per fine element
    sigma: np.ndarray | None     # (m,) conductivity or None (= 0)
    src: np.ndarray              # (n_src, d)
    rec: np.ndarray              # (n_src, n_rec, d)
    dt: float
    n_steps: int
    wavelet: np.ndarray          # (n_steps,) w_l = w(l dt)
    f0: float
    body: object
    n_samples: int
    spec: dict = field(default_factory=dict)
    pml: tuple | None = None     # (xi (m,), zeta (m, d)) split-field PML, or None

    @property
    def sample_steps(self) -> np.ndarray:
        return acq.sample_steps(self.n_steps, self.n_samples)


def make(name: str, pml: bool = False, **over) -> Problem:
    spec = dict(SPECS[name])
    spec.update(over)
    d, N, L = spec["d"], spec["N"], spec["L"]
    mesh = kuhn_mesh(d, N, L)
    if d == 2:
        body = bd.make_body2d(spec["seed"], spec["n_voids"])
    else:
        body = bd.make_body3d(spec["seed"], spec["n_voids"])
    eps = bd.element_permittivity(mesh.centroids, body, noise=spec["noise"],
                                  noise_seed=spec["seed"] + 1000)
    n_src = spec["n_src"]
    src = acq.circle_points(n_src) if d == 2 else acq.sphere_points(n_src)
    rec = acq.monostatic(src) if spec["n_rec"] == 1 else acq.bistatic_antipodal(src)
    dt = acq.time_step(d, mesh.h, float(eps.min()))
    f0 = acq.wavelet_f0()
    wav = acq.sample_wavelet(dt, spec["n_steps"], f0)
    sigma, layer = None, None
    if pml:
        layer = pml_in.pml_coefficients(mesh.centroids)
        sigma = pml_in.lossy_sigma(eps, body.inside(mesh.centroids))
        spec["pml"] = dict(rho1=pml_in.RHO1, rho2=pml_in.RHO2, varsigma=pml_in.VARSIGMA)
    return Problem(name=name, mesh=mesh, eps=eps, sigma=sigma, src=src, rec=rec, dt=dt,
                   n_steps=spec["n_steps"], wavelet=wav, f0=f0, body=body,
                   n_samples=spec["n_samples"], spec=spec, pml=layer)


def coarse_centroids(mesh: Mesh) -> np.ndarray:
    return mesh.coords[mesh.coarse_verts].mean(axis=1)


def prior_eps_fine(p: Problem) -> np.ndarray:
    """Fine-element permittivity of the linearisation point: 4 on coarse elements whose
    centroid is inside the body, 1 elsewhere."""
    cp = bd.prior_permittivity(coarse_centroids(p.mesh), p.body)
    return cp[p.mesh.coarse_of_elem]


def fd_columns(M: int, k: int = 32, seed: int = NOISE_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(M, size=k, replace=False)).astype(np.int64)
