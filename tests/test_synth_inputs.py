"""Checks of the seeded input generator (meshes, nesting, acquisition) and the paper's
printed values (tests/golden/paper_values.json)."""
import json
import os

import numpy as np
import pytest

from synth import acquisition as acq
from synth import configs
from synth.mesh import kuhn_mesh

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_blackman_harris_window_values():
    g = GOLD["blackman_harris"]
    T = g["window_length"]
    assert acq.blackman_harris(np.array([0.0]), T)[0] == pytest.approx(g["value_at_start"], abs=1e-12)
    assert acq.blackman_harris(np.array([T / 2]), T)[0] == pytest.approx(g["value_at_centre"], abs=1e-12)
    assert acq.blackman_harris(np.array([1.5 * T]), T)[0] == 0.0


def test_paper_time_grid_arithmetic():
    g = GOLD["time_grid"]
    assert round(g["T"] / g["dt"]) == g["steps"]
    assert round(g["sampling"] / g["dt"]) == g["steps_per_sample"]


@pytest.mark.parametrize("d,N,L", [(2, 16, 2), (3, 8, 1), (3, 8, 2)])
def test_nesting_is_exact(d, N, L):
    """Every fine simplex lies inside its coarse simplex (all its vertices have
    barycentric coordinates in [0, 1] w.r.t. the coarse vertices), and each coarse
    simplex holds (2^d)^L fine ones (regular edge-halving refinement, Fig. 2)."""
    ms = kuhn_mesh(d, N, L)
    cnt = np.bincount(ms.coarse_of_elem, minlength=ms.n_coarse)
    assert np.all(cnt == (2 ** d) ** L)
    X = ms.coords[ms.coarse_verts[ms.coarse_of_elem]]          # (m, d+1, d)
    V = np.concatenate([np.ones(X.shape[:2] + (1,)), X], axis=2)
    Y = ms.coords[ms.elems]                                      # (m, d+1, d)
    rhs = np.concatenate([np.ones(Y.shape[:2] + (1,)), Y], axis=2)
    lam = np.linalg.solve(np.transpose(V, (0, 2, 1)), np.transpose(rhs, (0, 2, 1)))
    assert lam.min() > -1e-12 and lam.max() < 1 + 1e-12


def test_table_v_sizes_follow_four_children_per_triangle():
    """Table V: single- vs dual-resolution unknowns differ by the 4 children of a
    triangle under edge halving; the 2D generator nests the same way."""
    t = GOLD["table_v"]
    assert t["single_res_unknowns"] == 4 * t["dual_res_unknowns"]
    assert t["full_MB"][0] / t["full_MB"][1] == pytest.approx(4.0, rel=0.01)
    assert t["projected_MB"][0] / t["projected_MB"][1] == pytest.approx(4.0, rel=0.01)
    ms = kuhn_mesh(2, 8, 1)
    assert ms.m == 4 * ms.n_coarse


@pytest.mark.parametrize("d", [2, 3])
def test_box_facets(d):
    N = 5
    ms = kuhn_mesh(d, N, 0)
    x = ms.coords[ms.bfacets]                                    # (nb, d, d)
    on_face = np.any(np.all(np.isclose(np.abs(x), 1.5), axis=1), axis=1)
    assert on_face.all()
    per_face = N ** (d - 1) * (1 if d == 2 else 2)
    assert ms.bfacets.shape[0] == 2 * d * per_face
    # every box facet is a facet of some element
    faces = set()
    for e in ms.elems:
        for k in range(d + 1):
            faces.add(tuple(sorted(np.delete(e, k))))
    assert all(tuple(sorted(f)) in faces for f in ms.bfacets)


def test_acquisition_layout():
    src = acq.circle_points(64)
    assert np.allclose(src[0], [0.0, 1.4], atol=1e-15)
    assert np.allclose(np.hypot(src[:, 0], src[:, 1]), 1.4)
    s3 = acq.sphere_points(16)
    assert np.allclose(np.linalg.norm(s3, axis=1), 1.4)
    rec = acq.bistatic_antipodal(s3)
    assert np.allclose(rec[:, 1], -s3)
    ss = acq.sample_steps(16000, 512)
    assert ss[-1] == 15999 and ss.size == 512 and np.all(np.diff(ss) > 0)


def test_config_c1_inputs():
    p = configs.make("c1")
    assert (p.mesh.n, p.mesh.m) == (16641, 32768)
    assert set(np.unique(p.eps)) <= {1.0, 4.0, 6.0}
    assert p.n_steps == 4000 and p.wavelet.shape == (4000,)
    assert p.dt == pytest.approx(acq.COURANT[2] * 3 / 128)
