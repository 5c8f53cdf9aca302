"""ctypes front end of the FP64 oracle (test infrastructure only).

Each method names the passage of the paper it follows; the arithmetic is in
``mgrt_oracle.c``.  Arrays are NumPy, FP64, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from .build import ensure_built

_LIB = None

dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
i64 = C.c_int64


def _opt(t):
    """nullable ndpointer"""
    base = np.ctypeslib.ndpointer(dtype=t, flags="C_CONTIGUOUS")

    def from_param(cls, obj):
        if obj is None:
            return None
        return base.from_param(obj)
    return type("Opt" + base.__name__, (base,), {"from_param": classmethod(from_param)})


odp = _opt(np.float64)
oip = _opt(np.int32)


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    lib = C.CDLL(ensure_built())
    lib.orc_geometry.argtypes = [C.c_int, i64, dp, ip, dp, dp]
    lib.orc_lumped_mass.argtypes = [C.c_int, i64, i64, ip, dp, odp, dp]
    lib.orc_boundary_damping.argtypes = [C.c_int, i64, dp, i64, ip, odp, dp]
    lib.orc_locate.argtypes = [C.c_int, dp, i64, ip, i64, dp, ip, dp]
    lib.orc_apply_stiffness.argtypes = [C.c_int, i64, i64, ip, dp, dp, dp, dp]
    lib.orc_lambda_max.argtypes = [C.c_int, i64, i64, ip, dp, dp, dp, C.c_int,
                                   C.POINTER(C.c_double)]
    lib.orc_forward.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double, i64,
                                i64, oip, odp, odp, i64, i64, ip, dp, dp,
                                odp, odp, odp, odp, odp]
    lib.orc_tangent.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double, i64,
                                i64, ip, dp, dp, i64, i64, ip, dp, i64, dp, dp]
    lib.orc_complex_step.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double, i64,
                                     ip, dp, dp, i64, ip, dp, dp, C.c_double, dp]
    lib.orc_record_velocity.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double,
                                        i64, ip, dp, dp, i64, ip, dp]
    lib.orc_record_field.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double,
                                     i64, ip, dp, dp, i64, ip, dp]
    lib.orc_node_responses.argtypes = [C.c_int, i64, i64, ip, dp, dp, odp, dp, dp, C.c_double,
                                       i64, i64, ip, dp, i64, ip, dp, dp]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = None
    _LIB = lib
    return lib


def _c(a, t=np.float64):
    return np.ascontiguousarray(a, dtype=t)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


class Oracle:
    """Mixed-form FP64 reference for one mesh and one permittivity.

    Operators (App. A, eq. system1/2 matrices): element volumes |T| and P1 gradients,
    lumped eps-mass M_i = sum_T eps_T |T|/(d+1), lumped damping r = R_sigma + r_boundary,
    where the absorbing boundary adds Y |F|/d per facet node (Y = 1: the box surface is
    in vacuum).  Split-field PML (App. A, matrices S and T^(k)): pml = (xi, zeta) with xi
    (m,) the S weight, lumped into r like sigma (and, like it, taken at the midpoint), and
    zeta (m, d) the per-direction coefficients of T^(k) = zeta^(k) A in leap-frog1.
    """

    def __init__(self, d, coords, elems, eps, sigma=None, bfacets=None, admittance=None,
                 coarse_of_elem=None, coarse_verts=None, pml=None):
        self.lib = load_library()
        self.d = int(d)
        self.coords = _c(coords)
        self.elems = _c(elems, np.int32)
        self.n = self.coords.shape[0]
        self.m = self.elems.shape[0]
        self.vol = np.empty(self.m)
        self.grad = np.empty((self.m, self.d + 1, self.d))
        _check(self.lib.orc_geometry(self.d, self.m, self.coords, self.elems, self.vol,
                                     self.grad), "geometry")
        self.eps = _c(eps)
        self.M = np.empty(self.n)
        _check(self.lib.orc_lumped_mass(self.d, self.n, self.m, self.elems, self.vol,
                                        self.eps, self.M), "mass")
        self.r = np.zeros(self.n)
        if sigma is not None:
            rs = np.empty(self.n)
            self.lib.orc_lumped_mass(self.d, self.n, self.m, self.elems, self.vol, _c(sigma), rs)
            self.r += rs
        if bfacets is not None and len(bfacets):
            bf = _c(bfacets, np.int32)
            self.lib.orc_boundary_damping(self.d, self.n, self.coords, bf.shape[0], bf,
                                          None if admittance is None else _c(admittance),
                                          self.r)
        self.zeta = None
        if pml is not None:
            xi, zeta = pml
            rx = np.empty(self.n)
            self.lib.orc_lumped_mass(self.d, self.n, self.m, self.elems, self.vol, _c(xi), rx)
            self.r += rx
            self.zeta = _c(np.asarray(zeta).reshape(self.m, self.d))
        self.coarse_of_elem = None if coarse_of_elem is None else np.asarray(coarse_of_elem)
        self.coarse_verts = None if coarse_verts is None else np.asarray(coarse_verts)

    @classmethod
    def from_problem(cls, prob, eps=None, absorbing=True):
        ms = prob.mesh
        pml = getattr(prob, "pml", None)
        return cls(ms.d, ms.coords, ms.elems, prob.eps if eps is None else eps, prob.sigma,
                   ms.bfacets if absorbing and pml is None else None, None, ms.coarse_of_elem,
                   ms.coarse_verts, pml=pml)

    # ---------------------------------------------------------------- basic pieces
    @property
    def threads(self) -> int:
        return int(self.lib.orc_num_threads())

    def set_threads(self, n: int) -> None:
        """OpenMP threads of the oracle's later calls in this process."""
        self.lib.orc_set_threads(int(n))

    def locate(self, pts):
        """P1 point stencil (Sec. II-A point source): nodes and barycentric weights."""
        pts = _c(np.asarray(pts).reshape(-1, self.d))
        nodes = np.empty((pts.shape[0], self.d + 1), dtype=np.int32)
        w = np.empty((pts.shape[0], self.d + 1))
        _check(self.lib.orc_locate(self.d, self.coords, self.m, self.elems, pts.shape[0], pts,
                                   nodes, w), "locate")
        return nodes, w

    def apply_stiffness(self, p):
        out = np.empty(self.n)
        _check(self.lib.orc_apply_stiffness(self.d, self.n, self.m, self.elems, self.vol,
                                            self.grad, _c(p), out), "stiffness")
        return out

    def lambda_max(self, iters=400):
        out = C.c_double()
        _check(self.lib.orc_lambda_max(self.d, self.n, self.m, self.elems, self.vol, self.grad,
                                       self.M, iters, C.byref(out)), "lambda_max")
        return out.value

    def dmass(self, deps):
        """Derivative of the lumped mass along a fine-element permittivity direction."""
        out = np.empty(self.n)
        self.lib.orc_lumped_mass(self.d, self.n, self.m, self.elems, self.vol, _c(deps), out)
        return out

    # ---------------------------------------------------------------- forward (leap-frog1/2)
    def forward(self, src, rec, wavelet, dt, n_steps, p0=None, q0=None, want_state=False):
        """Traces (n_src, n_rec, n_steps) of independent point-source runs.

        src (n_src, d) points or None; rec (n_src, n_rec, d); wavelet (n_steps,) shared or
        (n_src, n_steps)."""
        d = self.d
        rec = np.asarray(rec, dtype=np.float64)
        if src is None:
            nsim = 1
            sn = sw = None
            wav, ws = None, 0
        else:
            src = np.asarray(src, dtype=np.float64).reshape(-1, d)
            nsim = src.shape[0]
            sn, sw = self.locate(src)
            wav = _c(wavelet)
            ws = 0 if wav.ndim == 1 else wav.shape[1]
        rec = rec.reshape(nsim, -1, d)
        nrec = rec.shape[1]
        rn, rw = self.locate(rec.reshape(-1, d))
        traces = np.empty((nsim, nrec, n_steps))
        pl = pp = ql = None
        if want_state:
            pl, pp, ql = np.empty(self.n), np.empty(self.n), np.empty((self.m, d))
        _check(self.lib.orc_forward(d, self.n, self.m, self.elems, self.vol, self.grad,
                                    self.zeta, self.M, self.r, float(dt), int(n_steps), nsim, sn, sw, wav,
                                    ws, nrec, rn, rw, traces,
                                    None if p0 is None else _c(p0),
                                    None if q0 is None else _c(q0), pl, pp, ql), "forward")
        if want_state:
            return traces, pl, pp, ql
        return traces

    def time_forward(self, src, rec, wavelet, dt, n_steps):
        t0 = time.perf_counter()
        tr = self.forward(src, rec, wavelet, dt, n_steps)
        return tr, time.perf_counter() - t0

    # ---------------------------------------------------------------- linearisation
    def coarse_direction(self, j):
        """Fine-element indicator of coarse element j (eps = sum_j c_j chi'_j, Sec. II-B)."""
        return (self.coarse_of_elem == j).astype(np.float64)

    def tangent(self, src, rec, wavelet, dt, n_steps, deps_list):
        """Exact Jacobian-vector products (eq. approx_1 with the exact auxiliary source):
        dtraces (n_src, ndir, n_rec, n_steps) for fine-element directions deps_list."""
        d = self.d
        src = np.asarray(src, dtype=np.float64).reshape(-1, d)
        nsim = src.shape[0]
        sn, sw = self.locate(src)
        wav = _c(wavelet)
        ws = 0 if wav.ndim == 1 else wav.shape[1]
        rec = np.asarray(rec, dtype=np.float64).reshape(nsim, -1, d)
        nrec = rec.shape[1]
        rn, rw = self.locate(rec.reshape(-1, d))
        dM = _c(np.stack([self.dmass(de) for de in deps_list]))
        out = np.empty((nsim, dM.shape[0], nrec, n_steps))
        _check(self.lib.orc_tangent(d, self.n, self.m, self.elems, self.vol, self.grad,
                                    self.zeta, self.M,
                                    self.r, float(dt), int(n_steps), nsim, sn, sw, wav, ws,
                                    nrec, rn, rw, dM.shape[0], dM, out), "tangent")
        return out

    def jacobian_exact(self, src, rec, wavelet, dt, n_steps, cols, sample_steps):
        """J1 columns (rows (s, r, k) = (s*n_rec + r)*n_samples + k), shape (rows, len(cols))."""
        dirs = [self.coarse_direction(j) for j in cols]
        tl = self.tangent(src, rec, wavelet, dt, n_steps, dirs)      # (S, C, R, N)
        tl = tl[..., np.asarray(sample_steps)]                        # (S, C, R, K)
        S, Cn, R, K = tl.shape
        return tl.transpose(0, 2, 3, 1).reshape(S * R * K, Cn)

    def complex_step_column(self, src, rec, wavelet, dt, n_steps, deps, delta=1e-30):
        d = self.d
        sn, sw = self.locate(np.asarray(src).reshape(1, d))
        rec = np.asarray(rec, dtype=np.float64).reshape(-1, d)
        rn, rw = self.locate(rec)
        out = np.empty((rec.shape[0], n_steps))
        _check(self.lib.orc_complex_step(d, self.n, self.m, self.elems, self.vol, self.grad,
                                         self.zeta, self.M, self.r, float(dt), int(n_steps), sn, sw,
                                         _c(wavelet), rec.shape[0], rn, rw, self.dmass(deps),
                                         float(delta), out), "complex_step")
        return out

    def record_field(self, src, wavelet, dt, n_steps, nodes):
        """p_{l+1} at the listed nodes for a point source at src, (n_steps, nnodes)."""
        sn, sw = self.locate(np.asarray(src).reshape(1, self.d))
        nodes = _c(nodes, np.int32)
        out = np.empty((n_steps, nodes.size))
        _check(self.lib.orc_record_field(self.d, self.n, self.m, self.elems, self.vol,
                                         self.grad, self.zeta, self.M, self.r, float(dt),
                                         int(n_steps), sn, sw, _c(wavelet), nodes.size, nodes,
                                         out), "record_field")
        return out

    def record_velocity(self, src, wavelet, dt, n_steps, nodes):
        sn, sw = self.locate(np.asarray(src).reshape(1, self.d))
        nodes = _c(nodes, np.int32)
        out = np.empty((n_steps, nodes.size))
        _check(self.lib.orc_record_velocity(self.d, self.n, self.m, self.elems, self.vol,
                                            self.grad, self.zeta, self.M, self.r, float(dt),
                                            int(n_steps),
                                            sn, sw, _c(wavelet), nodes.size, nodes, out),
               "record_velocity")
        return out

    def node_responses(self, nodes, series, rec, dt, n_steps):
        nodes = _c(nodes, np.int32)
        rec = np.asarray(rec, dtype=np.float64).reshape(-1, self.d)
        rn, rw = self.locate(rec)
        out = np.empty((nodes.size, rec.shape[0], n_steps))
        _check(self.lib.orc_node_responses(self.d, self.n, self.m, self.elems, self.vol,
                                           self.grad, self.zeta, self.M, self.r, float(dt),
                                           int(n_steps),
                                           nodes.size, nodes, _c(series), rec.shape[0], rn, rw,
                                           out), "node_responses")
        return out

    def coarse_volume(self):
        """|T'_j| of the coarse simplices from their vertex coordinates."""
        x = self.coords[self.coarse_verts]                 # (M, d+1, d)
        E = x[:, 1:, :] - x[:, :1, :]
        fact = 2.0 if self.d == 2 else 6.0
        return np.abs(np.linalg.det(E)) / fact

    def jacobian_mg(self, src, rec, wavelet, dt, n_steps, sample_steps, cols=None):
        """Multigrid Jacobian J2 (eq. approx_2, App. A-3) by brute force.

        For each source s and each coarse node i', one auxiliary run with the nodal
        source b_{i'}(l) = -(p_{l+1,i'} - p_{l,i'})/dt gives the receiver responses
        D_{i'}; then J2[:, j] = |T'_j|/(d+1) * sum of D over the d+1 vertices of T'_j
        (coarse mass derivative lumped to the vertices).  Rows (s*n_rec + r)*K + k.
        cols: optional subset of coarse columns (only their vertices are run)."""
        d = self.d
        src = np.asarray(src, dtype=np.float64).reshape(-1, d)
        rec = np.asarray(rec, dtype=np.float64).reshape(src.shape[0], -1, d)
        cverts = self.coarse_verts if cols is None else self.coarse_verts[np.asarray(cols)]
        cnodes, cinv = np.unique(cverts, return_inverse=True)
        cinv = cinv.reshape(cverts.shape)
        wgt = self.coarse_volume() / (d + 1)
        if cols is not None:
            wgt = wgt[np.asarray(cols)]
        ss = np.asarray(sample_steps)
        blocks = []
        for s in range(src.shape[0]):
            b = self.record_velocity(src[s], wavelet, dt, n_steps, cnodes)     # (N, nc)
            resp = self.node_responses(cnodes, _c(b.T), rec[s], dt, n_steps)   # (nc, R, N)
            resp = resp[:, :, ss]                                              # (nc, R, K)
            J = np.einsum("j,jvrk->rkj", wgt, resp[cinv])                      # (R, K, M)
            blocks.append(J.reshape(-1, J.shape[-1]))
        return np.concatenate(blocks, axis=0)

    def gradient_coarse(self, src, rec, wavelet, dt, n_steps, residual):
        """J1^T rho over all coarse columns by explicit transpose (small meshes only):
        grad_j = sum_{s,r,l} residual[s,r,l] * dtrace[s,r,l]/dc_j."""
        Mc = self.coarse_verts.shape[0]
        dirs = [self.coarse_direction(j) for j in range(Mc)]
        tl = self.tangent(src, rec, wavelet, dt, n_steps, dirs)       # (S, C, R, N)
        return np.einsum("scrn,srn->c", tl, np.asarray(residual))
