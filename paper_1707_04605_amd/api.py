"""Python front end of libmgrt: one method per C-ABI entry point, same names.

Arrays may be NumPy arrays or CPU torch tensors; outputs are NumPy arrays unless an
``out`` torch tensor on the GPU is given, in which case the library writes it directly
(device pointer).  Every step of the computation runs inside libmgrt; this module only
converts arguments.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import native
from .native import MgrtError, RunOpts, Timing


def _arr(x, dtype):
    if x is None:
        return None
    if hasattr(x, "detach"):            # torch tensor
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def _solver_code(solver):
    codes = {"auto": native.TV_AUTO, "cg": native.TV_CG}
    if solver not in codes:
        raise ValueError(f"solver must be one of {sorted(codes)}")
    return codes[solver]


def projection_weights(sample_steps, dt, n_steps):
    """Quadrature weights (2 x n_samples) of the inner products of Sec. II-F on the sample
    grid (mgrt_projection_weights), input of Context.project_rows."""
    lib = native.load()
    ss = _arr(sample_steps, np.int64)
    q = np.empty((2, ss.shape[0]))
    rc = lib.mgrt_projection_weights(_ptr(ss), ss.shape[0], float(dt), int(n_steps), _ptr(q))
    if rc != native.MGRT_OK:
        raise native.MgrtError(rc, "mgrt_projection_weights: bad sample steps, dt or n_steps")
    return q


class Context:
    """One libmgrt context (device + stream).  By default it launches on torch's
    current stream so that its work is ordered with torch's."""

    def __init__(self, device: int = 0, stream=None, use_torch_stream: bool = True):
        self.lib = native.load()
        self._h = C.c_void_p()
        if stream is None and use_torch_stream:
            stream = _torch_stream()
        rc = self.lib.mgrt_create(int(device), C.c_void_p(stream) if stream else None,
                                  C.byref(self._h))
        if rc != 0:
            raise MgrtError(rc, f"mgrt_create(device={device}) failed")
        self.device = int(device)
        self.dim = None
        self.n_coarse = 0
        self.n_elems = 0

    def close(self):
        if self._h:
            self.lib.mgrt_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.mgrt_last_error(self._h)
            raise MgrtError(rc, f"{what}: {msg.decode() if msg else ''}")

    # ------------------------------------------------------------------ setup
    def upload_mesh(self, dim, coords, elems, bfacets=None, admittance=None,
                    coarse_of_elem=None, coarse_verts=None):
        coords = _arr(coords, np.float64)
        elems = _arr(elems, np.int32)
        bf = _arr(bfacets, np.int32)
        adm = _arr(admittance, np.float64)
        coe = _arr(coarse_of_elem, np.int32)
        cv = _arr(coarse_verts, np.int32)
        nc = 0 if cv is None else cv.shape[0]
        self._keep = (coords, elems, bf, adm, coe, cv)
        rc = self.lib.mgrt_upload_mesh(self._h, int(dim), coords.shape[0], _ptr(coords),
                                       elems.shape[0], _ptr(elems),
                                       0 if bf is None else bf.shape[0], _ptr(bf), _ptr(adm),
                                       nc, _ptr(coe), _ptr(cv))
        self._keep = None
        self._check(rc, "mgrt_upload_mesh")
        self.dim = int(dim)
        self.n_coarse = nc
        self.n_elems = elems.shape[0]

    def upload_permittivity(self, eps, sigma=None):
        e = _arr(eps, np.float64)
        s = _arr(sigma, np.float64)
        self._check(self.lib.mgrt_upload_permittivity(self._h, _ptr(e), _ptr(s)),
                    "mgrt_upload_permittivity")

    def upload_pml(self, xi=None, zeta=None):
        """mgrt_upload_pml: xi (m,), zeta (m, dim); both None removes the layer."""
        x = _arr(xi, np.float64)
        z = _arr(zeta, np.float64)
        self._check(self.lib.mgrt_upload_pml(self._h, _ptr(x), _ptr(z)), "mgrt_upload_pml")

    def stability_bound(self) -> float:
        out = C.c_double()
        self._check(self.lib.mgrt_stability_bound(self._h, C.byref(out)), "mgrt_stability_bound")
        return out.value

    @staticmethod
    def _opts(precision, variant, batch, timing, flags=0, mem_budget_gb=0.0, deconv_delta=0.0,
              launch=0):
        f = flags | (native.F_TIMING if timing else 0)
        v = {"batched": native.STEP_BATCHED, "plain": native.STEP_PLAIN}[variant] \
            if isinstance(variant, str) else int(variant)
        return RunOpts(int(precision), v, int(batch), f, float(mem_budget_gb), float(deconv_delta),
                       int(launch))

    def _device_out(self, out, shape):
        """Pointer of a caller's device output: a contiguous CUDA float64 tensor of `shape`
        on this context's device."""
        ok = (getattr(out, "is_cuda", False) and str(out.dtype) == "torch.float64"
              and out.is_contiguous() and tuple(out.shape) == tuple(shape)
              and out.device.index == self.device)
        if not ok:
            raise ValueError(f"out must be a contiguous float64 CUDA tensor of shape "
                             f"{tuple(shape)} on device {self.device}")
        return C.c_void_p(out.data_ptr())

    def _acq(self, src, rec):
        src = _arr(src, np.float64).reshape(-1, self.dim)
        rec = _arr(rec, np.float64).reshape(src.shape[0], -1, self.dim)
        return src, rec

    # ------------------------------------------------------------------ forward
    def forward_traces(self, src, rec, wavelet, dt, n_steps, precision=32, variant="batched",
                       batch=0, timing=False, out=None, skip_stability=False, launch=0,
                       graph=True, one_step=False):
        """launch: 0 = the tuned launch variant, 1..16 = variant launch - 1.  graph=False
        launches every step directly (MGRT_F_NO_GRAPH) instead of replaying captured runs
        of steps.  one_step=True (MGRT_F_ONE_STEP) keeps one launch per step where a small
        one-column run would take several steps per launch."""
        src, rec = self._acq(src, rec)
        wav = _arr(wavelet, np.float64)
        if wav.shape[0] < n_steps:
            raise ValueError("wavelet shorter than n_steps")
        flags = native.F_SKIP_STABILITY if skip_stability else 0
        if not graph:
            flags |= native.F_NO_GRAPH
        if one_step:
            flags |= native.F_ONE_STEP
        shape = (src.shape[0], rec.shape[1], int(n_steps))
        if out is not None:
            flags |= native.F_DEVICE_OUT
            optr = self._device_out(out, shape)
            res = out
        else:
            res = np.empty(shape)
            optr = _ptr(res)
        opts = self._opts(precision, variant, batch, timing, flags, launch=launch)
        rc = self.lib.mgrt_forward_traces(self._h, src.shape[0], _ptr(src), rec.shape[1],
                                          _ptr(rec), _ptr(wav), float(dt), int(n_steps),
                                          C.byref(opts), optr)
        self._check(rc, "mgrt_forward_traces")
        return res

    def forward_traces_noalloc(self, src, rec, wavelet, dt, n_steps, precision=32, batch=0,
                               out=None, skip_stability=False, launch=0):
        """mgrt_forward_traces_noalloc: the same traces without any device allocation in
        the library (a prior forward_traces call with the same arguments builds the
        operator).  out: optional float64 CUDA tensor, else a NumPy array."""
        src, rec = self._acq(src, rec)
        wav = _arr(wavelet, np.float64)
        if wav.shape[0] < n_steps:
            raise ValueError("wavelet shorter than n_steps")
        flags = native.F_SKIP_STABILITY if skip_stability else 0
        shape = (src.shape[0], rec.shape[1], int(n_steps))
        if out is not None:
            flags |= native.F_DEVICE_OUT
            optr = self._device_out(out, shape)
            res = out
        else:
            res = np.empty(shape)
            optr = _ptr(res)
        opts = self._opts(precision, "batched", batch, False, flags, launch=launch)
        rc = self.lib.mgrt_forward_traces_noalloc(self._h, src.shape[0], _ptr(src), rec.shape[1],
                                                  _ptr(rec), _ptr(wav), float(dt), int(n_steps),
                                                  C.byref(opts), optr)
        self._check(rc, "mgrt_forward_traces_noalloc")
        return res

    # ------------------------------------------------------------------ linearisation
    def jacobian_coarse(self, src, rec, wavelet, dt, n_steps, sample_steps, mode="mg",
                        cols=None, precision=32, batch=0, timing=False, mem_budget_gb=0.0,
                        deconv_delta=0.0, launch=0, out=None, pairing="auto", graph=True,
                        one_run=True):
        """mode "mg" (eq. approx_2), "exact" (eq. approx_1, listed cols) or "deconv" (the
        regularised-deconvolution route to eq. approx_2 with Tikhonov deconv_delta).
        pairing (MG mode): "auto" (the library's default for the precision), "split" or
        "direct" (MGRT_F_JAC_SPLIT / MGRT_F_JAC_DIRECT).  one_run=False keeps a source run
        and a receiver run per monostatic pair (MGRT_F_JAC_PAIRED).
        out: optional float64 CUDA tensor (rows x columns) that receives J in device
        memory (no copy to the host); else J is returned as a NumPy array."""
        src, rec = self._acq(src, rec)
        wav = _arr(wavelet, np.float64)
        ss = _arr(sample_steps, np.int64)
        m = {"mg": native.JAC_MG, "exact": native.JAC_EXACT, "deconv": native.JAC_DECONV}[mode]
        cl = _arr(cols, np.int64)
        ncol = self.n_coarse if cl is None else cl.shape[0]
        shape = (src.shape[0] * rec.shape[1] * ss.shape[0], ncol)
        flags = {"auto": 0, "split": native.F_JAC_SPLIT, "direct": native.F_JAC_DIRECT}[pairing]
        if not one_run:
            flags |= native.F_JAC_PAIRED
        if not graph:
            flags |= native.F_NO_GRAPH
        if out is not None:
            flags |= native.F_DEVICE_OUT
            J, jptr = out, self._device_out(out, shape)
        else:
            J = np.empty(shape)
            jptr = _ptr(J)
        opts = self._opts(precision, "batched", batch, timing, flags, mem_budget_gb,
                          deconv_delta, launch)
        rc = self.lib.mgrt_jacobian_coarse(self._h, src.shape[0], _ptr(src), rec.shape[1],
                                           _ptr(rec), _ptr(wav), float(dt), int(n_steps),
                                           ss.shape[0], _ptr(ss), m,
                                           0 if cl is None else cl.shape[0], _ptr(cl),
                                           C.byref(opts), jptr)
        self._check(rc, "mgrt_jacobian_coarse")
        return J

    def misfit_gradient(self, src, rec, wavelet, dt, n_steps, residual, level="coarse",
                        precision=32, batch=0, timing=False, mem_budget_gb=0.0, launch=0,
                        graph=True):
        src, rec = self._acq(src, rec)
        wav = _arr(wavelet, np.float64)
        res = _arr(residual, np.float64).reshape(src.shape[0], rec.shape[1], int(n_steps))
        lv = {"coarse": 0, "fine": 1}[level]
        g = np.empty(self.n_coarse if lv == 0 else self.n_elems)
        opts = self._opts(precision, "batched", batch, timing, 0 if graph else native.F_NO_GRAPH,
                          mem_budget_gb, launch=launch)
        rc = self.lib.mgrt_misfit_gradient(self._h, src.shape[0], _ptr(src), rec.shape[1],
                                           _ptr(rec), _ptr(wav), float(dt), int(n_steps),
                                           _ptr(res), lv, C.byref(opts), _ptr(g))
        self._check(rc, "mgrt_misfit_gradient")
        return g

    @staticmethod
    def _matrix_arg(L):
        """(pointer, precision, rows, M, on_device, keep-alive) for a Jacobian-like matrix:
        NumPy (host, FP32/FP64) or a CUDA torch tensor (device)."""
        if hasattr(L, "is_cuda") and L.is_cuda:
            import torch
            Lc = L.contiguous()
            prec = 32 if Lc.dtype == torch.float32 else 64
            if Lc.dtype not in (torch.float32, torch.float64):
                raise TypeError("L must be float32 or float64")
            rows, M = Lc.shape
            return C.c_void_p(Lc.data_ptr()), prec, rows, M, 1, Lc
        La = np.asarray(L)
        if La.dtype != np.float32:
            La = La.astype(np.float64)
        La = np.ascontiguousarray(La)
        prec = 32 if La.dtype == np.float32 else 64
        rows, M = La.shape
        return _ptr(La), prec, rows, M, 0, La

    def tv_invert_level(self, L, r, D_rowptr, D_col, D_val, alpha, iters=3, cg_rtol=1e-10,
                        cg_maxit=1000, solver="auto"):
        """L: NumPy (host, FP32/FP64) or a CUDA torch tensor (device).  solver "auto"
        (dense Cholesky where the normal matrix is formed, else CG) or "cg"."""
        Lp, prec, rows, M, on_dev, keep = self._matrix_arg(L)
        r = _arr(r, np.float64)
        rp = _arr(D_rowptr, np.int64)
        dc = _arr(D_col, np.int32)
        dv = _arr(D_val, np.float64)
        z = np.empty((int(iters), M))
        it = np.zeros(int(iters), dtype=np.int32)
        rc = self.lib.mgrt_tv_invert_level(self._h, rows, M, Lp, prec, on_dev, _ptr(r),
                                           _ptr(rp), _ptr(dc), _ptr(dv), float(alpha),
                                           int(iters), float(cg_rtol), int(cg_maxit),
                                           _solver_code(solver), _ptr(z), _ptr(it))
        del keep
        self._check(rc, "mgrt_tv_invert_level")
        return z, it

    def project_rows(self, J, u, q):
        """mgrt_project_rows: J (n_traces*n_samples, M) NumPy or CUDA tensor (FP32/FP64),
        u (n_traces, n_samples), q (n_proj, n_samples) -> P (n_traces*n_proj, M)."""
        Jp, prec, rows, M, on_dev, keep = self._matrix_arg(J)
        u = _arr(u, np.float64)
        q = _arr(q, np.float64)
        if u.ndim != 2 or q.ndim != 2 or q.shape[1] != u.shape[1]:
            raise ValueError("u must be n_traces x n_samples and q n_proj x n_samples")
        nt, ns = u.shape
        if rows != nt * ns:
            raise ValueError("J must have n_traces * n_samples rows")
        P = np.empty((nt * q.shape[0], M))
        rc = self.lib.mgrt_project_rows(self._h, nt, ns, M, Jp, prec, on_dev, _ptr(u),
                                        q.shape[0], _ptr(q), _ptr(P))
        del keep
        self._check(rc, "mgrt_project_rows")
        return P

    def tv_invert_two_level(self, L, r, elem_verts, parent, M2, Dc, Df, alpha, iters=3,
                            n_keep=None, cg_rtol=1e-10, cg_maxit=1000, solver="auto"):
        """Coarse-to-fine inversion (mgrt_tv_invert_two_level).  Dc, Df: (rowptr, col, val)
        CSR triples on T'' and T'.  n_keep None keeps every parent's fluctuations.
        solver as for tv_invert_level.  Returns dict x (iters x M), zc (iters x M2), kept
        (iters x n_keep), cg_iters (iters x 2; 0 where a level was solved directly)."""
        Lp, prec, rows, M, on_dev, keep = self._matrix_arg(L)
        r = _arr(r, np.float64)
        ev = _arr(elem_verts, np.int32)
        par = _arr(parent, np.int32)
        if ev.ndim != 2 or ev.shape[0] != M or par.shape != (M,):
            raise ValueError("elem_verts must be M x (dim+1) and parent length M")
        dim = ev.shape[1] - 1
        M2 = int(M2)
        n_keep = M2 if n_keep is None else int(n_keep)
        kk = min(n_keep, M2)
        c_rp, c_cl, c_vl = (_arr(Dc[0], np.int64), _arr(Dc[1], np.int32), _arr(Dc[2], np.float64))
        f_rp, f_cl, f_vl = (_arr(Df[0], np.int64), _arr(Df[1], np.int32), _arr(Df[2], np.float64))
        x = np.empty((int(iters), M))
        zc = np.empty((int(iters), M2))
        kept = np.empty((int(iters), kk), dtype=np.int32)
        it = np.zeros((int(iters), 2), dtype=np.int32)
        rc = self.lib.mgrt_tv_invert_two_level(
            self._h, rows, M, Lp, prec, on_dev, _ptr(r), dim, _ptr(ev), M2, _ptr(par),
            _ptr(c_rp), _ptr(c_cl), _ptr(c_vl), _ptr(f_rp), _ptr(f_cl), _ptr(f_vl),
            float(alpha), int(iters), n_keep, float(cg_rtol), int(cg_maxit),
            _solver_code(solver), _ptr(x),
            _ptr(zc), _ptr(kept) if kk else None, _ptr(it))
        del keep
        self._check(rc, "mgrt_tv_invert_two_level")
        return {"x": x, "zc": zc, "kept": kept, "cg_iters": it}

    def last_timing(self) -> dict:
        t = Timing()
        self.lib.mgrt_last_timing(self._h, C.byref(t))
        out = {}
        for k, _ in Timing._fields_:
            v = getattr(t, k)
            out[k] = list(v) if isinstance(v, C.Array) else v
        return out


def context_for_problem(prob, device=0, eps=None, absorbing=True):
    """Context with the problem's mesh and permittivity uploaded (and its split-field PML,
    which then replaces the first-order absorbing boundary)."""
    ctx = Context(device)
    ms = prob.mesh
    pml = getattr(prob, "pml", None)
    ctx.upload_mesh(ms.d, ms.coords, ms.elems,
                    ms.bfacets if absorbing and pml is None else None, None,
                    ms.coarse_of_elem, ms.coarse_verts)
    ctx.upload_permittivity(prob.eps if eps is None else eps, prob.sigma)
    if pml is not None:
        ctx.upload_pml(*pml)
    return ctx
