"""Python view of the C ABI (one StokesProblem per assembled system).

Method: Cortes & Coutinho, block-diagonally preconditioned MINRES (Sec. 5) for the
divergence-conforming B-spline Stokes system (Secs. 3-4).  Tensors are torch float64
CUDA (HIP) tensors; the library runs on torch's current stream.
"""
import ctypes

import numpy as np
import torch

from . import _native as N


class StokesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("stokes error %d: %s" % (code, msg))
        self.code = code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev(t, name, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float64 tensor on the GPU" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return t


class StokesProblem:
    """stokes_setup_nitsche(n, p, dim, nu, geometry, c_pen): n elements per direction,
    pressure degree p (= k'), velocity degree p+1 with maximal continuity, on the unit square
    (dim 2) or cube (dim 3), or (geometry = GEOMETRY_ANNULUS, 2D) on the 1/8 annulus; c_pen < 0
    selects the paper's Nitsche constant 5(k'+1)."""

    def __init__(self, n, p, dim=2, nu=1.0, device=None, geometry=N.GEOMETRY_SQUARE, c_pen=-1.0):
        self._L = N.lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self._L.stokes_setup_nitsche(int(n), int(p), int(dim), float(nu), int(geometry),
                                              float(c_pen), ctypes.byref(self._h))
        if rc != 0 or not self._h:
            raise StokesError(rc, "stokes_setup(%d, %d, %d, %g, c_pen %g) failed" % (n, p, dim, nu, c_pen))
        self.n, self.p, self.dim, self.nu, self.geometry = n, p, dim, nu, geometry
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._L.stokes_sizes(self._h, ctypes.byref(a), ctypes.byref(b))
        self.n_u, self.n_p = a.value, b.value

    # -- plumbing -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._L.stokes_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        self._L.stokes_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, rc, allow_nc=True):
        if rc == 0 or (allow_nc and rc == N.STOKES_NOT_CONVERGED):
            return rc
        raise StokesError(rc, self.last_error())

    def last_error(self):
        m = self._L.stokes_last_error(self._h)
        return m.decode() if m else ""

    def empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    # -- configuration ------------------------------------------------------
    def set_nu(self, nu):
        self._stream()
        self._check(self._L.stokes_set_nu(self._h, float(nu)), allow_nc=False)
        self.nu = nu

    def set_inner_tol(self, rtol):
        self._L.stokes_set_inner_tol(self._h, float(rtol))

    def set_refine_tol(self, rtol):
        self._check(self._L.stokes_set_refine_tol(self._h, float(rtol)), allow_nc=False)

    def set_maxit(self, outer=0, inner=0):
        self._L.stokes_set_maxit(self._h, int(outer), int(inner))

    def set_restarts(self, max_cycles):
        """Inner-CG preconditioners: 0 = one MINRES run (the paper's method, default),
        1..30 = MINRES restarted on the true residual at most that many times."""
        self._check(self._L.stokes_set_restarts(self._h, int(max_cycles)), allow_nc=False)

    def profile(self, enable=-1):
        """Per-category kernel time (ms) and launch counts recorded with HIP events:
        spmv, trsv_fwd, trsv_bwd, lanczos, update.  enable: 1 start/reset, 0 stop, -1 read."""
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int64 * 5)()
        self._check(self._L.stokes_profile(self._h, int(enable), ms, cnt), allow_nc=False)
        names = ("spmv", "trsv_fwd", "trsv_bwd", "lanczos", "update")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(names)}

    def levels(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        self._check(self._L.stokes_levels(self._h, ctypes.byref(a), ctypes.byref(b)), allow_nc=False)
        return a.value, b.value

    # -- load vectors -------------------------------------------------------
    def load(self, manufactured=True, modes=None, nrhs=1):
        """Assembled load vectors [nrhs, n_u]; modes = (amp[R,dim,M], wave[R,M,dim], phase[R,dim,M])."""
        spec = N.StokesForcing()
        spec.manufactured = 1 if manufactured else 0
        keep = []
        if modes is not None:
            amp = np.ascontiguousarray(modes[0], np.float64)
            wave = np.ascontiguousarray(modes[1], np.int32)
            phase = np.ascontiguousarray(modes[2], np.float64)
            nrhs = amp.shape[0]
            spec.nmodes = amp.shape[2]
            spec.amp, spec.wave, spec.phase = amp.ctypes.data, wave.ctypes.data, phase.ctypes.data
            keep = [amp, wave, phase]
        else:
            spec.nmodes = 0
        f = self.empty(nrhs, self.n_u)
        self._stream()
        self._check(self._L.stokes_load(self._h, ctypes.byref(spec), int(nrhs), _ptr(f)), allow_nc=False)
        del keep
        return f

    def load_cavity(self, kind=N.CAVITY_LID):
        """2D load vector [n_u] with tangential boundary data through the Nitsche form l_h:
        CAVITY_LID (lid-driven cavity) or CAVITY_VERIFY (a flow in the discrete space)."""
        f = self.empty(self.n_u)
        self._stream()
        self._check(self._L.stokes_load_cavity(self._h, int(kind), _ptr(f)), allow_nc=False)
        return f

    # -- solves -------------------------------------------------------------
    def solve(self, f, tol=1e-8, precond=N.PC_IC0, precision=N.FP64, out=None):
        """u [n_u], p [n_p] (zero mean), info dict."""
        _dev(f, "f", self.n_u)
        u = self.empty(self.n_u) if out is None else out[0]
        p = self.empty(self.n_p) if out is None else out[1]
        info = N.StokesInfo()
        self._stream()
        rc = self._L.stokes_solve_precision(self._h, _ptr(f), _ptr(u), _ptr(p), float(tol), int(precond),
                                            int(precision), ctypes.byref(info))
        self._check(rc)
        return u, p, info.as_dict()

    def solve_noalloc(self, f, u, p, tol=1e-8, precond=N.PC_IC0):
        """stokes_solve_noalloc: the library allocates nothing; u [n_u] and p [n_p] are the
        caller's output tensors.  Returns the info dict."""
        _dev(f, "f", self.n_u)
        _dev(u, "u", self.n_u)
        _dev(p, "p", self.n_p)
        info = N.StokesInfo()
        self._stream()
        rc = self._L.stokes_solve_noalloc(self._h, _ptr(f), _ptr(u), _ptr(p), float(tol), int(precond),
                                          ctypes.byref(info))
        self._check(rc)
        return info.as_dict()

    def solve_batched(self, F, tol=1e-8, precond=N.PC_IC0, precision=N.FP64):
        """F [nrhs, n_u] -> U [nrhs, n_u], P [nrhs, n_p], infos (list of dicts)."""
        _dev(F, "F")
        R = F.shape[0]
        if F.numel() != R * self.n_u:
            raise ValueError("F must have shape [nrhs, n_u]")
        U, P = self.empty(R, self.n_u), self.empty(R, self.n_p)
        infos = (N.StokesInfo * R)()
        self._stream()
        rc = self._L.stokes_solve_batched(self._h, int(R), _ptr(F), _ptr(U), _ptr(P), float(tol), int(precond),
                                          int(precision), infos)
        self._check(rc)
        return U, P, [i.as_dict() for i in infos]

    def solve_adjoint(self, G, tol=1e-8, precond=N.PC_IC0):
        """G [nrhs, n_u + n_p] (dL/du, dL/dp) -> Lambda [nrhs, n_u + n_p], infos."""
        _dev(G, "G")
        squeeze = G.dim() == 1
        if squeeze:
            G = G.reshape(1, -1)
        R = G.shape[0]
        Lam = self.empty(R, self.n_u + self.n_p)
        infos = (N.StokesInfo * R)()
        self._stream()
        rc = self._L.stokes_solve_adjoint_batched(self._h, int(R), _ptr(G.contiguous()), _ptr(Lam), float(tol),
                                                  int(precond), infos)
        self._check(rc)
        return (Lam[0] if squeeze else Lam), [i.as_dict() for i in infos]

    def dnu_dot(self, lam_u, u):
        """lam_u[r]^T A u[r] / nu for each row r of [nrhs, n_u] tensors (host list)."""
        lam_u = lam_u.reshape(-1, self.n_u).contiguous()
        u = u.reshape(-1, self.n_u).contiguous()
        R = lam_u.shape[0]
        out = (ctypes.c_double * R)()
        self._stream()
        self._check(self._L.stokes_dnu_dot(self._h, int(R), _ptr(lam_u), _ptr(u), out), allow_nc=False)
        return list(out)

    # -- operators (checks) -------------------------------------------------
    def apply(self, x):
        _dev(x, "x", self.n_u + self.n_p)
        y = self.empty(self.n_u + self.n_p)
        self._stream()
        self._check(self._L.stokes_apply(self._h, _ptr(x), _ptr(y)), allow_nc=False)
        return y

    def apply_precond(self, r, precond=N.PC_IC0):
        _dev(r, "r", self.n_u + self.n_p)
        y = self.empty(self.n_u + self.n_p)
        it = ctypes.c_int(0)
        self._stream()
        self._check(self._L.stokes_apply_precond(self._h, int(precond), _ptr(r), _ptr(y), ctypes.byref(it)),
                    allow_nc=False)
        return y, it.value

    def export_csr(self, which=0):
        """(indptr int64, indices int32, data float64) numpy arrays; which 0 = saddle, 1 = IC(0) of A,
        2 = IC(0) of the pressure mass matrix Q."""
        nnz = ctypes.c_int64()
        self._check(self._L.stokes_export_csr(self._h, int(which), ctypes.byref(nnz), None, None, None),
                    allow_nc=False)
        rows = {0: self.n_u + self.n_p, 1: self.n_u, 2: self.n_p}[which]
        ptr = np.zeros(rows + 1, np.int64)
        col = np.zeros(nnz.value, np.int32)
        val = np.zeros(nnz.value, np.float64)
        self._stream()
        self._check(self._L.stokes_export_csr(self._h, int(which), ctypes.byref(nnz), ptr.ctypes.data_as(
            ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p), val.ctypes.data_as(ctypes.c_void_p)),
            allow_nc=False)
        return ptr, col, val

    def export_pressure_mass(self):
        d = np.zeros(self.n_p)
        w = np.zeros(self.n_p)
        self._stream()
        self._check(self._L.stokes_export_pressure_mass(self._h, d.ctypes.data_as(ctypes.c_void_p),
                                                        w.ctypes.data_as(ctypes.c_void_p)), allow_nc=False)
        return d, w
