"""ctypes wrapper around the FP64 CPU oracle (``stokes_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The oracle shares
no code with the HIP path.

Preconditioner codes (block-diagonal M = blkdiag(M_A, M_Q), paper Sec. 5.1):
  pc_A: 0 IC(0), 1 IC(0)-PCG (inner, relative 2-norm tolerance), 2 Jacobi,
        3 exact (dense Cholesky, small meshes only), 4 Jacobi-PCG
  pc_Q: 0 Diag(Q)/(2 nu), 1 exact Q/(2 nu) (dense Cholesky), 2 Jacobi-PCG on Q,
        3 IC(0) of Q applied once, 4 IC(0)-PCG on Q
Forcing problems: 0 none, 1 manufactured curl solution with p = prod cos(pi x),
  2 the paper's square-domain solution (Sec. 6.2, divergence-free sign),
  3 pure gradient forcing f = grad(sin(2 pi x) cos(pi y) [cos(pi z)]),
  4 (1/8 annulus) u = curl(a^2 b^2), a = (r^2 - 1)(r^2 - 4), b = y (y - x); p = x y^2.
Geometry (Sec. 3.2): GEOM_SQUARE the identity map on the unit square/cube, GEOM_ANNULUS
  (2D) one eighth of the annulus 1 < r < 2, 0 < theta < pi/4 (Sec. 6.3) by the polar map
  r = 1 + xi_0, theta = (pi/4) xi_1; velocities by the Piola transform, pressures by the
  integral-preserving one.  evaluate() takes parametric points.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

PC_IC0, PC_ICPCG, PC_JACOBI, PC_EXACT, PC_JPCG = 0, 1, 2, 3, 4
GEOM_SQUARE, GEOM_ANNULUS = 0, 1
PQ_DIAG, PQ_EXACT, PQ_JPCG, PQ_IC0, PQ_ICPCG = 0, 1, 2, 3, 4


def build(force=False):
    """Compile the oracle with g++ (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = "%s.tmp%d" % (_LIB, os.getpid())
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        L.or_setup.restype = vp
        L.or_setup.argtypes = [i32, i32, i32, dbl, dbl, i32]
        L.or_free.argtypes = [vp]
        L.or_sizes.argtypes = [vp, P(i64), P(i64)]
        L.or_nnz.restype = i64
        L.or_nnz.argtypes = [vp, i32]
        L.or_get_csr.argtypes = [vp, i32, vp, vp, vp]
        L.or_get_diagQ_w.argtypes = [vp, vp, vp]
        L.or_ic0.restype = i32
        L.or_ic0.argtypes = [vp, P(i32)]
        L.or_ic0_q.restype = i32
        L.or_ic0_q.argtypes = [vp]
        L.or_set_sum_order.argtypes = [i32]
        L.or_load.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.or_matvec.argtypes = [vp, vp, vp]
        L.or_precond.restype = i32
        L.or_precond.argtypes = [vp, i32, i32, dbl, vp, vp, P(i32)]
        L.or_minres.restype = i32
        L.or_minres.argtypes = [vp, vp, vp, dbl, i32, i32, i32, dbl, i32, vp, vp, vp]
        L.or_solve.restype = i32
        L.or_solve.argtypes = [vp, vp, vp, vp, dbl, i32, i32, i32, dbl, i32, vp]
        L.or_project.argtypes = [vp, vp]
        L.or_adjoint.restype = i32
        L.or_adjoint.argtypes = [vp, vp, vp, vp, vp, dbl, i32, i32, i32, dbl, vp]
        L.or_dnu_dot.restype = dbl
        L.or_dnu_dot.argtypes = [vp, vp, vp]
        L.or_eval.argtypes = [vp, vp, vp, i64, vp, vp]
        L.or_errors.argtypes = [vp, i32, vp, vp, vp]
        L.or_load_cavity.restype = i32
        L.or_load_cavity.argtypes = [vp, i32, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Info(dict):
    """iters, inner_total, status, ic_shift_steps, relres_est, relres_true_2, relres_true_Minv"""

    KEYS = ("iters", "inner_total", "status", "ic_shift_steps", "relres_est", "relres_true_2",
            "relres_true_Minv")

    @classmethod
    def from_array(cls, a):
        d = cls(zip(cls.KEYS, a.tolist()))
        for k in ("iters", "inner_total", "status", "ic_shift_steps"):
            d[k] = int(d[k])
        return d


class Oracle:
    """One assembled Stokes problem on the unit square/cube with N elements per direction,
    pressure degree kp (= k'), velocity degree kp+1, viscosity nu; cpen < 0 selects the
    paper's C_pen = 5(k'+1)."""

    def __init__(self, N, kp, dim=2, nu=1.0, cpen=-1.0, pattern_only=False, geometry=0):
        self._L = lib()
        flags = int(bool(pattern_only)) | (2 if geometry == GEOM_ANNULUS else 0)
        self.h = self._L.or_setup(int(N), int(kp), int(dim), float(nu), float(cpen), flags)
        if not self.h:
            raise ValueError("oracle setup rejected the arguments")
        self.N, self.kp, self.dim, self.nu, self.geometry = N, kp, dim, nu, geometry
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._L.or_sizes(self.h, ctypes.byref(a), ctypes.byref(b))
        self.n_u, self.n_p = a.value, b.value
        self.n = self.n_u + self.n_p

    def __del__(self):
        if getattr(self, "h", None):
            self._L.or_free(self.h)
            self.h = None

    # -- matrices -----------------------------------------------------------
    _WHICH = {"A": 0, "B": 1, "Q": 2, "L": 3, "LQ": 4}

    def nnz(self, which):
        return int(self._L.or_nnz(self.h, self._WHICH[which]))

    def csr(self, which):
        """(indptr int64, indices int32, data float64) of A, B, Q, L (IC(0) of A) or LQ (IC(0)
        of Q)."""
        w = self._WHICH[which]
        rows = {"A": self.n_u, "B": self.n_p, "Q": self.n_p, "L": self.n_u, "LQ": self.n_p}[which]
        nnz = self.nnz(which)
        ptr = np.zeros(rows + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float64)
        self._L.or_get_csr(self.h, w, _p(ptr), _p(col), _p(val))
        return ptr, col, val

    def scipy(self, which):
        import scipy.sparse as sp
        ptr, col, val = self.csr(which)
        rows = {"A": self.n_u, "B": self.n_p, "Q": self.n_p, "L": self.n_u, "LQ": self.n_p}[which]
        cols = {"A": self.n_u, "B": self.n_u, "Q": self.n_p, "L": self.n_u, "LQ": self.n_p}[which]
        return sp.csr_matrix((val, col, ptr), shape=(rows, cols))

    def saddle(self):
        import scipy.sparse as sp
        A, B = self.scipy("A"), self.scipy("B")
        return sp.bmat([[A, B.T], [B, None]], format="csr")

    def diagQ_w(self):
        d = np.zeros(self.n_p)
        w = np.zeros(self.n_p)
        self._L.or_get_diagQ_w(self.h, _p(d), _p(w))
        return d, w

    def ic0(self):
        s = ctypes.c_int(0)
        rc = self._L.or_ic0(self.h, ctypes.byref(s))
        return rc, s.value

    def ic0_q(self):
        """IC(0) factor of the pressure mass matrix Q (0, or -4 on breakdown)."""
        return int(self._L.or_ic0_q(self.h))

    @staticmethod
    def set_sum_order(reverse):
        """Sum the oracle's inner products forward (False, default) or in reverse (True):
        the same mathematics with another rounding, for sensitivity checks."""
        lib().or_set_sum_order(int(bool(reverse)))

    # -- vectors ------------------------------------------------------------
    def load(self, problem=1, modes=None):
        """Assembled load vector(s).  modes = (amp[R,dim,M], wave[R,M,dim], phase[R,dim,M]) or None."""
        if modes is None:
            f = np.zeros(self.n_u)
            self._L.or_load(self.h, int(problem), 1, 0, None, None, None, _p(f))
            return f
        amp, wave, phase = (_f64(modes[0]), np.ascontiguousarray(modes[1], np.int32), _f64(modes[2]))
        R, M = amp.shape[0], amp.shape[2]
        f = np.zeros((R, self.n_u))
        self._L.or_load(self.h, int(problem), R, M, _p(amp), _p(wave), _p(phase), _p(f))
        return f

    def load_cavity(self, kind=0):
        """2D load vector with tangential boundary data through the Nitsche form l_h
        (eq. nitsche_rhs): kind 0 the lid-driven cavity (Sec. 6.4), kind 1 the verification
        flow u = curl(x(1-x)y(1-y)), p = 0."""
        f = np.zeros(self.n_u)
        if self._L.or_load_cavity(self.h, int(kind), _p(f)) != 0:
            raise ValueError("cavity load: 2D only, kind 0 or 1")
        return f

    def matvec(self, x):
        x = _f64(x)
        y = np.zeros(self.n)
        self._L.or_matvec(self.h, _p(x), _p(y))
        return y

    def precond(self, r, pc_A=PC_IC0, pc_Q=PQ_DIAG, inner_tol=1e-2):
        r = _f64(r)
        z = np.zeros(self.n)
        it = ctypes.c_int(0)
        rc = self._L.or_precond(self.h, pc_A, pc_Q, float(inner_tol), _p(r), _p(z), ctypes.byref(it))
        if rc != 0:
            raise RuntimeError("oracle preconditioner setup failed (IC breakdown)")
        return z, it.value

    def minres(self, b, tol=1e-8, maxit=10000, pc_A=PC_IC0, pc_Q=PQ_DIAG, inner_tol=1e-2, fixed=False,
               history=False, x_history=False):
        b = _f64(b)
        x = np.zeros(self.n)
        info = np.zeros(7)
        eta = np.zeros(maxit + 1) if history else None
        xh = np.zeros((maxit, self.n)) if x_history else None
        self._L.or_minres(self.h, _p(b), _p(x), float(tol), int(maxit), int(pc_A), int(pc_Q),
                          float(inner_tol), int(bool(fixed)), _p(info), _p(eta), _p(xh))
        inf = Info.from_array(info)
        out = [x, inf]
        if history:
            out.append(eta[: inf["iters"] + 1])
        if x_history:
            out.append(xh[: inf["iters"]])
        return tuple(out)

    def solve(self, f, tol=1e-8, maxit=10000, pc_A=PC_IC0, pc_Q=PQ_DIAG, inner_tol=1e-2, fixed=False):
        f = _f64(f)
        u = np.zeros(self.n_u)
        p = np.zeros(self.n_p)
        info = np.zeros(7)
        self._L.or_solve(self.h, _p(f), _p(u), _p(p), float(tol), int(maxit), int(pc_A), int(pc_Q),
                         float(inner_tol), int(bool(fixed)), _p(info))
        return u, p, Info.from_array(info)

    def solve_refined(self, f, tol=1e-8, maxit=10000, pc_A=PC_ICPCG, pc_Q=PQ_DIAG, inner_tol=1e-2, cycles=6):
        """MINRES restarted on the true residual until ||b - Acal x||_{M^-1} <= tol ||b||_{M^-1}
        with M the fixed block preconditioner that the inner solves approximate:
        blkdiag(IC(0), Diag(Q)/(2 nu)) for IC(0)-PCG on A, blkdiag(Diag(A), Diag(Q)/(2 nu))
        for Jacobi-PCG on A (and on Q).  Used for inner-PCG blocks, nonlinear preconditioners
        whose MINRES estimate |eta| measures the residual in a norm that changes between
        applications (Sec. 5: MINRES minimises in the norm of a fixed SPD preconditioner).
        Each cycle solves Acal d = r to the remaining relative reduction (at most 0.5) and
        projects p."""
        b0 = np.concatenate([_f64(f), np.zeros(self.n_p)])
        lin_A = PC_JACOBI if pc_A in (PC_JACOBI, PC_JPCG) else PC_IC0
        lin_Q = {PQ_JPCG: PQ_DIAG, PQ_ICPCG: PQ_IC0}.get(pc_Q, pc_Q)

        def mnorm2(v):
            z, _ = self.precond(v, pc_A=lin_A, pc_Q=lin_Q)
            return float(v @ z)

        bM = mnorm2(b0)
        x = np.zeros(self.n)
        b = b0.copy()
        tol_k, iters, inner, relM = tol, 0, 0, np.inf
        for _ in range(cycles):
            d, inf = self.minres(b, tol=tol_k, maxit=maxit, pc_A=pc_A, pc_Q=pc_Q, inner_tol=inner_tol)
            iters += inf["iters"]
            inner += inf["inner_total"]
            x = x + d
            x[self.n_u:] = self.project(x[self.n_u:])
            r = b0 - self.matvec(x)
            relM = np.sqrt(max(0.0, mnorm2(r)) / bM) if bM > 0 else 0.0
            if relM <= tol:
                break
            b = r
            tol_k = min(0.5, 0.5 * tol / relM)
        return x[: self.n_u], x[self.n_u:], {"iters": iters, "inner_total": inner, "relres_true_Minv": relM}

    def project(self, p):
        p = _f64(p).copy()
        self._L.or_project(self.h, _p(p))
        return p

    def adjoint(self, g_u, g_p, tol=1e-8, maxit=10000, pc_A=PC_IC0, pc_Q=PQ_DIAG, inner_tol=1e-2):
        g_u, g_p = _f64(g_u), _f64(g_p)
        lu = np.zeros(self.n_u)
        lp = np.zeros(self.n_p)
        info = np.zeros(7)
        self._L.or_adjoint(self.h, _p(g_u), _p(g_p), _p(lu), _p(lp), float(tol), int(maxit), int(pc_A),
                           int(pc_Q), float(inner_tol), _p(info))
        return lu, lp, Info.from_array(info)

    def dnu_dot(self, lam_u, u):
        return float(self._L.or_dnu_dot(self.h, _p(_f64(lam_u)), _p(_f64(u))))

    def evaluate(self, u, p, pts):
        """Discrete fields at the physical images of parametric points pts[npts, dim]:
        returns [npts, dim+2] = (u..., div u, p)."""
        pts = _f64(pts)
        out = np.zeros((pts.shape[0], self.dim + 2))
        self._L.or_eval(self.h, _p(_f64(u)), _p(_f64(p)), int(pts.shape[0]), _p(pts), _p(out))
        return out

    def errors(self, u, p, problem=1):
        out = np.zeros(3)
        self._L.or_errors(self.h, int(problem), _p(_f64(u)), _p(_f64(p)), _p(out))
        return out
