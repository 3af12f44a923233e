"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is either a
number printed in the paper (tests/golden/paper_tables.json, each entry cited),
a closed form, an invariant of the method, or an independent computation with a
library routine (scipy's B-spline evaluation, dense LAPACK solves/eigensolvers).
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle.oracle import (PC_EXACT, PC_IC0, PC_JACOBI, PC_JPCG, PC_ICPCG, PQ_DIAG, PQ_EXACT, PQ_JPCG, Oracle)


def _tab_row(tab, inv_h):
    for r in tab["rows"]:
        if r[0] == inv_h:
            return dict(zip(tab["columns"], r))
    raise KeyError(inv_h)


# ---------------------------------------------------------------------------
# Sizes and sparsity (Sec. 3.2 spaces, Sec. 6.4 size tables).  The paper's build
# carries two extra velocity functions at the corners; the reading used here
# drops them, and the difference is the same closed form at every mesh size:
# +2 velocity DOFs, +8(k'+1)^2+2 in nnz(A), +2(k'+1)^2 in nnz(B); the pressure
# space and nnz(Q) agree exactly.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kp,inv_hs", [(2, [8, 16, 32, 64, 128]), (3, [8, 16, 32, 64])])
def test_sizes_and_nnz_match_paper_tables(paper, kp, inv_hs):
    tab = paper["sizes_nnz_k%d" % kp]
    for inv_h in inv_hs:
        ref = _tab_row(tab, inv_h)
        o = Oracle(inv_h, kp, pattern_only=True)
        nnzA, nnzB, nnzQ = o.nnz("A"), o.nnz("B"), o.nnz("Q")
        assert o.n_p == ref["n_p"]
        assert nnzQ == ref["nnz_Q"]
        assert o.n_u + 2 == ref["n_u"]
        assert nnzA + 8 * (kp + 1) ** 2 + 2 == ref["nnz_A"]
        nnzB_paper = (ref["nnz_Acal"] - ref["nnz_A"]) // 2
        assert nnzB + 2 * (kp + 1) ** 2 == nnzB_paper
        assert ref["size_Acal"] == ref["n_u"] + ref["n_p"]


@pytest.mark.parametrize("kp,inv_hs", [(2, [8, 16, 32, 64, 128, 256]), (3, [8, 16, 32, 64])])
def test_ic0_factor_nnz_matches_paper(paper, kp, inv_hs):
    """nnz(IC(A)) = nnz(tril A) (zero fill); the paper's count exceeds ours by the lower
    half of its extra corner couplings, (8(k'+1)^2+2 + 2)/2."""
    tab = paper["nnz_ic_k%d" % kp]
    for inv_h in inv_hs:
        ref = _tab_row(tab, inv_h)
        o = Oracle(inv_h, kp, pattern_only=True)
        nnz_tril = (o.nnz("A") + o.n_u) // 2
        assert nnz_tril + (8 * (kp + 1) ** 2 + 4) // 2 == ref["nnz_ICA"]


def test_c1_workload_sizes():
    """The headline workload (N=256, k'=2) has the same velocity/pressure sizes as the
    paper's h=1/256 row up to the two corner functions."""
    o = Oracle(256, 2, pattern_only=True)
    assert (o.n_u, o.n_p) == (132612, 66564)
    assert (o.nnz("A"), o.nnz("B")) == (9307608, 3944448)


# ---------------------------------------------------------------------------
# Independent re-assembly (Sec. 2.2 tensor-product B-splines, Sec. 3.1/4 forms):
# on the identity map every block is a sum of Kronecker products of 1D integrals.
# The 1D functions come from scipy's B-spline implementation and the integrals
# from numpy's Gauss-Legendre rule; nothing is shared with the oracle's element loop.
# ---------------------------------------------------------------------------
def _spline_tables(deg, N):
    from scipy.interpolate import BSpline
    t = np.concatenate([np.zeros(deg + 1), np.arange(1, N) / N, np.ones(deg + 1)])
    n = N + deg
    spl = BSpline(t, np.eye(n), deg, extrapolate=False)
    dspl = spl.derivative()
    return spl, dspl, n


def _int1d(N, fa, fb, nq=8):
    """Matrix of integrals over [0,1] of fa_i(x) fb_j(x) (fa, fb: callables -> [npts, n])."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    xs, ws = [], []
    for e in range(N):
        xs.append((e + (xg + 1) / 2) / N)
        ws.append(wg / 2 / N)
    x = np.concatenate(xs)
    w = np.concatenate(ws)
    return (fa(x) * w[:, None]).T @ fb(x)


def _kron_assembly(N, kp, nu=1.0):
    p = kp + 1
    C = 5.0 * (kp + 1)
    h = 1.0 / N
    hi, dhi, nhi = _spline_tables(p, N)
    lo, dlo, nlo = _spline_tables(kp, N)
    keep_hi = np.arange(1, nhi - 1)
    # direction spaces of velocity component c: (space, derivative, retained indices)
    def dirspace(c, d):
        if c == d:
            return (lambda x: hi(x)[:, keep_hi]), (lambda x: dhi(x)[:, keep_hi])
        return (lambda x: lo(x)), (lambda x: dlo(x))

    def endval(f, x0):
        # value at the end points (the element-local polynomial, i.e. one-sided limit)
        eps = 1e-14
        return f(np.array([min(max(x0, eps), 1 - eps)]))[0]

    def T(c, d, k, l):
        """integral of (d_k B_i)(d_l B_j) with B_i of component c and B_j of component d."""
        facs = []
        for dr in range(2):
            fi, dfi = dirspace(c, dr)
            fj, dfj = dirspace(d, dr)
            a = dfi if k == dr else fi
            b = dfj if l == dr else fj
            facs.append(_int1d(N, a, b))
        return np.kron(facs[1], facs[0])

    def TF(c, d, k, l, fdir, x0):
        """face integral over {x_fdir = x0} of (d_k B_i)(d_l B_j); k or l may be None."""
        facs = []
        for dr in range(2):
            fi, dfi = dirspace(c, dr)
            fj, dfj = dirspace(d, dr)
            a = dfi if k == dr else fi
            b = dfj if l == dr else fj
            if dr == fdir:
                facs.append(np.outer(endval(a, x0), endval(b, x0)))
            else:
                facs.append(_int1d(N, a, b))
        return np.kron(facs[1], facs[0])

    blocks = [[None, None], [None, None]]
    for c in range(2):
        for d in range(2):
            M = nu * (T(c, d, d, c) + (T(c, d, 0, 0) + T(c, d, 1, 1) if c == d else 0.0))
            for fdir in range(2):
                for x0, s in ((0.0, -1.0), (1.0, 1.0)):
                    n = np.zeros(2)
                    n[fdir] = s
                    # (sym grad Phi_i n).Phi_j = 1/2 (delta_cd dn B_i + n_c d_d B_i) B_j
                    t1 = 0.5 * ((s * TF(c, d, fdir, None, fdir, x0) if c == d else 0.0)
                                + n[c] * TF(c, d, d, None, fdir, x0))
                    t2 = 0.5 * ((s * TF(c, d, None, fdir, fdir, x0) if c == d else 0.0)
                                + n[d] * TF(c, d, None, c, fdir, x0))
                    M = M - 2 * nu * (t1 + t2)
                    if c == d:
                        M = M + 2 * nu * (C / h) * TF(c, d, None, None, fdir, x0)
            blocks[c][d] = M
    A = np.block(blocks)
    Bs = []
    for c in range(2):
        facs = []
        for dr in range(2):
            fj, dfj = dirspace(c, dr)
            facs.append(_int1d(N, lambda x: lo(x), dfj if dr == c else fj))
        Bs.append(-np.kron(facs[1], facs[0]))
    B = np.hstack(Bs)
    Mlo = _int1d(N, lambda x: lo(x), lambda x: lo(x))
    Q = np.kron(Mlo, Mlo)
    return A, B, Q


@pytest.mark.parametrize("N,kp,nu", [(5, 1, 1.0), (4, 2, 0.3), (6, 2, 1.0), (4, 3, 1.0)])
def test_assembly_matches_kronecker_route(N, kp, nu):
    o = Oracle(N, kp, 2, nu)
    A, B, Q = _kron_assembly(N, kp, nu)
    Ao, Bo, Qo = (o.scipy(w).toarray() for w in "ABQ")
    scale = np.abs(A).max()
    assert np.abs(Ao - A).max() <= 1e-12 * scale
    assert np.abs(Bo - B).max() <= 1e-12 * np.abs(B).max()
    assert np.abs(Qo - Q).max() <= 1e-13 * np.abs(Q).max()
    # every stored entry is a structural (support-overlap) entry: values outside vanish
    assert np.count_nonzero(np.abs(A) > 1e-13 * scale) <= o.nnz("A")


# ---------------------------------------------------------------------------
# Structural properties: A symmetric positive definite (coercivity, Sec. 4),
# B^T 1 = 0 (enclosed flow, Sec. 5), w = Q 1 integrates the unit function.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,kp,dim", [(8, 1, 2), (8, 2, 2), (4, 1, 3)])
def test_A_spd_and_kernel(N, kp, dim):
    o = Oracle(N, kp, dim)
    A = o.scipy("A").toarray()
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    B = o.scipy("B")
    assert np.abs(B.T @ np.ones(o.n_p)).max() <= 1e-14 * np.abs(B).max() * 10
    d, w = o.diagQ_w()
    assert abs(w.sum() - 1.0) < 1e-13
    Q = o.scipy("Q")
    assert np.allclose(Q @ np.ones(o.n_p), w, rtol=0, atol=1e-15)
    assert np.array_equal(d, Q.diagonal())


# ---------------------------------------------------------------------------
# Divergence-free velocity (Sec. 3.2): div maps V_{0,h} onto Q_{0,h}, so B u = 0
# forces div u_h = 0 pointwise.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,kp,dim", [(8, 1, 2), (16, 2, 2), (8, 3, 2), (4, 1, 3)])
def test_pointwise_divergence_free(N, kp, dim):
    o = Oracle(N, kp, dim)
    f = o.load(1)
    u, p, info = o.solve(f, tol=1e-13)
    assert info["status"] == 0
    pts = np.random.default_rng(1).random((400, dim))
    ev = o.evaluate(u, p, pts)
    umax = np.abs(ev[:, :dim]).max()
    assert np.abs(ev[:, dim]).max() <= 1e-9 * umax * N


# ---------------------------------------------------------------------------
# Pressure robustness (follows from Sec. 3.2): for f = grad(phi) the discrete
# velocity is zero and the pressure is the L2 projection of phi onto Q_h.  The
# projection is computed here independently (scipy B-splines, Gauss rule).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,kp", [(6, 1), (8, 2)])
def test_pressure_robustness(N, kp):
    o = Oracle(N, kp)
    f = o.load(3)
    u, p, info = o.solve(f, tol=1e-13)
    lo, _, nlo = _spline_tables(kp, N)
    Mlo = _int1d(N, lambda x: lo(x), lambda x: lo(x), nq=10)
    bx = _int1d(N, lambda x: lo(x), lambda x: np.sin(2 * np.pi * x)[:, None], nq=10)[:, 0]
    by = _int1d(N, lambda x: lo(x), lambda x: np.cos(np.pi * x)[:, None], nq=10)[:, 0]
    Q = np.kron(Mlo, Mlo)
    pp = np.linalg.solve(Q, np.kron(by, bx))
    w = Q @ np.ones(nlo * nlo)
    pp -= (w @ pp) / w.sum()
    assert np.abs(p - pp).max() <= 1e-9 * np.abs(pp).max()
    assert np.abs(u).max() <= 1e-9 * np.abs(pp).max()


# ---------------------------------------------------------------------------
# Mass-matrix diagonal quality (Sec. 6.4 discussion): eig(Q, Diag Q) bounds.
# k'=1 closed form: the tensor product of the 1D hat-function symbol range [1/2, 3/2].
# ---------------------------------------------------------------------------
def test_gamma_Q(paper):
    ev = sl.eigh(Oracle(16, 1).scipy("Q").toarray(), np.diag(Oracle(16, 1).scipy("Q").diagonal()),
                 eigvals_only=True)
    assert ev[0] >= 0.25 - 1e-12 and ev[-1] <= 2.25 + 1e-12
    assert abs(ev[0] - 0.25) < 1e-2 and abs(ev[-1] - 2.25) < 1e-2
    for kp in (2, 3):
        Q = Oracle(32, kp).scipy("Q").toarray()
        ev = sl.eigh(Q, np.diag(np.diag(Q)), eigvals_only=True)
        g, G = paper["gamma_Q"]["k%d" % kp]
        assert abs(ev[0] - g) <= 0.05 * g
        assert abs(ev[-1] - G) <= 0.01 * G


# ---------------------------------------------------------------------------
# Inf-sup constant against the Nitsche penalty (Sec. 4 tables): beta_0^2 is the
# smallest non-zero eigenvalue of (B A^{-1} B^T, Q/(2 nu)).
# ---------------------------------------------------------------------------
def _schur_spectrum(o, MQ):
    A = o.scipy("A").toarray()
    B = o.scipy("B").toarray()
    S = B @ np.linalg.solve(A, B.T)
    return np.sort(sl.eigh(S, MQ, eigvals_only=True))


@pytest.mark.parametrize("kp", [2, 3])
def test_inf_sup_vs_penalty_table(paper, kp):
    tab = paper["inf_sup_k%d" % kp]
    for cpen, ref in zip(tab["C_pen"], tab["beta0"]):
        o = Oracle(16, kp, 2, 1.0, float(cpen))
        mu = _schur_spectrum(o, o.scipy("Q").toarray() / 2.0)
        assert abs(mu[0]) < 1e-10  # the constant pressure mode (kernel of B^T)
        assert abs(np.sqrt(mu[1]) - ref) <= 5e-3 * ref + 2e-4, (cpen, np.sqrt(mu[1]), ref)


# ---------------------------------------------------------------------------
# Spectra of the preconditioned system at h=1/32 (Sec. 6.4 tables).  For
# M_A = A the non-unit eigenvalues are (1 +- sqrt(1+4 mu)), mu in sig(S, M_Q)
# (Sec. 5.1 block factorisation).  The paper's C_b^2 = 1.0134 / 1.0367 versus
# exactly 1 here moves only the outer Ideal(A,Q) extremes (golden ratio here);
# this is attributed to the paper's two extra corner functions.
# ---------------------------------------------------------------------------
@pytest.mark.slow
@pytest.mark.parametrize("kp", [2, 3])
def test_eigenvalue_table(paper, kp):
    ref = paper["eigen_k%d_h32" % kp]
    o = Oracle(32, kp)
    A = o.scipy("A").toarray()
    Q = o.scipy("Q").toarray()

    def lam_from_mu(mu):
        mu = np.sort(mu)[1:]
        lm, lp = (1 - np.sqrt(1 + 4 * mu)) / 2, (1 + np.sqrt(1 + 4 * mu)) / 2
        return np.array([lm.min(), lm.max(), lp.min(), lp.max()])

    ideal = lam_from_mu(_schur_spectrum(o, Q / 2))
    np.testing.assert_allclose(ideal[[1, 2]], np.array(ref["ideal_A_Q"])[[1, 2]], rtol=1e-3)
    np.testing.assert_allclose(ideal[[0, 3]], np.array(ref["ideal_A_Q"])[[0, 3]], rtol=3e-2)
    np.testing.assert_allclose(ideal[[0, 3]], [(1 - 5 ** 0.5) / 2, (1 + 5 ** 0.5) / 2], rtol=1e-6)
    idiag = lam_from_mu(_schur_spectrum(o, np.diag(np.diag(Q)) / 2))
    np.testing.assert_allclose(idiag, ref["ideal_A_diagQ"], rtol=6e-3)
    K = o.saddle().toarray()

    def extremes(ev):
        ev = ev[np.abs(ev) > 1e-12]
        return np.array([ev[ev < 0].min(), ev[ev < 0].max(), ev[ev > 0].min(), ev[ev > 0].max()])

    np.testing.assert_allclose(extremes(np.linalg.eigvalsh(K)), ref["none"], rtol=5e-3)
    d = 1 / np.sqrt(np.concatenate([np.diag(A), np.diag(Q) / 2]))
    np.testing.assert_allclose(extremes(np.linalg.eigvalsh(K * d[:, None] * d[None, :])), ref["diag_A_Q"],
                               rtol=6e-3)


# ---------------------------------------------------------------------------
# Discretisation errors of the paper's square-domain solution (Sec. 6.2 tables)
# and convergence orders of the manufactured workload solution.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kp,inv_hs", [(2, [8, 16, 32]), (3, [8, 16])])
def test_square_errors_match_paper(paper, kp, inv_hs):
    ref = paper["errors_square_k%d" % kp]
    for inv_h in inv_hs:
        i = ref["inv_h"].index(inv_h)
        o = Oracle(inv_h, kp)
        u, p, info = o.solve(o.load(2), tol=1e-13)
        e = o.errors(u, p, 2)
        for k, name in enumerate(("H1_u", "L2_u", "L2_p")):
            assert abs(e[k] - ref[name][i]) <= 0.006 * ref[name][i], (inv_h, name, e[k], ref[name][i])


@pytest.mark.parametrize("kp,dim,Ns", [(1, 2, [8, 16, 32]), (2, 2, [8, 16, 32]), (1, 3, [4, 8])])
def test_convergence_orders(kp, dim, Ns):
    errs = []
    for N in Ns:
        o = Oracle(N, kp, dim)
        u, p, info = o.solve(o.load(1), tol=1e-13)
        errs.append(o.errors(u, p, 1))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    expect = np.array([kp, kp + 1, kp + 1])
    assert np.all(rates[-1] >= expect - 0.15), rates


# ---------------------------------------------------------------------------
# MINRES (Sec. 5): with a fixed SPD preconditioner |eta_j| equals the M^{-1}-norm
# of the true residual and is non-increasing; x_j is the minimiser over the Krylov
# space; the converged solution is the singular system's solution.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pc", [PC_IC0, PC_JACOBI])
def test_minres_residual_monotone_and_equal_to_estimate(pc):
    o = Oracle(6, 2)
    b = np.concatenate([o.load(1), np.zeros(o.n_p)])
    x, info, eta, xh = o.minres(b, tol=1e-10, maxit=400, pc_A=pc, history=True, x_history=True)
    K = o.saddle()
    rM = []
    for xx in xh:
        r = b - K @ xx
        z, _ = o.precond(r, pc_A=pc)
        rM.append(np.sqrt(r @ z))
    rM = np.array(rM)
    assert np.all(np.diff(rM) <= 1e-12 * rM[0])
    np.testing.assert_allclose(rM, eta[1:], rtol=1e-6, atol=1e-13 * eta[0])


@pytest.mark.parametrize("pc", [PC_IC0, PC_EXACT])
def test_minres_is_krylov_minimiser(pc):
    o = Oracle(4, 1)
    b = np.concatenate([o.load(1), np.zeros(o.n_p)])
    K = o.saddle().toarray()
    Minv = np.column_stack([o.precond(e, pc_A=pc, pc_Q=PQ_DIAG)[0] for e in np.eye(o.n)])
    Minv = (Minv + Minv.T) / 2
    Lm = np.linalg.cholesky(np.linalg.inv(Minv))  # M = Lm Lm^T
    x, info, xh = o.minres(b, maxit=10, pc_A=pc, fixed=True, x_history=True)
    # Krylov space K_j(M^{-1} K, M^{-1} b); minimise ||b - K x||_{M^{-1}}
    Vs = [Minv @ b]
    for j in range(1, 11):
        V = np.column_stack(Vs)
        Qb, _ = np.linalg.qr(V)
        G = np.linalg.solve(Lm, K @ Qb)  # ||r||_{M^-1} = ||Lm^{-1} r||_2
        y = np.linalg.lstsq(G, np.linalg.solve(Lm, b), rcond=None)[0]
        xk = Qb @ y
        assert np.linalg.norm(xh[j - 1] - xk) <= 1e-8 * np.linalg.norm(xk), j
        Vs.append(Minv @ (K @ Vs[-1]))
        Vs[-1] /= np.linalg.norm(Vs[-1])


def test_converged_solution_equals_direct_solve():
    o = Oracle(6, 2)
    f = o.load(1)
    u, p, info = o.solve(f, tol=1e-14)
    K = o.saddle().toarray()
    d, w = o.diagQ_w()
    c = np.concatenate([np.zeros(o.n_u), w])
    Kb = np.block([[K, c[:, None]], [c[None, :], np.zeros((1, 1))]])
    sol = np.linalg.solve(Kb, np.concatenate([f, np.zeros(o.n_p + 1)]))
    assert np.linalg.norm(u - sol[:o.n_u]) <= 1e-10 * np.linalg.norm(sol[:o.n_u])
    assert np.linalg.norm(p - sol[o.n_u:-1]) <= 1e-10 * np.linalg.norm(sol[o.n_u:-1])


@pytest.mark.slow
def test_iteration_counts_square_k2(paper):
    """The paper's P-MINRES counts (Sec. 6.2 table, tol 1e-12) measure the true 2-norm relative
    residual: with that stopping rule the oracle reproduces them; the M^{-1}-norm rule used by
    the solver stops a few iterations later."""
    ref = paper["iters_square_k2"]
    for i, inv_h in enumerate(ref["inv_h"]):
        if inv_h == 8:
            continue  # the paper's extra corner functions matter most on the coarsest mesh
        o = Oracle(inv_h, 2)
        b = np.concatenate([o.load(2), np.zeros(o.n_p)])
        K = o.saddle()
        for key, pa, pq, tol_in in (("ideal_A_Q", PC_EXACT, PQ_EXACT, 0), ("ideal_A_diagQ", PC_EXACT, PQ_DIAG, 0),
                                    ("pcg_A_diagQ", PC_JPCG, PQ_DIAG, 1e-6), ("diag_A_Q", PC_JACOBI, PQ_DIAG, 0)):
            x, info, xh = o.minres(b, tol=1e-14, maxit=900, pc_A=pa, pc_Q=pq, inner_tol=tol_in, x_history=True)
            r2 = np.linalg.norm(b - (K @ xh.T).T, axis=1) / np.linalg.norm(b)
            j2 = int(np.argmax(r2 <= 1e-12)) + 1
            assert abs(j2 - ref[key][i]) <= max(2, 0.035 * ref[key][i]), (inv_h, key, j2, ref[key][i])
        # PCG(A,Q): Jacobi-PCG on both blocks to 1e-6, a nonlinear preconditioner whose count
        # follows the inner solves' rounding; the paper's own column moves by +-5 between
        # meshes (50, 45, 41, 43, 45), so the bar is 6 iterations
        x, info, xh = o.minres(b, tol=1e-14, maxit=900, pc_A=PC_JPCG, pc_Q=PQ_JPCG, inner_tol=1e-6, x_history=True)
        r2 = np.linalg.norm(b - (K @ xh.T).T, axis=1) / np.linalg.norm(b)
        j2 = int(np.argmax(r2 <= 1e-12)) + 1
        assert abs(j2 - ref["pcg_A_Q"][i]) <= 6, (inv_h, "pcg_A_Q", j2, ref["pcg_A_Q"][i])


# ---------------------------------------------------------------------------
# The pressure half of PCG(A,Q) (Sec. 5.1): Jacobi-PCG on the mass matrix Q solves
# Q x = r to its relative tolerance, checked against a sparse direct solve of the
# oracle's Q; with a tight inner tolerance PCG(A,Q) takes the Ideal(A,Q) iteration count.
# ---------------------------------------------------------------------------
def test_pcg_on_Q_and_tight_pcg_A_Q():
    import scipy.sparse.linalg as sla
    o = Oracle(10, 2)
    Q = o.scipy("Q").tocsc()
    r = np.random.default_rng(5).standard_normal(o.n)
    for tol_in in (1e-4, 1e-10):
        z, it = o.precond(r, pc_A=PC_JACOBI, pc_Q=PQ_JPCG, inner_tol=tol_in)
        zq = z[o.n_u:] / (2.0 * o.nu)
        assert np.linalg.norm(Q @ zq - r[o.n_u:]) <= tol_in * np.linalg.norm(r[o.n_u:]) * 1.0001
        ref = sla.spsolve(Q, r[o.n_u:])
        assert np.linalg.norm(zq - ref) <= 50 * tol_in * np.linalg.norm(ref) + 1e-14, tol_in
        assert it > 0
    f = o.load(1)
    _, _, ie = o.solve(f, tol=1e-10, pc_A=PC_EXACT, pc_Q=PQ_EXACT)
    _, _, ip = o.solve(f, tol=1e-10, pc_A=PC_JPCG, pc_Q=PQ_JPCG, inner_tol=1e-12)
    assert abs(ip["iters"] - ie["iters"]) <= 1, (ip["iters"], ie["iters"])


# ---------------------------------------------------------------------------
# Viscosity scaling (Sec. 5.1, Q_nu = Q/(2 nu)): for fixed f, u(nu) = u(1)/nu and
# p(nu) = p(1), and the preconditioned iteration count does not change.
# ---------------------------------------------------------------------------
def test_viscosity_scaling():
    o1, o2 = Oracle(12, 2, 2, 1.0), Oracle(12, 2, 2, 0.01)
    f = o1.load(1)
    u1, p1, i1 = o1.solve(f, tol=1e-10)
    u2, p2, i2 = o2.solve(f, tol=1e-10)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert np.linalg.norm(u2 * 0.01 - u1) <= 1e-8 * np.linalg.norm(u1)
    assert np.linalg.norm(p2 - p1) <= 1e-8 * np.linalg.norm(p1)


# ---------------------------------------------------------------------------
# Adjoint (the system matrix is symmetric, Sec. 5): lambda_u^T f = g_u^T u + g_p^T p,
# the gradient in f checked by central differences (the loss is quadratic in f),
# and dL/dnu = -lambda_u^T (A/nu) u = -(u - u_t)^T u / nu (from the nu scaling).
# ---------------------------------------------------------------------------
def test_adjoint_identities():
    from synthetic_inputs import forcing_modes, random_vector
    o = Oracle(8, 2)
    f = o.load(1, forcing_modes([2000], 2))[0]
    tol = 1e-13
    u, p, _ = o.solve(f, tol=tol)
    ut = u + 1e-2 * random_vector(o.n_u, 3000)
    g_u = u - ut
    g_p = random_vector(o.n_p, 7)
    lu, lp, info = o.adjoint(g_u, g_p, tol=tol)
    assert info["status"] == 0
    lhs = lu @ f
    assert abs(lhs - (g_u @ u + g_p @ p)) <= 1e-9 * (abs(g_u @ u) + abs(g_p @ p))

    def loss(ff, oo=o):
        uu, pp, _ = oo.solve(ff, tol=tol)
        return 0.5 * np.sum((uu - ut) ** 2)

    lu0, _, _ = o.adjoint(g_u, np.zeros(o.n_p), tol=tol)
    d = random_vector(o.n_u, 11)
    eps = 1e-3 * np.linalg.norm(f) / np.linalg.norm(d)
    fd = (loss(f + eps * d) - loss(f - eps * d)) / (2 * eps)
    assert abs(fd - lu0 @ d) <= 1e-7 * abs(fd)
    dnu = -o.dnu_dot(lu0, u)
    assert abs(dnu - (-(u - ut) @ u / o.nu)) <= 1e-8 * abs(dnu)
    nu, dn = 1.0, 1e-4
    lp_, lm_ = Oracle(8, 2, 2, nu + dn), Oracle(8, 2, 2, nu - dn)
    fdn = (loss(f, lp_) - loss(f, lm_)) / (2 * dn)
    assert abs(fdn - dnu) <= 1e-6 * abs(dnu)


# ---------------------------------------------------------------------------
# IC(0) and its breakdown policy (Sec. 6.4 IC(0)): the factor has the pattern of
# tril(A) and is exact for a matrix whose Cholesky factor has no fill; without
# the Nitsche penalty A is indefinite and every shift fails (error code -4).
# ---------------------------------------------------------------------------
def test_ic0_pattern_and_exactness():
    o = Oracle(8, 1)
    rc, shift = o.ic0()
    assert rc == 0 and shift == 0
    L = o.scipy("L")
    A = o.scipy("A")
    import scipy.sparse as sp
    assert (L != 0).nnz <= sp.tril(A).nnz
    Lp = sp.tril(A).tocsr()
    assert np.array_equal(L.indptr, Lp.indptr) and np.array_equal(L.indices, Lp.indices)
    # on the pattern, (L L^T)_ij = A_ij (zero fill-in)
    LLt = (L @ L.T).tocsr()
    Ad = A.toarray()
    mask = A.toarray() != 0
    assert np.abs((LLt.toarray() - Ad)[mask]).max() <= 1e-12 * np.abs(Ad).max()
    # a tridiagonal SPD matrix has no fill: IC(0) = Cholesky.  Use the 1D-like case of a
    # single row of elements is not available; instead check against dense Cholesky on a
    # banded sub-block where the pattern is full.
    n = 6
    sub = Ad[:n, :n]
    if np.all(sub != 0):
        Ld = np.linalg.cholesky(sub)
        np.testing.assert_allclose(L.toarray()[:n, :n], Ld, rtol=1e-12, atol=1e-14)


def test_ic0_breakdown_reports_error():
    o = Oracle(6, 2, 2, 1.0, 0.0)  # no penalty: a_h loses coercivity
    A = o.scipy("A").toarray()
    if np.linalg.eigvalsh(A)[0] < 0:
        rc, shift = o.ic0()
        assert rc == -4 or shift > 0


# ---------------------------------------------------------------------------
# Tangential boundary data through the Nitsche form l_h (eq. nitsche_rhs, Sec. 4).
# Consistency: a flow that lies in the discrete space (u = curl(x(1-x)y(1-y)), p = 0,
# tangential on the boundary) is returned exactly.  The lid-driven cavity (Sec. 6.4):
# mirror symmetry about x = 1/2, zero net flux through x = 1/2 (the discrete velocity is
# divergence free), lid velocity close to 1, and l_h supported on the lid's functions.
# ---------------------------------------------------------------------------
def _verification_flow(pts):
    x, y = pts[:, 0], pts[:, 1]
    return np.stack([x * (1 - x) * (1 - 2 * y), -(1 - 2 * x) * y * (1 - y)], 1)


@pytest.mark.parametrize("N,kp,nu", [(6, 1, 1.0), (5, 2, 0.3), (4, 3, 1.0), (1, 2, 1.0)])
def test_cavity_load_reproduces_discrete_flow(N, kp, nu):
    o = Oracle(N, kp, nu=nu)
    f = o.load_cavity(1)
    pts = np.random.default_rng(3).uniform(0, 1, (40, 2))
    for pa in (PC_EXACT, PC_IC0):
        u, p, info = o.solve(f, tol=1e-14, pc_A=pa)
        v = o.evaluate(u, p, pts)
        assert np.abs(v[:, :2] - _verification_flow(pts)).max() <= 1e-11, pa
        assert np.abs(v[:, 3]).max() <= 1e-10


def test_cavity_lid_properties():
    o = Oracle(16, 2)
    f = o.load_cavity(0)
    u, p, info = o.solve(f, tol=1e-12)
    rng = np.random.default_rng(4)
    P1 = rng.uniform(0, 1, (20, 2))
    P2 = P1.copy()
    P2[:, 0] = 1 - P1[:, 0]
    a, b = o.evaluate(u, p, P1), o.evaluate(u, p, P2)
    assert np.abs(a[:, 0] - b[:, 0]).max() <= 1e-10
    assert np.abs(a[:, 1] + b[:, 1]).max() <= 1e-10
    # net flux through x = 1/2: Gauss rule per element, exact for the piecewise polynomial
    xg, wg = np.polynomial.legendre.leggauss(6)
    ys = np.concatenate([(e + (xg + 1) / 2) / 16 for e in range(16)])
    ws = np.concatenate([wg / 2 / 16 for e in range(16)])
    ux = o.evaluate(u, p, np.stack([np.full_like(ys, 0.5), ys], 1))[:, 0]
    assert abs(ws @ ux) <= 1e-10
    top = o.evaluate(u, p, np.stack([np.linspace(0.2, 0.8, 7), np.ones(7)], 1))[:, 0]
    assert np.abs(top - 1).max() <= 0.05
    # l_h acts only on functions whose support meets y = 1: the last k'+1 rows (y index) of
    # the first component, which has N + k' - 1 functions in x (degree k'+1, both end
    # functions removed) and N + k' in y, x fastest
    nx = o.N + o.kp - 1
    fx = f[: o.n_u // 2].reshape(o.N + o.kp, nx)
    assert np.abs(fx[: -(o.kp + 1)]).max() == 0.0 and np.abs(fx[-1]).max() > 0
    assert np.abs(f[o.n_u // 2:]).max() <= 1e-14 * np.abs(f).max()
    with pytest.raises(ValueError):
        Oracle(2, 1, dim=3).load_cavity(0)


@pytest.mark.slow
def test_iteration_counts_cavity_k2(paper):
    """The paper's cavity counts (Sec. 6.4 table, k' = 2, tol 1e-12 on the true 2-norm relative
    residual, inner PCG 1e-6) for the five preconditioners, with the lid load through l_h.
    Ideal(A,Q) within 2 and Diag(A,Q) within 3 %; the Diag(Q) variants, whose slow pressure
    convergence (gamma_Q ~ 0.058) makes the count sensitive to the discretisation's details
    (the paper adds corner functions), within 12 %; the PCG variants from h = 1/16 (on the
    coarsest mesh those functions weigh most, and the paper's PCG(A,Q) count of 48 at h = 1/8
    stands apart from its own column of 37s), PCG(A,Q) within 2."""
    ref = paper["iters_cavity_k2"]
    for i, inv_h in enumerate(ref["inv_h"][:3]):
        o = Oracle(inv_h, 2)
        b = np.concatenate([o.load_cavity(0), np.zeros(o.n_p)])
        K = o.saddle()
        for key, pa, pq, tol_in, bar in (("ideal_A_Q", PC_EXACT, PQ_EXACT, 0, 2), ("diag_A_Q", PC_JACOBI, PQ_DIAG, 0, 0.03),
                                         ("ideal_A_diagQ", PC_EXACT, PQ_DIAG, 0, 0.12),
                                         ("pcg_A_diagQ", PC_JPCG, PQ_DIAG, 1e-6, 0.12), ("pcg_A_Q", PC_JPCG, PQ_JPCG, 1e-6, 2)):
            if key.startswith("pcg") and inv_h == 8:
                continue
            x, info, xh = o.minres(b, tol=1e-14, maxit=1500, pc_A=pa, pc_Q=pq, inner_tol=tol_in, x_history=True)
            r2 = np.linalg.norm(b - (K @ xh.T).T, axis=1) / np.linalg.norm(b)
            j2 = int(np.argmax(r2 <= 1e-12)) + 1
            lim = bar if bar >= 1 else bar * ref[key][i]
            assert abs(j2 - ref[key][i]) <= lim, (inv_h, key, j2, ref[key][i])


# ---------------------------------------------------------------------------
# IC(0) of the pressure mass matrix Q (Sec. 6.4, the IC(0)-PCG(A,Q) preconditioner).
# On the identity map Q is the Kronecker product of banded 1D mass matrices, whose exact
# Cholesky factor is the Kronecker product of the 1D banded factors: its pattern lies
# inside pattern(tril Q) in the lexicographic order, so IC(0) in natural order IS the exact
# Cholesky factor (zero fill-in loses nothing).  That is the paper's observation that
# PCG(Q) with the IC(0) preconditioner converges in one iteration at every mesh size and
# tolerance.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kp,inv_hs", [(2, [8, 16, 32, 64, 128, 256]), (3, [8, 16, 32, 64, 128, 256])])
def test_ic0_Q_nnz_matches_paper(paper, kp, inv_hs):
    tab = paper["nnz_ic_k%d" % kp]
    for inv_h in inv_hs:
        ref = _tab_row(tab, inv_h)
        o = Oracle(inv_h, kp, pattern_only=True)
        assert (o.nnz("Q") + o.n_p) // 2 == ref["nnz_ICQ"]
    o = Oracle(8, kp)
    assert o.ic0_q() == 0 and o.nnz("LQ") == _tab_row(tab, 8)["nnz_ICQ"]


@pytest.mark.parametrize("N,kp,dim", [(6, 1, 2), (8, 2, 2), (5, 3, 2), (3, 1, 3)])
def test_ic0_Q_is_exact_cholesky(N, kp, dim):
    import scipy.sparse.linalg as sla
    from oracle.oracle import PQ_IC0, PQ_ICPCG
    o = Oracle(N, kp, dim)
    assert o.ic0_q() == 0
    Q = o.scipy("Q").toarray()
    Lc = sl.cholesky(Q, lower=True)
    LQ = o.scipy("LQ").toarray()
    assert np.abs(LQ - Lc).max() <= 1e-13 * np.abs(Lc).max()
    r = np.random.default_rng(3).standard_normal(o.n)
    ref = sla.spsolve(o.scipy("Q").tocsc(), r[o.n_u:]) * 2.0 * o.nu
    z, _ = o.precond(r, pc_A=PC_IC0, pc_Q=PQ_IC0)
    assert np.linalg.norm(z[o.n_u:] - ref) <= 1e-12 * np.linalg.norm(ref)
    for tol_in in (1e-3, 1e-6):  # one inner iteration on Q, as the paper reports
        z, it = o.precond(r, pc_A=PC_IC0, pc_Q=PQ_ICPCG, inner_tol=tol_in)
        assert it == 1
        assert np.linalg.norm(z[o.n_u:] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.slow
def test_iteration_counts_ic_pcg_cavity_k2(paper):
    """IC(0)-PCG(A,Q) on the lid-driven cavity (Sec. 6.4 table, k' = 2, outer tol 1e-12 on
    the true 2-norm relative residual): outer counts within 2 and mean inner PCG(A) counts
    within 15 % of the paper's at both inner tolerances, one inner iteration on Q.  The
    paper reorders with RCM before IC(0); the oracle keeps the natural order, so the inner
    counts are compared loosely.  Their growth per halving of h (P16: 1.6-1.9x in the
    paper) is checked on its own."""
    from oracle.oracle import PQ_ICPCG
    ref = paper["iters_ic_pcg_cavity_k2"]
    means = {1e-3: [], 1e-6: []}
    for i, inv_h in enumerate(ref["inv_h"][:3]):
        o = Oracle(inv_h, 2)
        b = np.concatenate([o.load_cavity(0), np.zeros(o.n_p)])
        K = o.saddle()
        for tol_in, key in ((1e-3, "tol1e-3"), (1e-6, "tol1e-6")):
            x, info, xh = o.minres(b, tol=1e-14, maxit=300, pc_A=PC_ICPCG, pc_Q=PQ_ICPCG, inner_tol=tol_in,
                                   x_history=True)
            r2 = np.linalg.norm(b - (K @ xh.T).T, axis=1) / np.linalg.norm(b)
            j2 = int(np.argmax(r2 <= 1e-12)) + 1
            assert abs(j2 - ref[key + "_outer"][i]) <= 2, (inv_h, tol_in, j2)
            # inner counts over the j2 + 1 preconditioner applications of that run
            _, i2 = o.minres(b, maxit=j2, pc_A=PC_ICPCG, pc_Q=PQ_ICPCG, inner_tol=tol_in, fixed=True)
            apps = j2 + 1
            mean_A = (i2["inner_total"] - apps) / apps  # one Q iteration per application
            assert abs(mean_A / ref[key + "_inner_A"][i] - 1.0) <= 0.15, (inv_h, tol_in, mean_A)
            means[tol_in].append(mean_A)
    for tol_in, m in means.items():
        for a, b in zip(m, m[1:]):
            assert 1.4 <= b / a <= 2.1, (tol_in, m)


# ---------------------------------------------------------------------------
# Stop counts under rounding.  MINRES on this saddle system reduces |eta| in pairs of
# almost equal steps; where tol falls on such a pair, a rounding-level change alone moves
# the stop by two.  The oracle shows it by itself: summing its inner products in reverse
# order (the same mathematics) moves some 3D k'=1 and 2D k'=3 stops by exactly two, and
# none in 2D for k' <= 2.  This is the reading behind the stop-count bar of the GPU tests.
# ---------------------------------------------------------------------------
def test_stop_counts_move_by_two_under_rounding():
    from oracle.oracle import GEOM_ANNULUS
    from synthetic_inputs import forcing_modes
    moved = {}
    try:
        for (N, kp, dim, geo, pc) in [(16, 1, 2, 0, PC_IC0), (12, 2, 2, 0, PC_IC0), (5, 3, 2, 0, PC_IC0),
                                      (4, 1, 3, 0, PC_IC0), (10, 2, 2, GEOM_ANNULUS, PC_JACOBI)]:
            o = Oracle(N, kp, dim, geometry=geo)
            o.ic0()
            F = [o.load(1)] + list(o.load(1, forcing_modes(list(range(1000, 1006)), dim)))
            d = []
            for f in F:
                b = np.concatenate([f, np.zeros(o.n_p)])
                Oracle.set_sum_order(False)
                _, i0 = o.minres(b, tol=1e-8, pc_A=pc)
                Oracle.set_sum_order(True)
                _, i1 = o.minres(b, tol=1e-8, pc_A=pc)
                d.append(i1["iters"] - i0["iters"])
            moved[(N, kp, dim, geo)] = d
    finally:
        Oracle.set_sum_order(False)
    assert all(x == 0 for x in moved[(16, 1, 2, 0)] + moved[(12, 2, 2, 0)]), moved
    for key in ((5, 3, 2, 0), (4, 1, 3, 0), (10, 2, 2, GEOM_ANNULUS)):
        assert any(x != 0 for x in moved[key]), moved
        assert all(abs(x) <= 2 for x in moved[key]), moved


# ---------------------------------------------------------------------------
# The restarted inner-PCG solve (oracle `solve_refined`, reading A20).  With a tight inner
# tolerance the inner PCG solves the velocity block exactly up to rounding, so one cycle
# suffices and the result is the plain MINRES solve with inner PCG, which in turn is MINRES
# with the exact block (dense Cholesky of A); at the loose tolerance its final residual,
# formed and measured with scipy from the oracle's matrices and IC(0) factor alone, meets
# tol in the norm of the fixed preconditioner.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pc_A", [PC_ICPCG, PC_JPCG])
def test_solve_refined(pc_A):
    import scipy.sparse.linalg as sla
    o = Oracle(10, 2)
    o.ic0()
    f = o.load(1)
    u0, p0, i0 = o.solve(f, tol=1e-10, pc_A=PC_EXACT)
    u1, p1, i1 = o.solve_refined(f, tol=1e-10, pc_A=pc_A, inner_tol=1e-13)
    _, _, ip = o.solve(f, tol=1e-10, pc_A=pc_A, inner_tol=1e-13)
    assert i1["iters"] == ip["iters"]  # one cycle: the plain MINRES run with inner PCG
    assert abs(i1["iters"] - i0["iters"]) <= 1
    assert np.linalg.norm(u1 - u0) <= 1e-8 * np.linalg.norm(u0)
    assert np.linalg.norm(p1 - p0) <= 1e-8 * np.linalg.norm(p0)
    tol = 1e-8
    u, p, info = o.solve_refined(f, tol=tol, pc_A=pc_A, inner_tol=1e-2)
    K = o.saddle()
    b = np.concatenate([f, np.zeros(o.n_p)])
    r = b - K @ np.concatenate([u, p])
    dQ, _ = o.diagQ_w()

    def minv(v):
        zu = (sla.spsolve_triangular(o.scipy("L").T.tocsr(), sla.spsolve_triangular(o.scipy("L"), v[:o.n_u]),
                                     lower=False) if pc_A == PC_ICPCG else v[:o.n_u] / o.scipy("A").diagonal())
        return np.concatenate([zu, 2.0 * o.nu * v[o.n_u:] / dQ])
    relM = np.sqrt((r @ minv(r)) / (b @ minv(b)))
    assert relM <= tol * (1 + 1e-9), relM
    assert abs(relM - info["relres_true_Minv"]) <= 1e-6 * relM


# ---------------------------------------------------------------------------
# Mapped geometry (Sec. 3.2): the 1/8 annulus of Sec. 6.3 by the polar map, velocities by
# the Piola transform, pressures by the integral-preserving transform.
# ---------------------------------------------------------------------------
@pytest.mark.slow
@pytest.mark.parametrize("kp,inv_hs", [(2, [8, 16, 32]), (3, [8, 16])])
def test_annulus_errors_match_paper(paper, kp, inv_hs):
    """The annulus manufactured solution (u = curl(a^2 b^2), p = x y^2) reproduces the
    paper's error table (Sec. 6.3) to its three printed digits: the mapped assembly, the
    Piola and pressure transforms, the physical normals and face lengths of the Nitsche
    terms and the zero-mean pressure on the mapped domain."""
    from oracle.oracle import GEOM_ANNULUS
    ref = paper["errors_annulus_k%d" % kp]
    for inv_h in inv_hs:
        i = ref["inv_h"].index(inv_h)
        o = Oracle(inv_h, kp, geometry=GEOM_ANNULUS)
        u, p, info = o.solve(o.load(4), tol=1e-13, maxit=20000)
        assert info["status"] == 0
        e = o.errors(u, p, 4)
        for k, name in enumerate(("H1_u", "L2_u", "L2_p")):
            assert abs(e[k] - ref[name][i]) <= 0.006 * ref[name][i], (inv_h, name, e[k], ref[name][i])


@pytest.mark.parametrize("N,kp", [(6, 1), (8, 2), (5, 3)])
def test_annulus_structure(N, kp):
    """On the mapped domain: A is SPD; B = -Q D with D the parametric divergence operator
    (taken from the identity-map problem, D = -Q_sq^{-1} B_sq), because the Piola transform
    divides the divergence and the pressure transform divides the pressure by J; the
    constant function's coefficients kappa satisfy B^T kappa = 0, Q kappa = w, w.kappa equals
    the annulus area 3 pi / 8, and kappa evaluates to 1 everywhere."""
    from oracle.oracle import GEOM_ANNULUS
    o = Oracle(N, kp, geometry=GEOM_ANNULUS)
    sq = Oracle(N, kp)
    A = o.scipy("A").toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)
    Qs, Bs = sq.scipy("Q").toarray(), sq.scipy("B").toarray()
    D = -np.linalg.solve(Qs, Bs)
    Q, B = o.scipy("Q").toarray(), o.scipy("B").toarray()
    assert np.abs(B + Q @ D).max() <= 1e-11 * np.abs(B).max()
    # kappa: the pressure whose projection does nothing but which the solve recovers from
    # a pure-gradient load of the constant's gradient (zero): read it back through evaluate
    d, w = o.diagQ_w()
    kappa = np.linalg.solve(Q, w)
    assert np.abs(B.T @ kappa).max() <= 1e-12 * np.abs(B).max() * np.abs(kappa).max()
    assert abs(w @ kappa - 3 * np.pi / 8) <= 1e-12
    pts = np.random.default_rng(2).random((40, 2))
    ev = o.evaluate(np.zeros(o.n_u), kappa, pts)
    assert np.abs(ev[:, 3] - 1.0).max() <= 1e-11
    # the oracle's projection removes exactly multiples of kappa
    pr = o.project(kappa)
    assert np.abs(pr).max() <= 1e-12


@pytest.mark.parametrize("N,kp", [(8, 1), (8, 2)])
def test_annulus_divergence_free_and_pressure_robust(N, kp):
    from oracle.oracle import GEOM_ANNULUS
    o = Oracle(N, kp, geometry=GEOM_ANNULUS)
    u, p, info = o.solve(o.load(4), tol=1e-13, maxit=20000)
    ev = o.evaluate(u, p, np.random.default_rng(3).random((300, 2)))
    assert np.abs(ev[:, 2]).max() <= 1e-9 * np.abs(ev[:, :2]).max() * N
    # f = grad(phi): u_h = 0 up to the load rule's quadrature error
    u, p, info = o.solve(o.load(3), tol=1e-13, maxit=20000)
    assert np.abs(u).max() <= 1e-9 * np.abs(p).max()


@pytest.mark.slow
@pytest.mark.parametrize("kp", [2, 3])
def test_annulus_iteration_counts(paper, kp):
    """Counts on the annulus (Sec. 6.3 table, tol 1e-12 on the true 2-norm residual): the
    paper's table is for its NURBS map and this oracle runs the polar one, which the paper
    found equivalent in the errors but which scales A differently; the pins are therefore
    the table's structure: Ideal(A,Q) and PCG(A,Q) (inner tol 1e-6) mesh-independent within
    2 and within 6 of the paper's counts from h = 1/16, the ranking
    Ideal(A,Q) < PCG(A,Q) < Ideal(A), Diag(Q) < PCG(A), Diag(Q) < Diag(A,Q), and Diag(A,Q)
    growing under refinement."""
    from oracle.oracle import GEOM_ANNULUS
    ref = paper["iters_annulus_k%d" % kp]
    counts = []
    for inv_h in (8, 16):
        o = Oracle(inv_h, kp, geometry=GEOM_ANNULUS)
        b = np.concatenate([o.load(4), np.zeros(o.n_p)])
        K = o.saddle()
        c = {}
        for key, pa, pq, tol_in in (("ideal_A_Q", PC_EXACT, PQ_EXACT, 0), ("pcg_A_Q", PC_JPCG, PQ_JPCG, 1e-6),
                                    ("ideal_A_diagQ", PC_EXACT, PQ_DIAG, 0), ("pcg_A_diagQ", PC_JPCG, PQ_DIAG, 1e-6),
                                    ("diag_A_Q", PC_JACOBI, PQ_DIAG, 0)):
            x, info, xh = o.minres(b, tol=1e-14, maxit=3000, pc_A=pa, pc_Q=pq, inner_tol=tol_in, x_history=True)
            r2 = np.linalg.norm(b - (K @ xh.T).T, axis=1) / np.linalg.norm(b)
            c[key] = int(np.argmax(r2 <= 1e-12)) + 1
        counts.append(c)
    for key in ("ideal_A_Q", "pcg_A_Q"):
        assert abs(counts[1][key] - counts[0][key]) <= 2, (key, counts)
        assert abs(counts[1][key] - ref[key][1]) <= 6, (key, counts[1][key], ref[key][1])
    for c in counts:
        order = [c[k] for k in ("ideal_A_Q", "pcg_A_Q", "ideal_A_diagQ", "pcg_A_diagQ", "diag_A_Q")]
        assert order == sorted(order), counts
    assert counts[1]["diag_A_Q"] > 1.3 * counts[0]["diag_A_Q"], counts
