/*
 * stokes.h -- C ABI of libstokes.so, an MI355X (gfx950) solver for the discrete Stokes
 * saddle-point system of a divergence-conforming (Raviart-Thomas type) B-spline
 * discretisation, by block-diagonally preconditioned MINRES.
 *
 * Method (Cortes & Coutinho, arXiv 1309.5048):
 *   Spaces (Sec. 3.2): on the unit square (dim = 2) or cube (dim = 3) with N uniform
 *     elements per direction, velocity component c has degree p = k'+1 in direction c and
 *     degree k' in the others, maximal continuity; the first/last function of direction c
 *     is removed (u.n = 0).  Pressure: degree k' in every direction, zero mean imposed
 *     after the solve.  Numbering: velocity component-major, x fastest; pressure after.
 *   Matrices (Sec. 4): [A]_ij = a(Phi_j,Phi_i) - eta_h(Phi_j,Phi_i) with the Nitsche form
 *     eta_h of eq. (nitsche_lhs), C_pen = 5(k'+1) (Sec. 6.2), h_F = 1/N; [B]_kj =
 *     -(div Phi_j, phi_k); system [A B^T; B 0][u; p] = [f; 0] (eq. stokes_linsys).
 *   Solver (Sec. 5): preconditioned MINRES with M = blkdiag(M_A, M_Q) (eq.
 *     general_precond_M), M_Q = Diag(Q)/(2 nu) (the scaled mass matrix Q_nu of Sec. 5.1
 *     replaced by its diagonal), M_A = IC(0) of A (Sec. 6.4), IC(0)-PCG on A (Sec. 6.4,
 *     relaxed inner tolerance) or Diag(A); and the other variants of Sec. 5.1 (inner
 *     Diag-CG on A and on Q, Ideal blocks by converged CG; STOKES_PC_*).  Stop when the
 *     preconditioned residual estimate |eta_j| <= tol * ||b||_{M^-1} (Sec. 5, M^{-1}-norm
 *     of the residual).
 *
 * Conventions
 *   - Every vector pointer is a DEVICE pointer to contiguous doubles (the caller owns it;
 *     the library never keeps it after the call returns).  Batched arrays are column-major
 *     with one right-hand side per column: F[r * n_u + i].
 *   - All work is ordered on the problem's stream (stokes_set_stream; default: the null
 *     stream).  Calls that return stokes_info synchronise that stream before returning.
 *   - A handle is not thread safe; distinct handles are independent.
 *   - Return codes: 0 OK; STOKES_NOT_CONVERGED (+1) the best iterate is still returned;
 *     STOKES_EINVAL (-1) bad argument / NaN input / unsupported (dim, p); STOKES_ENOMEM
 *     (-2) device allocation failed; STOKES_EHIP (-3) HIP runtime error (including a
 *     device-side wait that exceeded its spin limit); STOKES_EBREAKDOWN (-4) IC(0) pivot
 *     <= 0 after the last diagonal shift, or a negative Lanczos gamma^2.  The message of
 *     the last failure is returned by stokes_last_error.
 */
#ifndef STOKES_H
#define STOKES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STOKES_OK 0
#define STOKES_NOT_CONVERGED 1
#define STOKES_EINVAL (-1)
#define STOKES_ENOMEM (-2)
#define STOKES_EHIP (-3)
#define STOKES_EBREAKDOWN (-4)

/* Block preconditioner M = blkdiag(M_A, M_Q).  M_Q = Diag(Q)/(2 nu) unless stated. */
#define STOKES_PC_IC0 0    /* M_A = L L^T, IC(0) of A in natural order (Sec. 6.4)          */
#define STOKES_PC_ICPCG 1  /* M_A^{-1} r = IC(0)-preconditioned CG on A r, relative 2-norm
                              tolerance stokes_set_inner_tol (default 1e-2), x0 = 0      */
#define STOKES_PC_JACOBI 2 /* M_A = Diag(A)  (the Diag(A,Q) variant of Sec. 5.1)          */
#define STOKES_PC_JPCG 4   /* M_A^{-1} r = Diag(A)-preconditioned CG on A r, tolerance as
                              for STOKES_PC_ICPCG: the PCG(A), Diag(Q) variant of Sec. 5.1
                              (the paper's tables use the inner tolerance 1e-6)             */
#define STOKES_PC_PCGAQ 5  /* PCG(A,Q) of Sec. 5.1: STOKES_PC_JPCG on the velocity block and
                              M_Q^{-1} r = 2 nu x, x from Diag(Q)-preconditioned CG on
                              Q x = r (same tolerance)                                     */
#define STOKES_PC_ICPCG_AQ 7 /* IC(0)-PCG(A,Q) of Sec. 6.4 (the paper's best strategy, tables
                              of IC(0)-PCG(A,Q)): STOKES_PC_ICPCG on the velocity block and
                              M_Q^{-1} r = 2 nu x, x from CG on Q x = r preconditioned by
                              IC(0) of the pressure mass matrix Q (natural order, pattern of
                              tril(Q); built on first use), same inner tolerance; its fixed
                              counterpart is blkdiag(IC(0) of A, IC(0) of Q / (2 nu))        */
/* STOKES_PC_ICPCG, STOKES_PC_JPCG, STOKES_PC_PCGAQ and STOKES_PC_ICPCG_AQ change with their
 * input: by default
 * MINRES runs once with them and stops on its own estimate, as in Sec. 5.1;
 * stokes_set_restarts selects restarts on the true residual instead.                  */
#define STOKES_PC_IDEAL 3  /* Ideal(A,Q) of Sec. 5.1, M = blkdiag(A, Q/(2 nu)): each block
                              solved by Diag-preconditioned CG to the fixed relative residual
                              1e-12 (at most 100000 iterations; stokes_set_inner_tol and
                              stokes_set_maxit do not apply), so MINRES runs once, without
                              restarts, on a preconditioner fixed up to rounding.  Iterative
                              block solves stand in for the paper's direct ones.  FP64 only
                              (STOKES_MIXED: STOKES_EINVAL); relres_true_Minv is measured
                              in the blkdiag(Diag(A), Diag(Q)/(2 nu)) norm.                */
#define STOKES_PC_IDEAL_A 6 /* Ideal(A) + Diag(Q) of Sec. 5.1, M = blkdiag(A, Diag(Q)/(2 nu)):
                              the velocity block as for STOKES_PC_IDEAL, the pressure block
                              by its diagonal; one MINRES run; FP64 only                   */

/* Arithmetic of the Krylov iteration. */
#define STOKES_FP64 0  /* everything in double precision                                  */
#define STOKES_MIXED 1 /* iterative refinement: FP64 true residual, zero-mean projection
                          and Lanczos/Givens scalars; inner MINRES with FP32 matrices,
                          FP32 IC(0) factors and triangular solves, FP32 accumulation.
                          Refines until the true M^{-1}-norm residual is <= tol / 10,
                          so that the solution's error stays within that of an FP64 solve
                          at tol (status 0 once it is <= tol)                             */

typedef struct stokes_problem stokes_problem; /* opaque: owns all device matrices,
                                                  factors, schedules and workspaces   */

typedef struct {
  int32_t iters;             /* MINRES iterations (summed over refinement steps if MIXED) */
  int32_t inner_iters_total; /* inner CG iterations (both blocks) summed over the solve    */
  int32_t status;            /* return code of this right-hand side                       */
  int32_t ic_shift_steps;    /* IC(0) diagonal-shift retries used at setup (0 = none)     */
  int32_t refine_cycles;     /* MINRES runs on the true residual (1 unless MIXED, or an
                                inner-CG preconditioner with stokes_set_restarts > 0)      */
  int32_t reserved;          /* zero                                                       */
  double relres_est;         /* |eta|/gamma_1 at exit (M^{-1}-norm estimate)              */
  double relres_true_2;      /* ||b - Acal x||_2 / ||b||_2, computed on the device          */
  double relres_true_Minv;   /* ||b - Acal x||_{M^-1} / ||b||_{M^-1} (IC(0)/Jacobi M)       */
  double setup_ms;           /* time of stokes_setup (assembly, ordering, IC(0))          */
  double solve_ms;           /* device time of this solve (hipEvents on the stream)       */
} stokes_info;

/* Forcing description for stokes_load.  f_d(x) = [manufactured]_d(x)
 *   + sum_m amp[r][d][m] * sin(pi * (wave[r][m][0] x + wave[r][m][1] y [+ wave[r][m][2] z])
 *                              + phase[r][d][m]).
 * Manufactured: u = curl psi, psi = x^2(1-x)^2 y^2(1-y)^2 (2D) or u = curl(g,g,g),
 * g = phi(x)phi(y)phi(z), phi(t) = t^2(1-t)^2 (3D); p = prod_d cos(pi x_d);
 * f = -nu Lap u + grad p.  Arrays are HOST pointers, may be NULL when nmodes = 0. */
typedef struct {
  int32_t manufactured; /* 1: include the manufactured forcing, 0: modes only          */
  int32_t nmodes;       /* sinusoid modes per component (0..64)                         */
  const double* amp;    /* [nrhs][dim][nmodes]                                          */
  const int32_t* wave;  /* [nrhs][nmodes][dim]                                          */
  const double* phase;  /* [nrhs][dim][nmodes]                                          */
} stokes_forcing;

/* Build the problem: the spaces of Sec. 3.2 and their sparsity (host), Gauss-quadrature
 * assembly of A (the Nitsche form of Sec. 4, eq. nitsche_lhs), B, B^T (eq. stokes_linsys),
 * diag(Q) and w (integrals of the pressure functions) (device), level schedules of the
 * triangular solves (host) and the IC(0) factor of A (Sec. 6.4; device, shift retries
 * alpha = 1e-3, 1e-2, 1e-1 of diag(A) on breakdown).
 * n: elements per direction (1..4096); p: pressure degree k' (1..3); dim: 2 or 3;
 * nu > 0.  On success *out owns the problem; on failure *out = NULL. */
int stokes_setup(int n, int p, int dim, double nu, stokes_problem** out);

/* The same on a mapped domain (Sec. 3.2): the discrete spaces are pushed forward from the
 * parametric unit square by the geometry map F, velocities by the Piola transform
 * Phi = DF Phihat / det DF (divergence and normal component preserving), pressures by the
 * integral-preserving transform phi = phihat / det DF.
 *   STOKES_GEOMETRY_SQUARE:  the identity map (stokes_setup).
 *   STOKES_GEOMETRY_ANNULUS: one eighth of the annulus 1 < r < 2, 0 < theta < pi/4 (the
 *     domain of Sec. 6.3) by the polar map x = r cos(theta), y = r sin(theta),
 *     r = 1 + xi_0, theta = (pi/4) xi_1; 2D only.  Nitsche face terms use the physical
 *     outward normal and h_F = 1/(N |DF^{-1} n|), the element length normal to the face;
 *     matrices use k'+3 Gauss points per direction, loads k'+5.  The zero-mean pressure
 *     subtracts multiples of the constant function, whose coefficients are Q^{-1} w here.
 *     stokes_load evaluates the forcing at the physical points; stokes_load_cavity
 *     returns STOKES_EINVAL.
 * Other values, or the annulus with dim = 3: STOKES_EINVAL. */
#define STOKES_GEOMETRY_SQUARE 0
#define STOKES_GEOMETRY_ANNULUS 1
int stokes_setup_geometry(int n, int p, int dim, double nu, int geometry, stokes_problem** out);

/* The same with the Nitsche penalty constant of Sec. 4 chosen by the caller: the face terms
 * penalise with 2 nu c_pen / h_F.  c_pen < 0 selects the value of the paper's experiments,
 * C_pen = 5 (k'+1) (what stokes_setup and stokes_setup_geometry use); c_pen >= 0 is taken as
 * given (a value too small for coercivity leaves A indefinite: IC(0) then breaks down and
 * the shift retries of stokes_setup apply; ic_shift_steps reports how many were needed, and
 * STOKES_EBREAKDOWN is returned when the last shift fails).  A non-finite c_pen:
 * STOKES_EINVAL.  The same penalty enters the cavity load of stokes_load_cavity. */
int stokes_setup_nitsche(int n, int p, int dim, double nu, int geometry, double c_pen,
                         stokes_problem** out);

/* Sizes: n_u velocity unknowns, n_p pressure unknowns. */
int stokes_sizes(const stokes_problem* pb, int64_t* n_u, int64_t* n_p);

/* Order all later work of this handle on the given hipStream_t (NULL = null stream). */
int stokes_set_stream(stokes_problem* pb, void* hip_stream);

/* Change the viscosity without re-assembly: A and its IC(0) factor scale with nu
 * (A ~ nu, L ~ sqrt(nu)), M_Q = Diag(Q)/(2 nu). */
int stokes_set_nu(stokes_problem* pb, double nu);

/* Inner CG relative tolerance of STOKES_PC_ICPCG, STOKES_PC_JPCG and STOKES_PC_PCGAQ
 * (default 1e-2) and iteration limits (defaults: outer 20000, inner 200 per block and
 * application).  The Ideal preconditioners use their own fixed values.  Non-positive values
 * keep the current setting. */
int stokes_set_inner_tol(stokes_problem* pb, double rtol);
int stokes_set_maxit(stokes_problem* pb, int outer, int inner);

/* Outer method of the inner-CG preconditioners (STOKES_PC_ICPCG, STOKES_PC_JPCG,
 * STOKES_PC_PCGAQ, STOKES_PC_ICPCG_AQ) in STOKES_FP64.  Inner CG stopped at a relative tolerance is a nonlinear
 * preconditioner, while MINRES (Sec. 5) is built on a fixed SPD one, so its estimate |eta|
 * measures the residual in a norm that changes between applications.
 *   max_cycles = 0 (default): the paper's method (Sec. 5.1, Sec. 6.2/6.4 tables): one MINRES
 *     run, stopped when |eta_j| <= tol * gamma_1; relres_true_Minv then reports where the
 *     true residual landed.
 *   max_cycles in 1..30: MINRES restarted from the FP64 true residual until
 *     ||b - Acal x||_{M^-1} <= tol ||b||_{M^-1} for the fixed block preconditioner the inner
 *     solves approximate (M_A = IC(0) for STOKES_PC_ICPCG and STOKES_PC_ICPCG_AQ, Diag(A)
 *     otherwise; M_Q = IC(0) of Q / (2 nu) for STOKES_PC_ICPCG_AQ, Diag(Q)/(2 nu)
 *     otherwise), each cycle asking for the remaining reduction (at most 0.5), at most
 *     max_cycles cycles; status STOKES_NOT_CONVERGED if that norm still misses tol.
 * Other values: STOKES_EINVAL. */
int stokes_set_restarts(stokes_problem* pb, int max_cycles);

/* STOKES_MIXED refinement: relative residual reduction asked of the first FP32 inner MINRES
 * (default 1e-4, must be < 1).  Later cycles ask for the reduction still missing to reach
 * tol / 10 (with a factor 2 of margin), but never for more than rtol.  At most 30 cycles.
 * Non-positive values keep the current setting. */
int stokes_set_refine_tol(stokes_problem* pb, double rtol);

/* Assemble nrhs load vectors [f]_i = (f, Phi_i) on the device (Gauss rule with k'+4
 * points per direction) into f_dev [nrhs][n_u]. */
int stokes_load(stokes_problem* pb, const stokes_forcing* spec, int nrhs, double* f_dev);

/* Load vector with tangential boundary data imposed weakly (2D only):
 * f_i = (f, Phi_i) + l_h(Phi_i), l_h the Nitsche form of eq. nitsche_rhs (Sec. 4),
 * l_h(v) = sum_F int_F 2 nu ( -((sym grad v) n).g + (C_pen/h_F) g.v ) dS, Gauss rule with
 * k'+2 points per direction (exact for these data).  f_dev [n_u] (device) is overwritten.
 *   STOKES_CAVITY_LID:    the lid-driven cavity of Sec. 6.4: f = 0, g = (1, 0) on y = 1,
 *                         g = 0 on the other sides.
 *   STOKES_CAVITY_VERIFY: u = (x(1-x)(1-2y), -(1-2x)y(1-y)) (= curl of x(1-x)y(1-y)), p = 0,
 *                         f = -nu Lap u, g = u on every side.  u lies in the discrete space
 *                         for every k', so the solve returns it up to the solver tolerance.
 * Uses the current viscosity (stokes_set_nu).  3D or another kind: STOKES_EINVAL. */
#define STOKES_CAVITY_LID 0
#define STOKES_CAVITY_VERIFY 1
int stokes_load_cavity(stokes_problem* pb, int kind, double* f_dev);

/* Solve [A B^T; B 0][u; p] = [f; 0] (eq. stokes_linsys) by preconditioned MINRES (Sec. 5)
 * from x0 = 0: f [n_u] in, u [n_u] and pr [n_p] out (pr has zero mean, w.pr = 0, the
 * filtering of Sec. 6.2).  tol: relative M^{-1}-norm residual (e.g. 1e-8).
 * precond: STOKES_PC_*.  info may be NULL. */
int stokes_solve(stokes_problem* pb, const double* f, double* u, double* pr, double tol, int precond,
                 stokes_info* info);

/* nrhs independent solves of Sec. 5's MINRES in one launch sequence (block SpMM / block
 * triangular solves,
 * per-column Lanczos and Givens scalars, converged columns frozen).  F [nrhs][n_u],
 * U [nrhs][n_u], P [nrhs][n_p]; infos [nrhs] may be NULL.  precision: STOKES_FP64 or
 * STOKES_MIXED.  nrhs in 1..16. */
int stokes_solve_batched(stokes_problem* pb, int nrhs, const double* F, double* U, double* P,
                         double tol, int precond, int precision, stokes_info* infos);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): stokes_solve without any allocation.
 * precond must be STOKES_PC_IC0 or STOKES_PC_JACOBI (FP64, one right-hand side); the MINRES
 * work vectors live in a static device array of the library, 64 MiB per GPU, held from the
 * library's first setup on that GPU until the process ends, instead of in the handle's
 * lazily allocated workspace.  Limit: 10 vectors of n_u + n_p doubles (each rounded up to
 * 256 bytes) must fit, i.e. n_u + n_p <= 838,848 (the N = 512, k' = 2 problem fits);
 * larger problems, other preconditioners and a null pointer give STOKES_EINVAL.  The array
 * is shared by every handle on that GPU and keeps the last call's contents (every value
 * the solve reads is written by the call first): calls that overlap on one GPU, from
 * other threads or streams, race.  Same results, info and return codes as stokes_solve
 * (info->solve_ms from events created at setup); kernel timing (stokes_profile) is
 * paused during the call.  f [n_u] in, u [n_u] and pr [n_p] out, device pointers. */
int stokes_solve_noalloc(stokes_problem* pb, const double* f, double* u, double* pr, double tol, int precond,
                         stokes_info* info);

/* Single right-hand side with a precision choice (STOKES_FP64 is stokes_solve). */
int stokes_solve_precision(stokes_problem* pb, const double* f, double* u, double* pr, double tol,
                           int precond, int precision, stokes_info* info);

/* Adjoint solve for a loss L(u, p) of the zero-mean solution (Acal is symmetric, Sec. 5,
 * so the transposed system is solved by the same MINRES): with g = [g_u; g_p]
 * [n_u + n_p] (dL/du, dL/dp), solves Acal lambda = [g_u; g_p - w (kappa.g_p)/(w.kappa)]
 * (kappa the constant function's pressure coefficients, all ones on the unit square)
 * (Acal is symmetric, same MINRES and preconditioner); lambda [n_u + n_p] out with a
 * zero-mean pressure part.  Then dL/df = lambda_u and dL/dnu = -lambda_u^T (A/nu) u. */
int stokes_solve_adjoint(stokes_problem* pb, const double* g, double* lambda, double tol, int precond,
                         stokes_info* info);

/* Batched adjoint: G [nrhs][n_u + n_p] in, Lambda [nrhs][n_u + n_p] out. */
int stokes_solve_adjoint_batched(stokes_problem* pb, int nrhs, const double* G, double* Lambda,
                                 double tol, int precond, stokes_info* infos);

/* out[r] = lam_u[r]^T A u[r] / nu for r < nrhs (device arrays [nrhs][n_u]): the viscosity
 * derivative of the adjoint gradient, A being proportional to nu (the form a and the Nitsche
 * terms of Sec. 4 all carry the factor 2 nu).  out is a HOST array of nrhs doubles (any
 * nrhs >= 1), so the call synchronises the stream. */
int stokes_dnu_dot(stokes_problem* pb, int nrhs, const double* lam_u, const double* u, double* out);

/* Products with the assembled operators, for checks: y = Acal x (x, y [n_u + n_p]). */
int stokes_apply(stokes_problem* pb, const double* x, double* y);

/* y = M^{-1} r with the chosen block preconditioner (r, y [n_u + n_p]); *inner_iters
 * receives the inner CG iteration count of both blocks (0 without inner CG; may be NULL). */
int stokes_apply_precond(stokes_problem* pb, int precond, const double* r, double* y, int* inner_iters);

/* Copy the assembled matrices to HOST buffers (for checks).  which: 0 = saddle Acal
 * (rows n_u + n_p, columns sorted), 1 = the IC(0) factor L (rows n_u, lower triangle of
 * A's pattern, diagonal last), 2 = the IC(0) factor of the pressure mass matrix Q (rows
 * n_p, lower triangle of Q's pattern, diagonal last; factorised on first use, Sec. 6.4).
 * Pass NULL arrays to query *nnz only. rowptr is int64. */
int stokes_export_csr(stokes_problem* pb, int which, int64_t* nnz, int64_t* rowptr, int32_t* col,
                      double* val);

/* diag(Q) and w = Q 1 (integrals of the pressure functions) to HOST arrays [n_p]. */
int stokes_export_pressure_mass(stokes_problem* pb, double* diagQ, double* w);

/* Number of dependency levels of the forward / backward triangular solves (host). */
int stokes_levels(const stokes_problem* pb, int* fwd_levels, int* bwd_levels);

/* Live kernel timing with HIP events recorded on the problem's stream around each timed
 * launch of the MINRES loop.  enable = 1 resets the totals and starts timing, 0 stops it,
 * any other value only reads.  ms[5] / counts[5] (HOST, may be NULL) receive the summed
 * device time and the number of launches per category: [0] saddle SpMV, [1] forward
 * triangular solve, [2] backward triangular solve, [3] Lanczos update, [4] Givens and
 * w/x update.  Synchronises the stream. */
int stokes_profile(stokes_problem* pb, int enable, double* ms, int64_t* counts);

const char* stokes_last_error(const stokes_problem* pb);
void stokes_destroy(stokes_problem* pb);

#ifdef __cplusplus
}
#endif
#endif /* STOKES_H */
