"""Differentiation through the Stokes solve with a hand-written adjoint.

forward(F, nu): U, P = solve of [A(nu) B^T; B 0][u; p] = [f; 0] for every row f of F
(assembled load vectors), pressure zero-mean.  The system matrix is symmetric (Sec. 5 of
the paper), so the adjoint reuses MINRES with the same preconditioner:
  Acal [lam_u; lam_p] = [dL/du; P^T dL/dp],  P^T g_p = g_p - w (1.g_p)/(w.1)
  dL/dF = lam_u,   dL/dnu = -sum_b lam_u,b^T (A/nu) u_b      (A is proportional to nu).
"""
import torch

from . import _native as N
from .solver import StokesError


def _require_converged(infos, what):
    """A gradient built on an unconverged solve is wrong by more than the tolerance: raise."""
    for r, info in enumerate(infos):
        if info["status"] != 0:
            raise StokesError(N.STOKES_NOT_CONVERGED if info["status"] > 0 else info["status"],
                              "%s of right-hand side %d did not converge (status %d)" % (what, r, info["status"]))


class StokesSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, F, nu, problem, tol=1e-8, precond=N.PC_IC0):
        nu_val = float(nu)
        if abs(nu_val - problem.nu) > 0.0:
            problem.set_nu(nu_val)
        U, P, infos = problem.solve_batched(F.detach().contiguous(), tol=tol, precond=precond)
        _require_converged(infos, "forward solve")
        ctx.problem, ctx.tol, ctx.precond = problem, tol, precond
        ctx.save_for_backward(U)
        ctx.infos = infos
        return U, P

    @staticmethod
    def backward(ctx, gU, gP):
        problem = ctx.problem
        (U,) = ctx.saved_tensors
        R = U.shape[0]
        if gU is None:
            gU = torch.zeros_like(U)
        if gP is None:
            gP = torch.zeros(R, problem.n_p, dtype=U.dtype, device=U.device)
        G = torch.cat([gU.reshape(R, problem.n_u), gP.reshape(R, problem.n_p)], dim=1).contiguous()
        Lam, infos = problem.solve_adjoint(G, tol=ctx.tol, precond=ctx.precond)
        _require_converged(infos, "adjoint solve")
        lam_u = Lam[:, : problem.n_u].contiguous()
        dnu = -sum(problem.dnu_dot(lam_u, U))
        grad_nu = torch.tensor(dnu, dtype=torch.float64, device=U.device)
        return lam_u, grad_nu, None, None, None


def stokes_solve(F, nu, problem, tol=1e-8, precond=N.PC_IC0):
    """Differentiable batched solve: returns (U [B, n_u], P [B, n_p])."""
    if not torch.is_tensor(nu):
        nu = torch.tensor(float(nu), dtype=torch.float64, device=F.device)
    return StokesSolve.apply(F, nu, problem, tol, precond)
