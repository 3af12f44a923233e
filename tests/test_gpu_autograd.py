"""Differentiation through the solve (torch.autograd.Function with the hand-written adjoint),
on the GPU, checked two ways:

  - against the oracle's own adjoint gradient: for L = sum_b 0.5||u_b - t_b||^2 + 0.5 c||p_b||^2
    the oracle solves Acal lam_b = [u_b - t_b; c P^T p_b] and forms dL/df_b = lam_u,b and
    dL/dnu = -sum_b lam_u,b^T (A/nu) u_b from its own solutions u_b, p_b;
  - against central finite differences (step 1e-4), in nu and along a random direction in F.
    L is quadratic in F, so the F-difference is exact up to rounding and solve tolerance;
    in nu the truncation error is O(h^2), about 1e-8 relative.  The step is not smaller
    because the two solves behind a difference, each converged to tol, differ by about
    1e-11 relative (3D), which the quotient amplifies by 1/(2h).

Solves run at tol 1e-13.  Bar: 1e-6 relative for finite differences, 1e-7 against the
oracle adjoint.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from synthetic_inputs import forcing_modes, target_perturbations  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-13
CP = 0.3  # weight of the pressure term of the loss


def _loss(U, P, Ut):
    return 0.5 * ((U - Ut) ** 2).sum() + 0.5 * CP * (P ** 2).sum()


@pytest.fixture(scope="module", params=[(12, 2, 2), (4, 1, 3)], ids=["2d_k2_n12", "3d_k1_n4"])
def setup(request):
    from paper_1309_5048_amd import StokesProblem
    N, kp, dim = request.param
    print("\n[case] autograd N=%d k'=%d dim=%d" % (N, kp, dim), flush=True)
    gp = StokesProblem(N, kp, dim, 1.0)
    o = Oracle(N, kp, dim, 1.0)
    o.ic0()
    B = 3
    F = gp.load(True, forcing_modes(list(range(2000, 2000 + B)), dim))
    u0, _, _ = gp.solve(gp.load(True)[0].contiguous(), tol=TOL)
    Ut = u0.unsqueeze(0) + 1e-2 * torch.as_tensor(target_perturbations(gp.n_u, B), device="cuda")
    return gp, o, F, Ut


def _grads(gp, F, Ut, nu_val):
    from paper_1309_5048_amd import stokes_solve
    nu = torch.tensor(nu_val, dtype=torch.float64, device="cuda", requires_grad=True)
    Fv = F.clone().requires_grad_(True)
    U, P = stokes_solve(Fv, nu, gp, TOL)
    L = _loss(U, P, Ut)
    L.backward()
    return float(L), Fv.grad.detach().clone(), float(nu.grad), U.detach(), P.detach()


def _loss_at(gp, F, Ut, nu_val):
    from paper_1309_5048_amd import stokes_solve
    nu = torch.tensor(nu_val, dtype=torch.float64, device="cuda")
    with torch.no_grad():
        U, P = stokes_solve(F, nu, gp, TOL)
    return float(_loss(U, P, Ut))


def test_gradient_vs_oracle_adjoint(setup):
    gp, o, F, Ut = setup
    L, dF, dnu, U, P = _grads(gp, F, Ut, 1.0)
    Fh, Uth = F.cpu().numpy(), Ut.cpu().numpy()
    dnu_o = 0.0
    for b in range(F.shape[0]):
        uo, po, _ = o.solve(Fh[b], tol=TOL)
        lu, lp, _ = o.adjoint(uo - Uth[b], CP * po, tol=TOL)
        got = dF[b].cpu().numpy()
        assert np.linalg.norm(got - lu) <= 1e-7 * np.linalg.norm(lu), b
        dnu_o -= o.dnu_dot(lu, uo)
    assert abs(dnu - dnu_o) <= 1e-7 * abs(dnu_o), (dnu, dnu_o)


def test_gradient_vs_finite_differences(setup):
    gp, o, F, Ut = setup
    L, dF, dnu, U, P = _grads(gp, F, Ut, 1.0)
    h = 1e-4
    fd_nu = (_loss_at(gp, F, Ut, 1.0 + h) - _loss_at(gp, F, Ut, 1.0 - h)) / (2 * h)
    assert abs(fd_nu - dnu) <= 1e-6 * abs(dnu), (fd_nu, dnu)
    D = torch.as_tensor(np.random.default_rng(77).standard_normal(tuple(F.shape)), device="cuda")
    D *= float(F.norm()) / float(D.norm())
    fd_F = (_loss_at(gp, F + h * D, Ut, 1.0) - _loss_at(gp, F - h * D, Ut, 1.0)) / (2 * h)
    an_F = float((dF * D).sum())
    assert abs(fd_F - an_F) <= 1e-6 * abs(an_F), (fd_F, an_F)
    gp.set_nu(1.0)
