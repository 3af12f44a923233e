"""stokes_solve_noalloc (the entry point for callers that cannot allocate device memory)
against stokes_solve, through the C ABI: the same MINRES kernels on the same inputs, with the
work vectors in the library's static per-GPU array instead of the handle's workspace.

Two calls in a row on one GPU, the second on a smaller problem (the array keeps the first
call's contents), each for IC(0) and Jacobi blocks: iteration counts equal and u, p within
1e-12 (the kernels and their summation order are the same, so the results agree to
rounding; the FP64 parity bar against the oracle is 1e-10).  Then the error paths: a
preconditioner other than IC(0)/Jacobi and a problem above the 64 MiB workspace.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _close(a, b, tol):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    d = np.abs(a - b).max()
    assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b), np.linalg.norm(a - b) / np.linalg.norm(b)
    assert d <= tol * np.abs(b).max(), d / np.abs(b).max()


@pytest.mark.parametrize("case", [(24, 2), (10, 1)], ids=["first_n24_k2", "second_smaller_n10_k1"])
def test_noalloc_matches_solve(case):
    from paper_1309_5048_amd import PC_IC0, PC_JACOBI, StokesProblem
    N, kp = case
    print("\n[case] noalloc N=%d k'=%d" % (N, kp), flush=True)
    gp = StokesProblem(N, kp, 2, 1.0)
    f = gp.load(True)[0]
    for pc in (PC_IC0, PC_JACOBI):
        u_ref, p_ref, info_ref = gp.solve(f, tol=1e-10, precond=pc)
        u = torch.full((gp.n_u,), float("nan"), dtype=torch.float64, device="cuda")
        p = torch.full((gp.n_p,), float("nan"), dtype=torch.float64, device="cuda")
        info = gp.solve_noalloc(f, u, p, tol=1e-10, precond=pc)
        assert info["status"] == 0 and info_ref["status"] == 0
        assert info["iters"] == info_ref["iters"], (info["iters"], info_ref["iters"])
        _close(u, u_ref, 1e-12)
        _close(p, p_ref, 1e-12)
        assert abs(info["relres_true_Minv"] - info_ref["relres_true_Minv"]) <= 1e-6 * info_ref["relres_true_Minv"]
    gp.close()


def test_noalloc_rejects():
    from paper_1309_5048_amd import PC_ICPCG, StokesError, StokesProblem
    gp = StokesProblem(8, 1, 2, 1.0)
    f = gp.load(True)[0]
    u, p = gp.empty(gp.n_u), gp.empty(gp.n_p)
    with pytest.raises(StokesError):
        gp.solve_noalloc(f, u, p, precond=PC_ICPCG)
    gp.close()
    # n_u + n_p = 2*640*641 + 641^2 = 1,231,361 > 838,848
    big = StokesProblem(640, 1, 2, 1.0)
    f = big.load(True)[0]
    u, p = big.empty(big.n_u), big.empty(big.n_p)
    with pytest.raises(StokesError):
        big.solve_noalloc(f, u, p)
    big.close()
