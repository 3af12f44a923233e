"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only names the workloads and
draws the random numbers that define them (numpy ``default_rng`` with fixed seeds),
so that both sides receive identical inputs.

Workloads (unit square / cube, uniform N^dim mesh, pressure degree kp = k',
velocity degree k'+1, maximal continuity, C_pen = 5(k'+1), nu = 1):
  c0_2d_k1_n16      N=16,  k'=1, 2D, manufactured forcing, tol 1e-8 (small parity case)
  c1_2d_k2_n256     N=256, k'=2, 2D, manufactured forcing, FP64 (headline workload)
  c2_2d_k2_n512     N=512, k'=2, 2D, mixed FP32/FP64 vs FP64
  c3_3d_k1_n32_r16  N=32,  k'=1, 3D, 16 forcings: manufactured + 8 random sinusoid modes
  c4_2d_k2_n256_r8  N=256, k'=2, 2D, 8 forcings (seeds 2000+b), loss targets (seeds 3000+b)

Random forcing recipe (per right-hand side r, rng = default_rng(seed_r)):
  amp   = rng.standard_normal((dim, M))            mode amplitudes a_{d,m} ~ N(0,1)
  wave  = rng.integers(1, 5, size=(M, dim))        integer wave vectors k_m in {1..4}^dim
  phase = rng.uniform(0, 2 pi, size=(dim, M))      phases
  f_d(x) = f_d^manufactured(x) + sum_m a_{d,m} sin(pi k_m . x + phase_{d,m})
"""
import numpy as np

WORKLOADS = {
    "c0_2d_k1_n16": dict(N=16, kp=1, dim=2, nu=1.0, tol=1e-8, nrhs=1, seeds=None),
    "c1_2d_k2_n256": dict(N=256, kp=2, dim=2, nu=1.0, tol=1e-8, nrhs=1, seeds=None),
    "c2_2d_k2_n512": dict(N=512, kp=2, dim=2, nu=1.0, tol=1e-8, nrhs=1, seeds=None),
    "c3_3d_k1_n32_r16": dict(N=32, kp=1, dim=3, nu=1.0, tol=1e-8, nrhs=16, seeds=list(range(1000, 1016))),
    "c4_2d_k2_n256_r8": dict(N=256, kp=2, dim=2, nu=1.0, tol=1e-8, nrhs=8, seeds=list(range(2000, 2008))),
}

NMODES = 8


def forcing_modes(seeds, dim, nmodes=NMODES):
    """Mode tables (amp [R,dim,M] f64, wave [R,M,dim] int32, phase [R,dim,M] f64), one row per seed."""
    R = len(seeds)
    amp = np.zeros((R, dim, nmodes))
    wave = np.zeros((R, nmodes, dim), np.int32)
    phase = np.zeros((R, dim, nmodes))
    for r, s in enumerate(seeds):
        rng = np.random.default_rng(int(s))
        amp[r] = rng.standard_normal((dim, nmodes))
        wave[r] = rng.integers(1, 5, size=(nmodes, dim))
        phase[r] = rng.uniform(0.0, 2.0 * np.pi, size=(dim, nmodes))
    return amp, wave, phase


def target_perturbations(n_u, batch, base_seed=3000):
    """xi_b ~ N(0, I) of length n_u for b = 0..batch-1 (default_rng(base_seed + b))."""
    return np.stack([np.random.default_rng(base_seed + b).standard_normal(n_u) for b in range(batch)])


def random_vector(n, seed):
    """A plain N(0,1) vector, for solver-only checks."""
    return np.random.default_rng(int(seed)).standard_normal(n)
