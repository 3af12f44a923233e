"""Benchmark: time-to-solution of block-diagonally preconditioned MINRES for the
divergence-conforming B-spline Stokes system on one MI355X.

Headline workload (one "step" = one complete solve from the assembled load vector to the
zero-mean (u, p), inputs resident in HBM): 2D unit square, N = 256 elements per
direction, pressure degree k' = 2 (velocity degree 3), nu = 1, manufactured forcing,
FP64, M = blkdiag(IC(0) of A, Diag(Q)/(2 nu)), relative M^{-1}-norm residual 1e-8.

Printed: one JSON line with the headline value (seconds per solve), MINRES iterations/s,
a roofline object for the dominant kernel (algorithmic bytes per launch over its average
launch time, measured with HIP events on the solver's stream during the timed solves), the
same for the saddle SpMV, the CPU oracle timed on one host core on a bounded sample, and
the variant comparisons (IC(0)-PCG, mixed precision at N = 512, batched 3D, adjoint).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-solution @ rel.res 1e-8 (s), MINRES iters/s, SpMV HBM GB/s vs peak"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def trsv_bytes(nnzL, n_u, R=1, wbytes=8):
    """Algorithmic bytes of one triangular solve: every off-diagonal factor entry (value +
    int32 column) and diagonal once, the right-hand side read and the result written once."""
    return (wbytes + 4) * (nnzL - n_u) + wbytes * n_u + 2 * wbytes * n_u * R


def spmv_bytes(nnz, n, R=1, wbytes=8):
    """Algorithmic bytes of one saddle product q = Acal z with the fused dot q.z: values and
    int32 columns once, row pointers, z read once, q written once."""
    return (wbytes + 4) * nnz + 4 * (n + 1) + 2 * wbytes * n * R


def measured_traffic():
    """HBM bytes per launch of the triangular solve and the saddle product, from the committed
    rocprofv3 counter summary, while the kernel sources are the ones it was measured on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "trsv_spmv_c1_2d_k2_n256_traffic.md")
    try:
        txt = open(path).read()
    except OSError:
        return {}
    m = re.search(r"traffic_source_sha256: ([0-9a-f]+)", txt)
    t = re.search(r"traffic_bytes_per_launch: trsv=(\d+) spmv=(\d+)", txt)
    h = hashlib.sha256()
    for src in ("k_trsv.hip", "k_krylov.hip"):
        with open(os.path.join(ROOT, "paper_1309_5048_amd", "csrc", src), "rb") as fh:
            h.update(fh.read())
    if not m or not t or m.group(1) != h.hexdigest():
        return {}
    return {"trsv_fwd": int(t.group(1)), "trsv_bwd": int(t.group(1)), "spmv": int(t.group(2))}


def sync():
    import torch
    torch.cuda.synchronize()


def timed_solves(gp, f, steps, warmup, **kw):
    for _ in range(warmup):
        gp.solve(f, **kw)
    sync()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(gp.solve(f, **kw)[2])
    sync()
    return (time.perf_counter() - t0) / steps, infos


def cpu_baseline(N, kp, dim, iters_needed, sample_iters):
    """Oracle (one host core, FP64) on a bounded sample: setup and IC(0) untimed, then
    `sample_iters` MINRES-IC(0) iterations timed; time-to-solution extrapolated to the
    iteration count the solve needs."""
    from oracle.oracle import Oracle
    import numpy as np
    t = time.perf_counter()
    o = Oracle(N, kp, dim, 1.0)
    o.ic0()
    f = o.load(1)
    t_setup = time.perf_counter() - t
    b = np.concatenate([f, np.zeros(o.n_p)])
    t0 = time.perf_counter()
    o.minres(b, maxit=sample_iters, fixed=True)
    dt = time.perf_counter() - t0
    ips = sample_iters / dt
    return {"value": iters_needed / ips, "unit": "s", "cores": 1, "kind": "oracle",
            "iters_per_s": ips,
            "sample": "%d MINRES-IC(0) iterations of the N=%d k'=%d dim=%d system (setup %.1f s untimed), "
                      "extrapolated to %d iterations" % (sample_iters, N, kp, dim, t_setup, iters_needed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extra", action="store_true", help="skip the variant comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=150)
    ap.add_argument("--precond", default="ic0", choices=["ic0", "pcgAQ", "jpcg", "icpcg", "ideal"],
                    help="preconditioner of the timed solves (default ic0, the headline); the others "
                         "report time and iteration counts only (their inner-CG kernels are not in the "
                         "live per-kernel timing), for profiling")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the solves, run a plain elementwise copy of MIB MiB three times "
                         "(reads and writes MIB MiB each): the reference for scaling memory counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this solver path is built and measured on a single "
              "MI355X (no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_5048_amd import StokesProblem, PC_IC0, PC_ICPCG, PC_IDEAL, PC_IDEAL_A, PC_JPCG, PC_PCGAQ, MIXED, FP64, CAVITY_LID

    torch.cuda.set_device(0)
    N, kp, dim, tol = 256, 2, 2, 1e-8
    log("setup N=%d k'=%d dim=%d" % (N, kp, dim))
    t = time.perf_counter()
    gp = StokesProblem(N, kp, dim, 1.0)
    setup_s = time.perf_counter() - t
    f = gp.load(True)[0]
    nnz = gp.export_csr(0)[1].size
    nnzL = gp.export_csr(1)[1].size
    n = gp.n_u + gp.n_p
    lev_f, lev_b = gp.levels()
    log("n_u=%d n_p=%d nnz=%d nnzL=%d levels=%d/%d setup %.1fs" % (gp.n_u, gp.n_p, nnz, nnzL, lev_f, lev_b, setup_s))

    if args.precond != "ic0":
        pc = {"pcgAQ": PC_PCGAQ, "jpcg": PC_JPCG, "icpcg": PC_ICPCG, "ideal": PC_IDEAL}[args.precond]
        gp.set_inner_tol(1e-2)
        sec, infos = timed_solves(gp, f, args.steps, args.warmup, tol=tol, precond=pc)
        log("solve %.4f s, %d iterations, %d inner, relres %.2e" % (
            sec, infos[-1]["iters"], infos[-1]["inner_iters_total"], infos[-1]["relres_true_Minv"]))
        print(json.dumps({
            "metric": "time-to-solution @ rel.res 1e-8 (s), MINRES iters/s, SpMV HBM GB/s vs peak",
            "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "c1_2d_k2_n256", "N": N, "kprime": kp, "dim": dim, "nu": 1.0, "tol": tol,
                       "precond": args.precond, "inner_tol": 1e-2, "forcing": "manufactured"},
            "iters": infos[-1]["iters"], "inner_iters_total": infos[-1]["inner_iters_total"],
            "relres_true_Minv": infos[-1]["relres_true_Minv"], "roofline": None}), flush=True)
        return

    # warmup, then the timed solves with live kernel timing on the solver's stream
    for _ in range(args.warmup):
        gp.solve(f, tol=tol, precond=PC_IC0)
    sync()
    gp.profile(1)
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        u, p, info = gp.solve(f, tol=tol, precond=PC_IC0)
        infos.append(info)
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    prof = gp.profile(0)
    iters = infos[-1]["iters"]
    log("solve %.4f s, %d iterations, relres %.2e" % (sec, iters, infos[-1]["relres_true_Minv"]))

    traffic = measured_traffic()

    def roof(name, bytes_per_launch):
        ms, cnt = prof[name]
        if cnt == 0:
            return None
        avg_s = ms / cnt / 1e3
        gbs = bytes_per_launch / avg_s / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": traffic.get(name), "kernel": name,
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "launches": int(cnt)}

    tb = trsv_bytes(nnzL, gp.n_u)
    sb = spmv_bytes(nnz, n)
    r_f, r_b, r_s = roof("trsv_fwd", tb), roof("trsv_bwd", tb), roof("spmv", sb)
    dominant = max((r for r in (r_f, r_b, r_s) if r), key=lambda r: r["avg_launch_us"] * r["launches"])
    kernel_ms = {k: round(v[0], 3) for k, v in prof.items()}

    out = {
        "metric": METRIC, "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c1_2d_k2_n256", "N": N, "kprime": kp, "dim": dim, "nu": 1.0, "tol": tol,
                   "precond": "ic0+diagQ", "n_u": gp.n_u, "n_p": gp.n_p, "nnz": int(nnz), "nnz_L": int(nnzL),
                   "trsv_levels": [lev_f, lev_b], "forcing": "manufactured"},
        "iters": iters, "iters_per_s": round(iters / sec, 2),
        "relres_true_Minv": infos[-1]["relres_true_Minv"], "relres_true_2": infos[-1]["relres_true_2"],
        "setup_s": round(setup_s, 3),
        "roofline": dominant, "roofline_spmv": r_s,
        "kernel_ms_in_timed_region": kernel_ms,
    }

    if not args.no_extra:
        extra = {}
        try:
            gp.set_inner_tol(1e-2)
            s_pcg, inf_pcg = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_ICPCG)
            extra["c1_icpcg_inner1e-2"] = {"s": round(s_pcg, 5), "iters": inf_pcg[-1]["iters"],
                                           "inner_iters_total": inf_pcg[-1]["inner_iters_total"],
                                           "relres_true_Minv": inf_pcg[-1]["relres_true_Minv"]}
            log("icpcg", extra["c1_icpcg_inner1e-2"])
        except Exception as e:  # report, keep the headline
            extra["c1_icpcg_inner1e-2"] = {"error": str(e)}
        try:
            # the PCG(A), Diag(Q) variant: Jacobi-preconditioned inner CG on A
            s_j, inf_j = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_JPCG)
            extra["c1_jpcg_inner1e-2"] = {"s": round(s_j, 5), "iters": inf_j[-1]["iters"],
                                          "inner_iters_total": inf_j[-1]["inner_iters_total"],
                                          "relres_true_Minv": inf_j[-1]["relres_true_Minv"]}
            log("jpcg", extra["c1_jpcg_inner1e-2"])
        except Exception as e:  # report, keep the headline
            extra["c1_jpcg_inner1e-2"] = {"error": str(e)}
        try:
            # PCG(A,Q): Jacobi-preconditioned inner CG on both blocks
            s_q, inf_q = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_PCGAQ)
            extra["c1_pcgAQ_inner1e-2"] = {"s": round(s_q, 5), "iters": inf_q[-1]["iters"],
                                           "inner_iters_total": inf_q[-1]["inner_iters_total"],
                                           "relres_true_Minv": inf_q[-1]["relres_true_Minv"]}
            log("pcgAQ", extra["c1_pcgAQ_inner1e-2"])
        except Exception as e:  # report, keep the headline
            extra["c1_pcgAQ_inner1e-2"] = {"error": str(e)}
        try:
            # Ideal(A,Q): both blocks solved by inner CG to the fixed relative residual 1e-12
            s_i, inf_i = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_IDEAL)
            extra["c1_ideal"] = {"s": round(s_i, 5), "iters": inf_i[-1]["iters"],
                                 "inner_iters_total": inf_i[-1]["inner_iters_total"],
                                 "relres_true_Minv": inf_i[-1]["relres_true_Minv"]}
            log("ideal", extra["c1_ideal"])
        except Exception as e:  # report, keep the headline
            extra["c1_ideal"] = {"error": str(e)}
        try:
            # Ideal(A) + Diag(Q): the velocity block as in Ideal(A,Q), Diag(Q) on the pressure
            s_ia, inf_ia = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_IDEAL_A)
            extra["c1_ideal_A_diagQ"] = {"s": round(s_ia, 5), "iters": inf_ia[-1]["iters"],
                                         "inner_iters_total": inf_ia[-1]["inner_iters_total"],
                                         "relres_true_Minv": inf_ia[-1]["relres_true_Minv"]}
            log("ideal_A_diagQ", extra["c1_ideal_A_diagQ"])
        except Exception as e:  # report, keep the headline
            extra["c1_ideal_A_diagQ"] = {"error": str(e)}
        try:
            # the lid-driven cavity on the C1 mesh: load through the Nitsche form l_h
            fc = gp.load_cavity(CAVITY_LID)
            s_c0, inf_c0 = timed_solves(gp, fc, 1, 1, tol=tol, precond=PC_IC0)
            s_cq, inf_cq = timed_solves(gp, fc, 1, 1, tol=tol, precond=PC_PCGAQ)
            extra["c1_cavity"] = {"ic0_s": round(s_c0, 5), "ic0_iters": inf_c0[-1]["iters"],
                                  "pcgAQ_s": round(s_cq, 5), "pcgAQ_iters": inf_cq[-1]["iters"],
                                  "pcgAQ_inner_iters_total": inf_cq[-1]["inner_iters_total"]}
            log("cavity", extra["c1_cavity"])
        except Exception as e:  # report, keep the headline
            extra["c1_cavity"] = {"error": str(e)}
        del gp
        torch.cuda.empty_cache()
        try:
            g2 = StokesProblem(512, 2, 2, 1.0)
            f2 = g2.load(True)[0]
            s64, i64 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_IC0, precision=FP64)
            log("c2 fp64 %.3f s, %d iterations" % (s64, i64[-1]["iters"]))
            s32, i32 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_IC0, precision=MIXED)
            log("c2 mixed %.3f s, %d iterations, %d refinement cycles" % (s32, i32[-1]["iters"],
                                                                        i32[-1]["refine_cycles"]))
            u64, p64, _ = g2.solve(f2, tol=1e-13)
            um, pm, _ = g2.solve(f2, tol=tol, precision=MIXED)
            eu = float((um - u64).norm() / u64.norm())
            ep = float((pm - p64).norm() / p64.norm())
            extra["c2_n512_mixed_vs_fp64"] = {"fp64_s": round(s64, 5), "fp64_iters": i64[-1]["iters"],
                                              "mixed_s": round(s32, 5), "mixed_iters": i32[-1]["iters"],
                                              "speedup": round(s64 / s32, 3), "mixed_rel_err_u": eu,
                                              "mixed_rel_err_p": ep,
                                              "mixed_relres_true_Minv": i32[-1]["relres_true_Minv"]}
            log("c2", extra["c2_n512_mixed_vs_fp64"])
            # PCG(A,Q) at N = 512: the inner Diag-CG products are bandwidth-bound, so the mixed
            # mode (FP32 inner MINRES and inner CG) pays there
            g2.set_inner_tol(1e-2)
            q64, j64 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_PCGAQ, precision=FP64)
            q32, j32 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_PCGAQ, precision=MIXED)
            extra["c2_n512_pcgAQ_mixed_vs_fp64"] = {
                "fp64_s": round(q64, 5), "fp64_iters": j64[-1]["iters"], "mixed_s": round(q32, 5),
                "mixed_iters": j32[-1]["iters"], "mixed_refine_cycles": j32[-1]["refine_cycles"],
                "speedup": round(q64 / q32, 3), "mixed_relres_true_Minv": j32[-1]["relres_true_Minv"]}
            log("c2 pcgAQ", extra["c2_n512_pcgAQ_mixed_vs_fp64"])
            del g2
            torch.cuda.empty_cache()
        except Exception as e:
            extra["c2_n512_mixed_vs_fp64"] = {"error": str(e)}
        try:
            from synthetic_inputs import forcing_modes, WORKLOADS
            w3 = WORKLOADS["c3_3d_k1_n32_r16"]
            g3 = StokesProblem(w3["N"], w3["kp"], w3["dim"], 1.0)
            F3 = g3.load(True, forcing_modes(w3["seeds"], 3))
            g3.solve_batched(F3, tol=tol)
            sync()
            log("c3 warm-up done")
            t = time.perf_counter()
            U3, P3, inf3 = g3.solve_batched(F3, tol=tol)
            sync()
            sb3 = time.perf_counter() - t
            t = time.perf_counter()
            for r in range(F3.shape[0]):
                g3.solve(F3[r].contiguous(), tol=tol)
            sync()
            ss3 = time.perf_counter() - t
            extra["c3_3d_n32_16rhs"] = {"batched_s": round(sb3, 5), "sequential_s": round(ss3, 5),
                                        "speedup": round(ss3 / sb3, 3),
                                        "iters": [i["iters"] for i in inf3]}
            log("c3", extra["c3_3d_n32_16rhs"])
            del g3
            torch.cuda.empty_cache()
        except Exception as e:
            extra["c3_3d_n32_16rhs"] = {"error": str(e)}
        try:
            from synthetic_inputs import forcing_modes, target_perturbations, WORKLOADS
            from paper_1309_5048_amd import stokes_solve
            w4 = WORKLOADS["c4_2d_k2_n256_r8"]
            g4 = StokesProblem(w4["N"], w4["kp"], 2, 1.0)
            F4 = g4.load(True, forcing_modes(w4["seeds"], 2))
            ut = (g4.solve_batched(g4.load(True).repeat(8, 1).contiguous(), tol=tol)[0]
                  + 1e-2 * torch.as_tensor(target_perturbations(g4.n_u, 8), device="cuda"))
            nu = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
            Fv = F4.clone().requires_grad_(True)
            sync()
            t = time.perf_counter()
            U4, P4 = stokes_solve(Fv, nu, g4, tol)
            sync()
            tf = time.perf_counter() - t
            log("c4 forward %.3f s" % tf)
            loss = 0.5 * ((U4 - ut) ** 2).sum()
            t = time.perf_counter()
            loss.backward()
            sync()
            tb4 = time.perf_counter() - t
            extra["c4_adjoint_8rhs"] = {"forward_s": round(tf, 5), "backward_s": round(tb4, 5),
                                        "ratio_fwd_plus_bwd_over_2fwd": round((tf + tb4) / (2 * tf), 3),
                                        "dloss_dnu": float(nu.grad)}
            log("c4", extra["c4_adjoint_8rhs"])
            del g4
        except Exception as e:
            extra["c4_adjoint_8rhs"] = {"error": str(e)}
        out["variants"] = extra

    if args.copy_probe > 0:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        sync()
        out["copy_probe_bytes"] = nbytes
        log("copy probe: 3 x %d bytes read and written" % nbytes)
    if not args.no_cpu:
        log("cpu baseline (oracle, 1 core)")
        out["cpu_baseline"] = cpu_baseline(N, kp, dim, iters, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
