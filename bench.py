"""Benchmark: time-to-solution of block-diagonally preconditioned MINRES for the
divergence-conforming B-spline Stokes system on one MI355X.

Headline workload (one "step" = one complete solve from the assembled load vector to the
zero-mean (u, p), inputs resident in HBM): 2D unit square, N = 256 elements per
direction, pressure degree k' = 2 (velocity degree 3), nu = 1, manufactured forcing,
FP64, M = blkdiag(IC(0) of A, Diag(Q)/(2 nu)), relative M^{-1}-norm residual 1e-8.

Printed: one JSON line with the headline value (seconds per solve, timed with nothing but
the solves on the stream), MINRES iterations/s, a roofline object for the dominant kernel
(algorithmic bytes per launch over its average launch time, measured with HIP events on the
solver's stream in a second, profiled pass of the same solves), the same for the saddle
SpMV, the CPU oracle timed on one host core for one whole solve, and the variant
comparisons (the inner-CG preconditioners, IC(0)-PCG(A,Q), the cavity, mixed precision at
N = 512, batched 3D, adjoint).  --only runs one workload alone, for profiling.
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


def host_cpu():
    """Host threads available and the CPU model name (from /proc/cpuinfo, as lscpu shows it)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(N, kp, dim, tol):
    """Oracle (plain single-threaded C++, FP64) on one host core: setup and IC(0) untimed,
    then one whole MINRES-IC(0) solve of the same system to the same tolerance, timed with
    the host clock around the solve only."""
    from oracle.oracle import Oracle
    t = time.perf_counter()
    o = Oracle(N, kp, dim, 1.0)
    o.ic0()
    f = o.load(1)
    t_setup = time.perf_counter() - t
    t0 = time.perf_counter()
    _, _, info = o.solve(f, tol=tol)
    dt = time.perf_counter() - t0
    nproc, model = host_cpu()
    return {"value": round(dt, 4), "unit": "s", "cores": 1, "kind": "oracle",
            "iters": info["iters"], "iters_per_s": round(info["iters"] / dt, 2),
            "host_nproc": nproc, "host_cpu": model,
            "sample": "one whole MINRES-IC(0) solve of the N=%d k'=%d dim=%d system to tol %g (%d iterations; "
                      "setup %.1f s untimed), single thread" % (N, kp, dim, tol, info["iters"], t_setup)}


def info_summary(inf):
    keys = ("iters", "inner_iters_total", "refine_cycles", "relres_true_Minv", "relres_true_2", "status")
    return {k: inf[k] for k in keys}


def variant(extra, name, fn):
    """Run one comparison; an error is reported in its entry and the benchmark goes on."""
    try:
        extra[name] = fn()
        log(name, extra[name])
    except Exception as e:  # report, keep the headline
        extra[name] = {"error": str(e)}
        log(name, "error", e)


def c1_variants(gp, f, tol, extra):
    from paper_1309_5048_amd import (CAVITY_LID, PC_IC0, PC_ICPCG, PC_ICPCG_AQ, PC_IDEAL, PC_IDEAL_A, PC_JPCG,
                                     PC_PCGAQ)
    gp.set_inner_tol(1e-2)
    inner = {"icpcg": PC_ICPCG, "jpcg": PC_JPCG, "pcgAQ": PC_PCGAQ, "icpcgAQ": PC_ICPCG_AQ}
    for name, pc in inner.items():
        # the paper's outer method (one MINRES run with the inner PCG, Sec. 5.1)
        def run(pc=pc):
            sec, infos = timed_solves(gp, f, 1, 1, tol=tol, precond=pc)
            return dict(s=round(sec, 5), **info_summary(infos[-1]))
        variant(extra, "c1_%s_inner1e-2" % name, run)
    for name in ("pcgAQ", "icpcgAQ"):
        # MINRES restarted on the true residual until the fixed-block norm meets tol
        def run_r(pc=inner[name]):
            gp.set_restarts(6)
            try:
                sec, infos = timed_solves(gp, f, 1, 1, tol=tol, precond=pc)
            finally:
                gp.set_restarts(0)
            return dict(s=round(sec, 5), **info_summary(infos[-1]))
        variant(extra, "c1_%s_inner1e-2_restarted" % name, run_r)

    def run_paper_tol():
        # IC(0)-PCG(A,Q) at the paper's tighter inner tolerance 1e-3 (Sec. 6.4 tables)
        gp.set_inner_tol(1e-3)
        try:
            sec, infos = timed_solves(gp, f, 1, 1, tol=tol, precond=PC_ICPCG_AQ)
        finally:
            gp.set_inner_tol(1e-2)
        return dict(s=round(sec, 5), **info_summary(infos[-1]))
    variant(extra, "c1_icpcgAQ_inner1e-3", run_paper_tol)
    for name, pc in (("ideal", PC_IDEAL), ("ideal_A_diagQ", PC_IDEAL_A)):
        def run_i(pc=pc):
            sec, infos = timed_solves(gp, f, 1, 1, tol=tol, precond=pc)
            return dict(s=round(sec, 5), **info_summary(infos[-1]))
        variant(extra, "c1_" + name, run_i)

    def run_cavity():
        # the lid-driven cavity on the C1 mesh: load through the Nitsche form l_h
        fc = gp.load_cavity(CAVITY_LID)
        out = {}
        for name, pc in (("ic0", PC_IC0), ("pcgAQ", PC_PCGAQ), ("icpcgAQ", PC_ICPCG_AQ)):
            sec, infos = timed_solves(gp, fc, 1, 1, tol=tol, precond=pc)
            out[name] = dict(s=round(sec, 5), **info_summary(infos[-1]))
        return out
    variant(extra, "c1_cavity", run_cavity)


def c2_variants(tol, extra, only=None):
    import torch
    from paper_1309_5048_amd import FP64, MIXED, PC_IC0, PC_PCGAQ, StokesProblem
    g2 = StokesProblem(512, 2, 2, 1.0)
    f2 = g2.load(True)[0]
    try:
        if only in ("c2-fp64", "c2-mixed"):
            prec = FP64 if only == "c2-fp64" else MIXED
            sec, infos = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_IC0, precision=prec)
            extra[only] = dict(s=round(sec, 5), **info_summary(infos[-1]))
            return

        def run_ic0():
            s64, i64 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_IC0, precision=FP64)
            s32, i32 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_IC0, precision=MIXED)
            # errors against the FP64 solve at tol 1e-13, for both solves at the bench tolerance
            uref, pref, _ = g2.solve(f2, tol=1e-13)
            u64, p64, _ = g2.solve(f2, tol=tol)
            um, pm, _ = g2.solve(f2, tol=tol, precision=MIXED)

            def err(a, b):
                return float((a - b).norm() / b.norm())
            return {"fp64_s": round(s64, 5), "fp64_iters": i64[-1]["iters"],
                    "mixed_s": round(s32, 5), "mixed_iters": i32[-1]["iters"],
                    "mixed_refine_cycles": i32[-1]["refine_cycles"], "speedup": round(s64 / s32, 3),
                    "fp64_rel_err_u": err(u64, uref), "fp64_rel_err_p": err(p64, pref),
                    "mixed_rel_err_u": err(um, uref), "mixed_rel_err_p": err(pm, pref),
                    "fp64_relres_true_Minv": i64[-1]["relres_true_Minv"],
                    "mixed_relres_true_Minv": i32[-1]["relres_true_Minv"],
                    "reference": "FP64 GPU solve at tol 1e-13"}
        variant(extra, "c2_n512_mixed_vs_fp64", run_ic0)

        def run_pcg():
            # PCG(A,Q) at N = 512: the inner Diag-CG products are bandwidth-bound, so the mixed
            # mode (FP32 inner MINRES and inner CG) pays there
            g2.set_inner_tol(1e-2)
            g2.set_restarts(6)
            q64, j64 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_PCGAQ, precision=FP64)
            q32, j32 = timed_solves(g2, f2, 1, 1, tol=tol, precond=PC_PCGAQ, precision=MIXED)
            g2.set_restarts(0)
            return {"fp64_s": round(q64, 5), "fp64_iters": j64[-1]["iters"], "mixed_s": round(q32, 5),
                    "mixed_iters": j32[-1]["iters"], "mixed_refine_cycles": j32[-1]["refine_cycles"],
                    "speedup": round(q64 / q32, 3), "fp64_relres_true_Minv": j64[-1]["relres_true_Minv"],
                    "mixed_relres_true_Minv": j32[-1]["relres_true_Minv"]}
        variant(extra, "c2_n512_pcgAQ_restarted_mixed_vs_fp64", run_pcg)
    finally:
        g2.close()
        torch.cuda.empty_cache()


def c3_variant(tol, extra, only=None):
    import torch
    from paper_1309_5048_amd import StokesProblem
    from synthetic_inputs import forcing_modes, WORKLOADS
    w3 = WORKLOADS["c3_3d_k1_n32_r16"]
    g3 = StokesProblem(w3["N"], w3["kp"], w3["dim"], 1.0)
    try:
        F3 = g3.load(True, forcing_modes(w3["seeds"], 3))
        g3.solve_batched(F3, tol=tol)
        sync()
        t = time.perf_counter()
        U3, P3, inf3 = g3.solve_batched(F3, tol=tol)
        sync()
        sb3 = time.perf_counter() - t
        if only == "c3":
            extra["c3"] = {"batched_s": round(sb3, 5), "iters": [i["iters"] for i in inf3]}
            return
        t = time.perf_counter()
        for r in range(F3.shape[0]):
            g3.solve(F3[r].contiguous(), tol=tol)
        sync()
        ss3 = time.perf_counter() - t
        extra["c3_3d_n32_16rhs"] = {"batched_s": round(sb3, 5), "sequential_s": round(ss3, 5),
                                    "speedup": round(ss3 / sb3, 3), "iters": [i["iters"] for i in inf3]}
        log("c3", extra["c3_3d_n32_16rhs"])
    finally:
        g3.close()
        torch.cuda.empty_cache()


def c4_variant(tol, extra):
    import torch
    from synthetic_inputs import forcing_modes, target_perturbations, WORKLOADS
    from paper_1309_5048_amd import StokesProblem, stokes_solve
    w4 = WORKLOADS["c4_2d_k2_n256_r8"]
    g4 = StokesProblem(w4["N"], w4["kp"], 2, 1.0)
    try:
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
    finally:
        g4.close()
        torch.cuda.empty_cache()


def copy_probe(mib, out):
    """A plain elementwise copy of mib MiB, three times (the reference for scaling memory
    counters)."""
    if mib <= 0:
        return
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    sync()
    out["copy_probe_bytes"] = nbytes
    log("copy probe: 3 x %d bytes read and written" % nbytes)


ONLY = ("c1-ic0", "c1-pcgAQ", "c1-jpcg", "c1-icpcg", "c1-icpcgAQ", "c1-ideal", "c2-fp64", "c2-mixed", "c3", "c4")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extra", action="store_true", help="skip the variant comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default=None, choices=ONLY,
                    help="run one workload alone (for profiling): the C1 solve with one preconditioner "
                         "(inner tolerance 1e-2), the N = 512 solve in FP64 or mixed precision, the 3D "
                         "batched solve of 16 right-hand sides, or the forward and adjoint solves of 8")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the solves, run a plain elementwise copy of MIB MiB three times "
                         "(reads and writes MIB MiB each): the reference for scaling memory counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this solver path is built and measured on a single "
              "MI355X (no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_5048_amd import (StokesProblem, PC_IC0, PC_ICPCG, PC_ICPCG_AQ, PC_IDEAL, PC_JPCG,
                                     PC_PCGAQ)

    torch.cuda.set_device(0)
    N, kp, dim, tol = 256, 2, 2, 1e-8
    if args.only == "c1-ic0":  # the headline solves alone
        args.no_extra = args.no_cpu = True
    if args.only and not args.only.startswith("c1-"):
        extra = {}
        log("workload %s alone" % args.only)
        if args.only.startswith("c2"):
            c2_variants(tol, extra, args.only)
        elif args.only == "c3":
            c3_variant(tol, extra, "c3")
        else:
            c4_variant(tol, extra)
        out = {"only": args.only, "results": extra}
        copy_probe(args.copy_probe, out)
        print(json.dumps(out), flush=True)
        return

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

    if args.only and args.only != "c1-ic0":
        name = args.only[3:]
        pc = {"pcgAQ": PC_PCGAQ, "jpcg": PC_JPCG, "icpcg": PC_ICPCG, "icpcgAQ": PC_ICPCG_AQ,
              "ideal": PC_IDEAL}[name]
        gp.set_inner_tol(1e-2)
        sec, infos = timed_solves(gp, f, args.steps, args.warmup, tol=tol, precond=pc)
        log("solve %.4f s, %d iterations, %d inner, relres %.2e" % (
            sec, infos[-1]["iters"], infos[-1]["inner_iters_total"], infos[-1]["relres_true_Minv"]))
        print(json.dumps({"only": args.only, "s": round(sec, 6), **info_summary(infos[-1])}), flush=True)
        gp.close()
        return

    # warm-up, then the timed solves with nothing else on the stream
    for _ in range(args.warmup):
        gp.solve(f, tol=tol, precond=PC_IC0)
    sync()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        u, p, info = gp.solve(f, tol=tol, precond=PC_IC0)
        infos.append(info)
    sync()
    sec = (time.perf_counter() - t0) / args.steps
    iters = infos[-1]["iters"]
    log("solve %.4f s, %d iterations, relres %.2e" % (sec, iters, infos[-1]["relres_true_Minv"]))
    # the same solves again with HIP events recorded on the solver's stream around every
    # launch of the MINRES loop: per-kernel durations for the roofline
    psteps = max(2, args.steps // 4)
    gp.profile(1)
    t0 = time.perf_counter()
    for _ in range(psteps):
        gp.solve(f, tol=tol, precond=PC_IC0)
    sync()
    sec_prof = (time.perf_counter() - t0) / psteps
    prof = gp.profile(0)
    log("profiled pass %.4f s per solve" % sec_prof)

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
    kernel_ms = {k: round(v[0] / psteps, 3) for k, v in prof.items()}

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
        "profiled_pass": {"solves": psteps, "s_per_solve": round(sec_prof, 6),
                          "kernel_ms_per_solve": kernel_ms},
    }

    if not args.no_extra:
        extra = {}
        c1_variants(gp, f, tol, extra)
        gp.close()
        del gp
        torch.cuda.empty_cache()
        c2_variants(tol, extra)
        try:
            c3_variant(tol, extra)
        except Exception as e:
            extra["c3_3d_n32_16rhs"] = {"error": str(e)}
        try:
            c4_variant(tol, extra)
        except Exception as e:
            extra["c4_adjoint_8rhs"] = {"error": str(e)}
        out["variants"] = extra
    else:
        gp.close()

    copy_probe(args.copy_probe, out)
    if not args.no_cpu:
        log("cpu baseline (oracle, 1 core, one whole solve)")
        out["cpu_baseline"] = cpu_baseline(N, kp, dim, tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
