"""Throughput of the Fourier-basis FMM matvec on one MI355X.

Workload: N = 2^20 points uniform on the unit sphere (seed 0), kappa = 177, leaves of at most 64
points, complex64 charges N(0,1) (seed 1), FP32 path with eps = 1e-4. A step is one full matvec
(gather, P2M, M2M, M2L, L2L, L2P, P2P, scatter) with the inputs resident in HBM; plan creation
(octree, parameters, transfer tables) is setup and is reported separately. The line also carries
the adjoint and the FP64 path (eps = 1e-6), the per-stage times, the roofline of the dominant
stage, the error against the oracle's direct sum on a subset of targets, and that direct sum's
own throughput on the host cores (a reported baseline, not the target).
"""
import argparse
import json
import os
import sys
import time

import numpy as np


HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--kappa", type=float, default=177.0)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--targets", type=int, default=2048, help="direct-sum check targets")
    ap.add_argument("--depth", type=int, default=0,
                    help="leaf level (0: the plan's own choice from max_leaf and eps)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (PMC calibration)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2^23 ellipsoid points, kappa 500, eps 1e-3, 4 RHS run")
    ap.add_argument("--volume", action="store_true",
                    help="also run the volume workload: 2^12..2^22 points uniform in the unit cube, "
                         "kappa = 2 pi N^(1/3) / 2.52, FP32, eps 1e-4, automatic method and depth")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="run P2P in order on the calling stream (no overlap), so that a kernel "
                         "trace shows every kernel alone")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch configuration instead of the library's autotuner "
                         "(implied by --serial; counter and trace runs use it so that every "
                         "dispatch of a kernel has one configuration)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the autograd run (2^18 sphere points, kappa 88, loss sum |phi - phi_t|^2)")
    return ap.parse_args()


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def stage_work(info, stage):
    """Algorithmic work of one launch group of a stage (per right-hand side):
    returns (bound, amount, unit) with amount in GB or TFLOP."""
    L = info["depth"]
    n = info["n_points"]
    cs = 8 if info["precision"] == 1 else 16
    if stage in ("m2l", "leaf_m2l"):
        lv = [L] if stage == "leaf_m2l" else range(2, L + 1)
        flops = sum(8.0 * info["n_ilist"][l] * info["K"][l] for l in lv)
        return "alu", flops / 1e12, "TFLOP"
    if stage == "p2m":
        return "alu", 14.0 * n * info["K"][L] / 1e12, "TFLOP"
    if stage == "l2p":
        return "alu", 16.0 * n * info["K"][L] / 1e12, "TFLOP"
    if stage == "p2p":
        return "alu", 26.0 * info["n_near_pairs"] / 1e12, "TFLOP"
    if stage in ("m2m", "l2l"):
        byt = sum(cs * (info["n_boxes"][l] * info["K"][l] + info["n_boxes"][l - 1] * info["K"][l - 1])
                  for l in range(3, L + 1))
        return "hbm", byt / 1e9, "GB"
    if stage in ("gather", "scatter"):
        return "hbm", (2 * cs + 8) * n / 1e9, "GB"
    return "hbm", 0.0, "GB"


# HBM traffic of the dominant kernel: FETCH_SIZE and WRITE_SIZE per dispatch from rocprofv3 --pmc,
# scaled by the same counters on a plain device copy (profiles/, written by
# ``python -m paper_0911_4114_amd.profiling traffic``); reported only while the kernel's source file
# is the one the counters were taken on, else null.
TRAFFIC_FILES = {
    "p2p": ("profiles/traffic_p2p_fp32_sphere1M_k177.txt", "p2p_kernel<float, float2, false, true, 1>"),
    "m2l": ("profiles/traffic_m2l_fp32_sphere1M_k177.txt", "m2lp_kernel<float2*"),
}


def measured_traffic(stage, args):
    here = os.path.dirname(os.path.abspath(__file__))
    if stage not in TRAFFIC_FILES or args.n != 1 << 20 or args.kappa != 177.0 or args.eps != 1e-4:
        return None
    rel, kernel = TRAFFIC_FILES[stage]
    path = os.path.join(here, rel)
    if not os.path.exists(path):
        return None
    from paper_0911_4114_amd.profiling import file_sha256, read_traffic
    t = read_traffic(path)
    if t.get("kernel") != kernel or t.get("source_sha256") != file_sha256(os.path.join(here, t["source"])):
        return None
    return float(t["hbm_bytes_per_dispatch"])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))
        return
    import paper_0911_4114_amd as ff
    from paper_0911_4114_amd import workloads as wl

    dev = torch.device("cuda")
    n = args.n
    log("generating workload n=%d" % n)
    x = wl.sphere_points(n, seed=0)
    q = wl.complex_normal(n, seed=1)
    xt = torch.as_tensor(x, dtype=torch.float64, device=dev)
    q32 = torch.as_tensor(q, dtype=torch.complex128, device=dev).to(torch.complex64)

    log("plan fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = ff.Plan(xt, args.kappa, args.eps, precision="fp32", depth=args.depth or None)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tune_s = None
    if args.serial:
        plan.set_tuning(near_stream=0)
    elif not args.no_tune:
        # the library's autotuner picks the launch configuration on this workload (setup, not
        # timed, like plan creation)
        t0 = time.perf_counter()
        plan.autotune(q32)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
    info = plan.info()
    plan_tuning = plan.tuning()
    log("plan fp32 done in %.2fs depth=%d K=%s ell=%s" % (setup_s, info["depth"], info["K"][2:], info["ell"][2:]))

    ms = timed(lambda: plan.matvec(q32), args.steps, args.warmup)
    log("fp32 matvec %.3f ms" % ms)
    ms_adj = timed(lambda: plan.adjoint(q32), args.steps, args.warmup)
    log("fp32 adjoint %.3f ms" % ms_adj)

    # per-stage times (separate profiled pass: every stage alone on the calling stream, so P2P
    # gets the whole GPU instead of the share that the tuned configuration leaves it beside the
    # far field)
    plan.set_tuning(p2p_blocks_per_cu=0)
    plan.profile(True)
    prof_steps = max(3, min(args.steps, 10))
    for _ in range(prof_steps):
        plan.matvec(q32)
    prof = plan.profile_read()
    plan.profile(False)
    plan.set_tuning(**plan_tuning)
    stages = {k: {"ms_per_step": v[0] / prof_steps, "launches_per_step": v[1] / prof_steps}
              for k, v in prof.items()}
    cand = {k: v for k, v in stages.items() if k != "leaf_m2l"}
    m2l_total = stages["m2l"]["ms_per_step"] + stages["leaf_m2l"]["ms_per_step"]
    cand["m2l"] = {"ms_per_step": m2l_total,
                   "launches_per_step": stages["m2l"]["launches_per_step"] + stages["leaf_m2l"]["launches_per_step"]}
    dom = max(cand, key=lambda k: cand[k]["ms_per_step"])
    bound, amount, unit = stage_work(info, dom)
    nlaunch = max(cand[dom]["launches_per_step"], 1.0)
    per_launch_ms = cand[dom]["ms_per_step"] / nlaunch
    per_launch_amount = amount / nlaunch
    if bound == "hbm":
        achieved = per_launch_amount / (per_launch_ms * 1e-3)
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        achieved = per_launch_amount / (per_launch_ms * 1e-3)
        # P2P carries FP64 distance/phase arithmetic: priced against the FP64 vector peak (the
        # same lane rate as non-packed FP32); the other ALU stages against the FP32 vector peak
        peak = FP64_PEAK_TFLOPS if dom == "p2p" else FP32_PEAK_TFLOPS
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None}
    roof["stage"] = dom
    roof["launch_ms"] = per_launch_ms
    roof["traffic"] = measured_traffic(dom, args)

    # accuracy against the oracle's direct sum on a subset of targets (host FP64)
    out = plan.matvec(q32).cpu().numpy().astype(np.complex128)
    tg = wl.subset(n, args.targets, seed=7)
    cpu = None
    rel_err = None
    if not args.no_cpu:
        from oracle import direct
        cores = len(os.sched_getaffinity(0))
        log("direct sum on %d targets (%d host threads)" % (len(tg), cores))
        t1 = time.perf_counter()
        ref = direct.matvec(x, q, args.kappa, targets=tg)
        cpu_s = time.perf_counter() - t1
        rel_err = float(np.linalg.norm(out[tg] - ref) / np.linalg.norm(ref))
        cpu = {"value": len(tg) / cpu_s / 1e6, "unit": "Mpoints/s", "cores": cores,
               "kind": "oracle",
               "sample": "oracle direct sum (C/OpenMP FP64): %d of %d targets against all %d sources, %.1f s"
                         % (len(tg), n, n, cpu_s)}
        log("fp32 rel err %.3e; cpu %.4f Mpoints/s" % (rel_err, cpu["value"]))

    batched = None
    if not args.no_batched:
        # 16 incident plane waves q_j^(m) = e^{i kappa d_m . x_j} through one tree
        nb_rhs = 16
        qb = torch.as_tensor(wl.plane_wave_charges(x, args.kappa, nb_rhs, seed=2),
                             dtype=torch.complex128, device=dev).to(torch.complex64)
        pb = ff.Plan(xt, args.kappa, args.eps, precision="fp32", max_rhs=nb_rhs,
                     depth=args.depth or None)
        # the library's autotuner picks the launch configuration for 16 right-hand sides (setup)
        t0 = time.perf_counter()
        tuned = pb.autotune(qb)
        tune_s = time.perf_counter() - t0
        msb = timed(lambda: pb.matvec(qb), max(3, args.steps // 2), 1)
        batched = {"nrhs": nb_rhs, "value": n * nb_rhs / (msb * 1e-3) / 1e6, "ms_per_step": msb,
                   "tuning": tuned, "autotune_s": tune_s}
        if not args.no_cpu:
            ob = pb.matvec(qb)[3].cpu().numpy().astype(np.complex128)
            qh = wl.plane_wave_charges(x, args.kappa, nb_rhs, seed=2)[3]
            refb = direct.matvec(x, qh, args.kappa, targets=tg[:512])
            batched["rel_err_rhs3"] = float(np.linalg.norm(ob[tg[:512]] - refb) / np.linalg.norm(refb))
        log("batched %d rhs: %.3f ms (%.1f Mpoints/s)" % (nb_rhs, msb, batched["value"]))
        del pb
        torch.cuda.empty_cache()

    large = None
    if not args.no_large:
        nl = 1 << 23
        xl = wl.ellipsoid_points(nl, seed=0)
        ql = wl.complex_normal(nl, seed=1, nrhs=4)
        xlt = torch.as_tensor(xl, dtype=torch.float64, device=dev)
        qlt = torch.as_tensor(ql, dtype=torch.complex128, device=dev).to(torch.complex64)
        t0 = time.perf_counter()
        pl = ff.Plan(xlt, 500.0, 1e-3, precision="fp32", max_rhs=4)
        torch.cuda.synchronize()
        sl = time.perf_counter() - t0
        msl = timed(lambda: pl.matvec(qlt), 3, 1)
        il = pl.info()
        large = {"n": nl, "nrhs": 4, "value": nl * 4 / (msl * 1e-3) / 1e6, "ms_per_step": msl,
                 "setup_s": sl, "depth": il["depth"]}
        if not args.no_cpu:
            tl = wl.subset(nl, 256, seed=7)
            ol = pl.matvec(qlt)[0].cpu().numpy().astype(np.complex128)
            refl = direct.matvec(xl, ql[0], 500.0, targets=tl)
            large["rel_err"] = float(np.linalg.norm(ol[tl] - refl) / np.linalg.norm(refl))
        log("large: %s" % large)
        del pl
        torch.cuda.empty_cache()

    volume = None
    if args.volume:
        # O(N) at constant points per wavelength with the time-optimal level count, and the
        # FMM/direct crossover (the volume workload of the paper's running-time study)
        volume = []
        for e in (12, 14, 16, 18, 20, 22):
            nv = 1 << e
            kv = 2.0 * np.pi * nv ** (1.0 / 3.0) / 2.52
            xv = wl.cube_points(nv, seed=0)
            qv = wl.complex_normal(nv, seed=1)
            xvt = torch.as_tensor(xv, dtype=torch.float64, device=dev)
            qvt = torch.as_tensor(qv, dtype=torch.complex128, device=dev).to(torch.complex64)
            t0 = time.perf_counter()
            pv = ff.Plan(xvt, kv, 1e-4, precision="fp32", method="auto")
            torch.cuda.synchronize()
            sv = time.perf_counter() - t0
            iv = pv.info()
            msv = timed(lambda: pv.matvec(qvt), 5, 1)
            ent = {"n": nv, "kappa": kv, "method": iv["method"], "depth": iv["depth"], "ms": msv,
                   "value": nv / (msv * 1e-3) / 1e6, "setup_s": sv}
            if nv <= 1 << 18:
                pd = ff.Plan(xvt, kv, 1e-4, precision="fp32", method="direct")
                ent["direct_ms"] = timed(lambda: pd.matvec(qvt), 3, 1)
                del pd
            if not args.no_cpu:
                tv = wl.subset(nv, min(nv, 256), seed=7)
                ov = pv.matvec(qvt).cpu().numpy().astype(np.complex128)[tv]
                rv = direct.matvec(xv, qv, kv, targets=tv)
                ent["rel_err"] = float(np.linalg.norm(ov - rv) / np.linalg.norm(rv))
            log("volume: %s" % ent)
            volume.append(ent)
            del pv
            torch.cuda.empty_cache()

    grad = None
    if not args.no_grad:
        # forward + backward of loss = sum |phi - phi_t|^2 through the differentiable matvec;
        # backward = one adjoint matvec plus one two-RHS field-gradient call
        ng, kg = 1 << 18, 88.0
        xg = wl.sphere_points(ng, seed=0)
        qg = wl.complex_normal(ng, seed=1)
        phit = wl.complex_normal(ng, seed=3)
        xgt = torch.as_tensor(xg, dtype=torch.float64, device=dev)
        qgt = torch.as_tensor(qg, dtype=torch.complex128, device=dev).to(torch.complex64).requires_grad_(True)
        xgr = xgt.clone().requires_grad_(True)
        ptt = torch.as_tensor(phit, dtype=torch.complex128, device=dev).to(torch.complex64)
        pg = ff.Plan(xgt, kg, args.eps, precision="fp32", max_rhs=2)

        def fwd_bwd():
            xgr.grad = None
            qgt.grad = None
            phi = ff.apply(pg, xgr, qgt)
            (phi - ptt).abs().pow(2).sum().backward()

        msg = timed(fwd_bwd, max(3, args.steps // 2), 1)
        msf = timed(lambda: pg.matvec(qgt.detach()), max(3, args.steps // 2), 1)
        grad = {"n": ng, "kappa": kg, "ms_fwd_bwd": msg, "ms_matvec": msf,
                "value": ng / (msg * 1e-3) / 1e6, "depth": pg.info()["depth"]}
        if not args.no_cpu:
            # the backward's parts against the oracle on 256 targets: the forward phi, the adjoint
            # of a seeded vector g, and the field gradient of q (the full gradient needs phi at
            # every point; the GPU tests check it at small N)
            tgg = wl.subset(ng, 256, seed=7)
            gv = wl.complex_normal(ng, seed=4)
            gvt = torch.as_tensor(gv, dtype=torch.complex128, device=dev).to(torch.complex64)
            qd = qgt.detach()
            phig = pg.matvec(qd).cpu().numpy()[tgg]
            adj = pg.adjoint(gvt).cpu().numpy()[tgg]
            fld = pg.field_gradient(qd).cpu().numpy()[tgg]
            r_phi = direct.matvec(xg, qg, kg, targets=tgg)
            r_adj = np.conj(direct.matvec(xg, np.conj(gv), kg, targets=tgg))
            r_fld = direct.gradient(xg, qg, kg, targets=tgg)
            rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            grad["rel_err_phi"] = rel(phig, r_phi)
            grad["rel_err_adjoint"] = rel(adj, r_adj)
            grad["rel_err_field_gradient"] = rel(fld, r_fld)
        log("autograd: %s" % grad)
        del pg
        torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        del plan
        torch.cuda.empty_cache()
        log("plan fp64")
        q64 = torch.as_tensor(q, dtype=torch.complex128, device=dev)
        t0 = time.perf_counter()
        p64 = ff.Plan(xt, args.kappa, 1e-6, precision="fp64")
        torch.cuda.synchronize()
        s64 = time.perf_counter() - t0
        ms64 = timed(lambda: p64.matvec(q64), max(3, args.steps // 2), 2)
        out64 = p64.matvec(q64).cpu().numpy()
        i64 = p64.info()
        fp64 = {"value": n / (ms64 * 1e-3) / 1e6, "ms_per_step": ms64, "setup_s": s64,
                "depth": i64["depth"], "eps": 1e-6}
        if not args.no_cpu:
            fp64["rel_err"] = float(np.linalg.norm(out64[tg] - ref) / np.linalg.norm(ref))
        log("fp64 %.3f ms err %s" % (ms64, fp64.get("rel_err")))

    line = {
        "metric": "FMM matvec Mpoints/s at rel err 1e-4 (FP32) vs 1e-6 (FP64); fwd+adjoint",
        "value": n / (ms * 1e-3) / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere N=%d kappa=%g leaf<=64 FP32 eps=%g nrhs=1" % (n, args.kappa, args.eps),
                   "n": n, "kappa": args.kappa, "eps": args.eps, "nrhs": 1,
                   "depth": info["depth"], "ell": info["ell"][2:], "K": info["K"][2:],
                   "boxes": info["n_boxes"][2:], "ilist": info["n_ilist"][2:],
                   "near_pairs": info["n_near_pairs"]},
        "rel_err": rel_err,
        "adjoint": {"value": n / (ms_adj * 1e-3) / 1e6, "ms_per_step": ms_adj},
        "setup_s": setup_s,
        "tuning": plan_tuning,
        "autotune_s": tune_s,
        "stages_ms": {k: round(v["ms_per_step"], 4) for k, v in stages.items()},
        "fp64": fp64,
        "batched": batched,
        "large": large,
        "autograd": grad,
        "volume": volume,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
