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
    ap.add_argument("--no-fast", action="store_true",
                    help="skip the run with the opt-in FP32 near-field distance and phase")
    ap.add_argument("--no-cube", action="store_true",
                    help="skip the 4096-point cube (kappa 8 pi, depth 3, FP64, eps 1e-6)")
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


class omp_threads:
    """Limit the OpenMP threads of the oracle's C sums (libgomp) inside a with block."""

    def __init__(self, n):
        import ctypes
        self.n = n
        self.gomp = ctypes.CDLL("libgomp.so.1")
        self.old = None

    def __enter__(self):
        self.old = self.gomp.omp_get_max_threads()
        self.gomp.omp_set_num_threads(self.n)

    def __exit__(self, *exc):
        self.gomp.omp_set_num_threads(self.old)


def oracle_ffmm_timing(eps):
    """Seconds per matvec of the oracle's CPU Fourier-basis FMM (FP64, NumPy) on 2^16 points on
    the unit sphere at kappa = 177 (2^16 / 2^20)^(1/2) (the benchmark's points per wavelength),
    with every host core available to its libraries and with one."""
    from threadpoolctl import threadpool_limits
    from oracle.ffmm import Plan as OPlan
    from paper_0911_4114_amd import workloads as wl
    n = 1 << 16
    kappa = 177.0 * (n / 2.0 ** 20) ** 0.5
    x = wl.sphere_points(n, seed=0)
    q = wl.complex_normal(n, seed=1)
    t0 = time.perf_counter()
    op = OPlan(x, kappa, eps)
    for l in range(2, op.depth + 1):
        op.table(l)
    setup = time.perf_counter() - t0
    res = {"n": n, "kappa": kappa, "eps": eps, "depth": op.depth, "setup_s": setup,
           "unit": "Mpoints/s", "kind": "oracle FMM"}
    for key, lim in (("all_cores", None), ("one_core", 1)):
        with threadpool_limits(lim):
            t0 = time.perf_counter()
            op.matvec(q)
            dt = time.perf_counter() - t0
        res[key] = {"matvec_s": dt, "value": n / dt / 1e6,
                    "cores": len(os.sched_getaffinity(0)) if lim is None else 1}
    return res


def workload_label(n, kappa, eps, info):
    L = info["depth"]
    return ("sphere N=%d kappa=%g FP32 eps=%g nrhs=1, depth %d (leaves of up to %d points: the "
            "leaf level of depth %d, where every leaf holds <= 64, is in the low-frequency "
            "breakdown for eps in FP32)" % (n, kappa, eps, L, info.get("max_leaf_points", 0), L + 1))


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


# Peaks (MI355X published figures): FP32 vector (packed) and FP64 vector FLOP/s, the FP32
# transcendental rate (sine, cosine, reciprocal square root issue at a quarter of the lane rate:
# 256 CUs x 16 lanes x 2.4 GHz) and HBM bandwidth.
TRANS_PEAK_TPS = 256 * 16 * 2.4e9 / 1e12


def stage_work(info, stage):
    """Algorithmic work of one stage per right-hand side: dict with FLOPs, transcendental
    evaluations and HBM bytes, and the FLOP peak that applies (TFLOP/s)."""
    L = info["depth"]
    n = info["n_points"]
    cs = 8 if info["precision"] == 1 else 16
    rs = cs // 2
    K, nb = info["K"], info["n_boxes"]
    kp = K[L] // 2
    fpk = FP32_PEAK_TFLOPS if info["precision"] == 1 else FP64_PEAK_TFLOPS
    w = {"flops": 0.0, "trans": 0.0, "bytes": 0.0, "peak": fpk}
    if stage in ("m2l", "leaf_m2l"):
        lv = [L] if stage == "leaf_m2l" else range(2, L + 1)
        w["flops"] = sum(8.0 * info["n_ilist"][l] * K[l] for l in lv)
        w["bytes"] = sum(cs * (2.0 * nb[l] * K[l] + 34.0 * K[l]) for l in lv)
    elif stage in ("p2m", "l2p"):
        # per (point, antipodal direction pair): phase 3 FMA, one sine and one cosine, 4 FMA
        w["flops"] = 14.0 * n * kp
        w["trans"] = 2.0 * n * kp
        w["bytes"] = n * (3 * rs + 2 * cs) + cs * nb[L] * K[L]
    elif stage == "p2p":
        # per ordered pair: FP64 differences (3), R^2 (5), the Newton step for R (6) and the phase
        # (1); FP32 e^{i kR}/R (2) and the complex MAC (8); reciprocal square root, sine and cosine
        w["flops"] = 25.0 * info["n_near_pairs"]
        w["trans"] = 3.0 * info["n_near_pairs"]
        w["bytes"] = n * (24 + 2 * cs)
        w["peak"] = FP64_PEAK_TFLOPS
    elif stage == "m2m":
        w["bytes"] = sum(cs * (nb[l] * K[l] + nb[l - 1] * K[l - 1]) for l in range(3, L + 1))
    elif stage == "l2l":
        w["bytes"] = sum(cs * (nb[l] * K[l] + 2.0 * nb[l + 1] * K[l + 1]) for l in range(2, L))
    elif stage == "gather":
        w["bytes"] = (2 * cs + 8) * n
    elif stage == "scatter":
        w["bytes"] = (3 * cs + 8) * n
    return w


def stage_roofline(info, stage, ms):
    """Roofline time of a stage (the largest of FLOPs / peak, transcendentals / rate and bytes /
    HBM bandwidth), its bound and the achieved rates against the peaks."""
    w = stage_work(info, stage)
    t = {"alu": w["flops"] / (w["peak"] * 1e12), "trans": w["trans"] / (TRANS_PEAK_TPS * 1e12),
         "hbm": w["bytes"] / (HBM_PEAK_GBS * 1e9)}
    bound = max(t, key=t.get)
    s = ms * 1e-3
    return {"ms": round(ms, 4), "bound": bound, "roofline_ms": round(t[bound] * 1e3, 4),
            "frac": t[bound] / s if s > 0 else None,
            "tflops": w["flops"] / s / 1e12, "flops_peak": w["peak"],
            "ttrans_per_s": w["trans"] / s / 1e12, "gbs": w["bytes"] / s / 1e9}


# HBM traffic of the dominant kernel: FETCH_SIZE and WRITE_SIZE per dispatch from rocprofv3 --pmc,
# scaled by the same counters on a plain device copy (profiles/, written by
# ``python -m paper_0911_4114_amd.profiling traffic``); reported only while the kernel's source file
# is the one the counters were taken on, else null.
TRAFFIC_FILES = {
    "p2p": ("profiles/traffic_p2p_fp32_sphere1M_k177.txt", "p2p_kernel<float, float2, false, false, 1>"),
    "m2l": ("profiles/traffic_m2l_fp32_sphere1M_k177.txt", "m2lt_kernel<float2, 64, false>*"),
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
    nlaunch = max(cand[dom]["launches_per_step"], 1.0)
    per_launch_ms = cand[dom]["ms_per_step"] / nlaunch
    wd = stage_work(info, dom)
    if dom in ("m2m", "l2l", "gather", "scatter"):
        achieved = wd["bytes"] / nlaunch / (per_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        # the FLOP peak of the stage's precision: P2P carries FP64 distance and phase arithmetic
        # (FP64 vector peak), the other ALU stages FP32 vector arithmetic
        achieved = wd["flops"] / nlaunch / (per_launch_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": wd["peak"], "unit": "TFLOP/s",
                "frac": achieved / wd["peak"], "traffic": None,
                "trans_frac": wd["trans"] / nlaunch / (per_launch_ms * 1e-3) / 1e12 / TRANS_PEAK_TPS}
    roof["stage"] = dom
    roof["launch_ms"] = per_launch_ms
    roof["traffic"] = measured_traffic(dom, args)
    # every stage against its own roofline, and the whole matvec: the sum of the stages'
    # roofline times over the measured matvec time
    stage_roof = {k: stage_roofline(info, k, v["ms_per_step"]) for k, v in cand.items()}
    roof_sum_ms = sum(v["roofline_ms"] for v in stage_roof.values())
    matvec_roof = {"roofline_ms": roof_sum_ms, "measured_ms": ms, "frac": roof_sum_ms / ms,
                   "stages_alone_ms": sum(v["ms"] for v in stage_roof.values())}

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
                         % (len(tg), n, n, cpu_s),
               "cpu_model": cpu_model()}
        # the same sum on one host core (OpenMP limited to one thread), 256 targets
        t1 = time.perf_counter()
        with omp_threads(1):
            direct.matvec(x, q, args.kappa, targets=tg[:256])
        s1 = time.perf_counter() - t1
        cpu["one_core"] = {"value": 256 / s1 / 1e6, "unit": "Mpoints/s", "cores": 1,
                           "sample": "oracle direct sum, 256 of %d targets, %.1f s" % (n, s1)}
        # the oracle's Fourier-basis FMM (CPU FP64, NumPy) per matvec on a reduced sphere of the
        # same points per wavelength: 2^16 points, kappa = 177 (2^16 / 2^20)^(1/2); transfer
        # tables built before the timed call (setup)
        cpu["ffmm"] = oracle_ffmm_timing(args.eps)
        log("fp32 rel err %.3e; cpu %.4f Mpoints/s (one core %.5f; oracle FMM %s)"
            % (rel_err, cpu["value"], cpu["one_core"]["value"], cpu["ffmm"]))

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
        tune_b_s = time.perf_counter() - t0
        msb = timed(lambda: pb.matvec(qb), max(3, args.steps // 2), 1)
        # per-stage times of the batched matvec (every stage alone, P2P on the whole GPU)
        pb.set_tuning(p2p_blocks_per_cu=0)
        pb.profile(True)
        pb.matvec(qb)
        profb = pb.profile_read()
        pb.profile(False)
        pb.set_tuning(**tuned)
        batched = {"nrhs": nb_rhs, "value": n * nb_rhs / (msb * 1e-3) / 1e6, "ms_per_step": msb,
                   "tuning": tuned, "autotune_s": tune_b_s,
                   "stages_ms": {k: round(v[0], 4) for k, v in profb.items()}}
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

    # the FP32 near field with the opt-in FP32 distance and phase (fast_near_phase), beside the
    # default FP64 distance and phase: time and error of the same workload
    fast = None
    if not args.no_fast:
        pf = ff.Plan(xt, args.kappa, args.eps, precision="fp32", depth=args.depth or None,
                     fast_near_phase=True)
        pf.set_tuning(**plan_tuning)
        msf = timed(lambda: pf.matvec(q32), args.steps, args.warmup)
        pf.set_tuning(near_stream=0, p2p_blocks_per_cu=0)
        pf.profile(True)
        for _ in range(3):
            pf.matvec_stages(q32, ff.STAGE_NEAR)
        p2p_fast = pf.profile_read()["p2p"][0] / 3
        pf.profile(False)
        pf.set_tuning(**plan_tuning)
        fast = {"ms_per_step": msf, "value": n / (msf * 1e-3) / 1e6, "p2p_ms": p2p_fast}
        if not args.no_cpu:
            of = pf.matvec(q32).cpu().numpy().astype(np.complex128)
            fast["rel_err"] = float(np.linalg.norm(of[tg] - ref) / np.linalg.norm(ref))
        log("fast near phase: %s" % fast)
        del pf
        torch.cuda.empty_cache()

    # the plain FP64 workload of the paper's volume shape: 4096 points uniform in the unit cube,
    # kappa = 8 pi, depth 3, eps 1e-6, against the full direct sum (and the oracle's CPU FMM)
    cube = None
    if not args.no_cube:
        nc, kc = 4096, 8.0 * np.pi
        xc = wl.cube_points(nc, seed=0)
        qc = wl.complex_normal(nc, seed=1)
        pc = ff.Plan(torch.as_tensor(xc, dtype=torch.float64, device=dev), kc, 1e-6,
                     precision="fp64", depth=3, best_effort=True)
        qct = torch.as_tensor(qc, dtype=torch.complex128, device=dev)
        msc = timed(lambda: pc.matvec(qct), args.steps, args.warmup)
        ic = pc.info()
        cube = {"n": nc, "kappa": kc, "depth": 3, "eps": 1e-6, "ms_per_step": msc,
                "value": nc / (msc * 1e-3) / 1e6, "predicted_err": max(ic["predicted_err"][2:4])}
        if not args.no_cpu:
            from oracle.ffmm import Plan as OPlan
            oc = pc.matvec(qct).cpu().numpy()
            rc = direct.matvec(xc, qc, kc)
            cube["rel_err"] = float(np.linalg.norm(oc - rc) / np.linalg.norm(rc))
            op = OPlan(xc, kc, 1e-6, depth=3)
            for l in range(2, 4):
                op.table(l)
            t0 = time.perf_counter()
            oo = op.matvec(qc)
            cube["cpu_ffmm_s"] = time.perf_counter() - t0
            cube["cpu_ffmm_rel_err"] = float(np.linalg.norm(oo - rc) / np.linalg.norm(rc))
        log("cube: %s" % cube)
        del pc
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
        tune64_s = None
        if not args.no_tune and not args.serial:
            # the FP64 plan's own launch configuration (setup, not timed)
            t0 = time.perf_counter()
            p64.autotune(q64)
            torch.cuda.synchronize()
            tune64_s = time.perf_counter() - t0
        ms64 = timed(lambda: p64.matvec(q64), max(3, args.steps // 2), 2)
        out64 = p64.matvec(q64).cpu().numpy()
        i64 = p64.info()
        # per-stage times of the FP64 plan (every stage alone, P2P on the whole GPU, as for FP32)
        tuned64 = p64.tuning()
        p64.set_tuning(p2p_blocks_per_cu=0)
        p64.profile(True)
        for _ in range(3):
            p64.matvec(q64)
        prof64 = p64.profile_read()
        p64.profile(False)
        p64.set_tuning(**tuned64)
        fp64 = {"value": n / (ms64 * 1e-3) / 1e6, "ms_per_step": ms64, "setup_s": s64,
                "depth": i64["depth"], "eps": 1e-6, "tuning": tuned64, "autotune_s": tune64_s,
                "stages_ms": {k: round(v[0] / 3, 4) for k, v in prof64.items()}}
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
        "config": {"workload": workload_label(n, args.kappa, args.eps, info),
                   "n": n, "kappa": args.kappa, "eps": args.eps, "nrhs": 1,
                   "depth": info["depth"], "ell": info["ell"][2:], "K": info["K"][2:],
                   "boxes": info["n_boxes"][2:], "ilist": info["n_ilist"][2:],
                   "near_pairs": info["n_near_pairs"]},
        "rel_err": rel_err,
        "adjoint": {"value": n / (ms_adj * 1e-3) / 1e6, "ms_per_step": ms_adj},
        "setup_s": setup_s,
        "tuning": plan_tuning,
        "autotune_s": tune_s,
        "stages": stage_roof,
        "matvec_roofline": matvec_roof,
        "fast_near_phase": fast,
        "cube": cube,
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
