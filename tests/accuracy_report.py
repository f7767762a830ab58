"""Accuracy of the HIP path across the box size in wavelengths (the error-control study of
Sections 3.3-3.5): for leaf boxes of ka = kappa a from 0.5 to 1000, the relative L2 error of phi
against the oracle's direct sum, next to the requested eps and the plan's own a priori prediction
(truncation of the Gegenbauer series plus the rounding floor, Section 2.1), for the FP64 path at
eps 1e-4 and 1e-8 and the FP32 path at eps 1e-4. Below ka ~ 2 the low-frequency breakdown caps
the reachable accuracy (Sections 2.1, 3.5.1), which the predicted column shows.

The oracle (CPU) computes the reference; this is a test-side measurement script (run it from the
repository root on a GPU machine):

    python tests/accuracy_report.py [--n 4096] [--ka 0.5,1,2,...] > report.md
"""
import os
import argparse
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_0911_4114_amd as ff  # noqa: E402
from paper_0911_4114_amd import workloads as wl  # noqa: E402

KA_DEFAULT = (0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0, 500.0, 1000.0)
CASES = (("fp64", 1e-4), ("fp64", 1e-8), ("fp32", 1e-4))


def run(n=4096, kas=KA_DEFAULT, cases=CASES, depth=2, log=None, alpha=None):
    """Rows of (ka, precision, eps, rel_err, predicted, ell, K, setup_s) for n uniform points in
    the unit cube at the given depth (leaf side a = root side / 2^depth)."""
    from oracle import direct
    dev = torch.device("cuda")
    x = wl.cube_points(n, seed=0)
    q = wl.complex_normal(n, seed=1)
    xt = torch.as_tensor(x, dtype=torch.float64, device=dev)
    side = ff.Plan(xt, 1.0, 1e-4, depth=depth, best_effort=True).info()["root_side"]
    a = side / 2 ** depth
    rows = []
    for ka in kas:
        kappa = ka / a
        ref = direct.matvec(x, q, kappa)
        for prec, eps in cases:
            t0 = time.perf_counter()
            # best effort: in the low-frequency breakdown the plan keeps the most accurate
            # parameters the precision allows, so that the study can show what is reached there
            p = ff.Plan(xt, kappa, eps, precision=prec, depth=depth, alpha=alpha, best_effort=True)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            qd = torch.as_tensor(q, dtype=torch.complex128, device=dev)
            if prec == "fp32":
                qd = qd.to(torch.complex64)
            out = p.matvec(qd).cpu().numpy().astype(np.complex128)
            info = p.info()
            err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
            row = (ka, prec, eps, err, max(info["predicted_err"][2:]), info["ell"][depth],
                   info["K"][depth], setup)
            rows.append(row)
            if log:
                log(row)
            del p
            torch.cuda.empty_cache()
    return rows


def markdown(rows, n, depth):
    out = ["| ka (leaf) | path | eps | measured rel. L2 error | predicted (per level) | ell (leaf) | "
           "K (leaf) | setup (s) |", "|---|---|---|---|---|---|---|---|"]
    for ka, prec, eps, err, pred, ell, K, setup in rows:
        out.append("| %g | %s | %.0e | %.2e | %.2e | %d | %d | %.2f |" % (ka, prec.upper(), eps, err, pred,
                                                                        ell, K, setup))
    out.append("")
    out.append("%d points uniform in the unit cube (seed 0), complex N(0,1) charges (seed 1), depth %d, "
               "reference: the oracle's direct sum." % (n, depth))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--ka", default=",".join("%g" % k for k in KA_DEFAULT))
    ap.add_argument("--alpha", type=float, default=None, help="design radius factor (default: the plan's)")
    a = ap.parse_args(argv)
    kas = [float(v) for v in a.ka.split(",")]
    rows = run(a.n, kas, depth=a.depth, alpha=a.alpha,
               log=lambda r: print("[accuracy] %s" % (r,), file=sys.stderr, flush=True))
    print(markdown(rows, a.n, a.depth))


if __name__ == "__main__":
    main()
