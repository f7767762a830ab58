"""Per-level error contributions of the matvec (test-side measurement).

A pair of points (i, j) interacts through the transfer pass of the first level l >= 2 at which
their boxes are not neighbours (Section 2: I(B) holds the boxes whose parents neighbour B's parent
but that do not neighbour B); pairs that are neighbours down to the leaf level form the near field.
The exact contribution of level l to phi_i is therefore the direct sum over the sources j whose
pair level with i is l, computed here from the tree's box indices. The HIP path gives the same
split through ffmm_plan_set_m2l_levels: its far field with only level l's transfer pass. The
per-level error is the difference, relative to the norm of the whole phi over the sampled targets.

Run from the repository root on a GPU machine: python tests/level_errors.py > levels.md
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_0911_4114_amd as ff  # noqa: E402
from paper_0911_4114_amd import workloads as wl  # noqa: E402
from oracle import tree as otree  # noqa: E402


def exact_by_level(x, q, kappa, depth, targets):
    """{l: exact level-l contribution at the targets} plus 'near' and 'total' (FP64)."""
    lo, side = otree.root_cube(x)
    idx = {l: otree.quantize(x, lo, side, l) for l in range(2, depth + 1)}
    out = {l: np.zeros(len(targets), complex) for l in list(range(2, depth + 1)) + ["near"]}
    for ti, i in enumerate(targets):
        d = x - x[i]
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        ok = r > 0.0
        g = np.where(ok, np.exp(1j * kappa * r) / np.where(ok, r, 1.0), 0.0) * q
        lev = np.zeros(len(x), np.int64)
        for l in range(2, depth + 1):
            far = np.abs(idx[l] - idx[l][i]).max(axis=1) >= 2
            lev = np.where((lev == 0) & far, l, lev)
        for l in range(2, depth + 1):
            out[l][ti] = g[lev == l].sum()
        out["near"][ti] = g[lev == 0].sum()
    out["total"] = sum(out[k] for k in out)
    return out


def gpu_by_level(plan, qt, depth):
    """{l: far field of the plan with only level l's transfer pass} in the caller's order."""
    res = {}
    for l in range(2, depth + 1):
        plan.set_m2l_levels([l])
        res[l] = plan.matvec_stages(qt, ff.STAGE_FAR).cpu().numpy().astype(complex)
    plan.set_m2l_levels(None)
    res["far"] = plan.matvec_stages(qt, ff.STAGE_FAR).cpu().numpy().astype(complex)
    res["all"] = plan.matvec(qt).cpu().numpy().astype(complex)
    return res


def study(n, kappa, eps, precision, depth=None, ntarget=512, seed=7):
    x = wl.sphere_points(n, seed=0)
    q = wl.complex_normal(n, seed=1)
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    p = ff.Plan(xt, kappa, eps, precision=precision, depth=depth)
    info = p.info()
    L = info["depth"]
    qt = torch.as_tensor(q, dtype=torch.complex128, device="cuda")
    if precision == "fp32":
        qt = qt.to(torch.complex64)
    got = gpu_by_level(p, qt, L)
    tg = wl.subset(n, ntarget, seed=seed)
    ex = exact_by_level(x, q, kappa, L, tg)
    nt = np.linalg.norm(ex["total"])
    a = info["root_side"] / 2 ** np.arange(L + 1)
    rows = []
    for l in range(2, L + 1):
        rows.append({"l": l, "ka": kappa * a[l], "ell": info["ell"][l], "K": info["K"][l],
                     "predicted": info["predicted_err"][l],
                     "err": float(np.linalg.norm(got[l][tg] - ex[l]) / nt),
                     "share": float(np.linalg.norm(ex[l]) / nt)})
    total = float(np.linalg.norm(got["all"][tg] - ex["total"]) / nt)
    far_sum = sum(got[l] for l in range(2, L + 1))
    split = float(np.linalg.norm(far_sum[tg] - got["far"][tg]) / np.linalg.norm(got["far"][tg]))
    del p
    torch.cuda.empty_cache()
    return {"n": n, "kappa": kappa, "eps": eps, "precision": precision, "depth": L, "rows": rows,
            "total": total, "split": split, "ntarget": ntarget}


def markdown(results):
    out = []
    for r in results:
        out.append("%s, N = %d on the unit sphere, kappa = %g, eps = %.0e, depth %d, %d sampled "
                   "targets; errors relative to |phi| over the targets (total %.2e; the per-level far "
                   "fields add up to the whole far field to %.1e):" % (r["precision"].upper(), r["n"],
                   r["kappa"], r["eps"], r["depth"], r["ntarget"], r["total"], r["split"]))
        out += ["", "| level | ka | ell | K | share of phi | predicted (design radius) | measured |",
                "|---|---|---|---|---|---|---|"]
        for row in r["rows"]:
            out.append("| %d | %.2f | %d | %d | %.3f | %.2e | %.2e |" % (row["l"], row["ka"], row["ell"], row["K"],
                                                                    row["share"], row["predicted"], row["err"]))
        out.append("")
    return "\n".join(out)


def main():
    res = []
    for n, kappa, depth, targets in ((1 << 16, 44.25, 4, 512), (1 << 20, 177.0, None, 256)):
        for prec, eps in (("fp64", 1e-6), ("fp32", 1e-4)):
            r = study(n, kappa, eps, prec, depth=depth, ntarget=targets)
            print("[levels] %s" % r, file=sys.stderr, flush=True)
            res.append(r)
    print(markdown(res))


if __name__ == "__main__":
    main()
