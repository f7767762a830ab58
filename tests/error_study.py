"""The error-control study of Section 3.5 on the HIP path's own parameters and tables
(test-side measurement; the oracle supplies only the reference series and the exact kernel).

* Single level (Section 3.5.1, Figs. Error_R0Z and Error_R0X): for a box of side a = 1 at
  wavenumber ka, a GPU plan chooses ell, N_theta and N_phi(theta_n) for the target eps and builds
  the transfer functions T^{s,LL} on the GPU. With those, the quadrature sum
  sum_k w_k e^{i ka s_k.r} T_{r0}(s_k) is compared, over many directions r-hat at the design
  radius |r|, with the exact e^{i ka |r + r0|} / |r + r0| (eps_T) and with the truncated Gegenbauer
  series (eps_I); eps_G is the series against the exact value (eqns. eps_T, eps_G, eps_I), for
  r0 = 2 z-hat (the worst case of the theta quadrature) and r0 = 2 x-hat (of the phi quadrature).
  The plan also reports K / 2(ell + 1)^2 (Fig. QuadSize; (4/pi)(ell+1)(ell+2)/2(ell+1)^2 -> 2/pi).
* Multilevel (Section 3.5.2, Fig. Error_Quad): two points at opposite corners of level-2 boxes of
  side 1 whose centres differ by 2 x-hat, kappa = 100, alpha = 0.8, L = 2..8 levels: eps_T^L of
  the GPU matvec and the drift |eps_I^L - eps_I^2| of the up- and downward passes.
* Convergence to eps_G (Fig. GegError_Quad): kappa = 100, alpha = 1/sqrt(3), two active levels,
  ell held fixed at level 2 and the quadrature grown by lowering its target: eps_T -> eps_G.

Run from the repository root on a GPU machine: python tests/error_study.py > study.md
"""
import argparse
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_0911_4114_amd as ff  # noqa: E402
from oracle import special as osp  # noqa: E402
from oracle.quadrature import LevelQuad  # noqa: E402

KA_DEFAULT = (0.5, 1.0, 2.0, 3.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0, 500.0, 1000.0)


def code_of(d):
    return (d[0] + 3) + 7 * (d[1] + 3) + 49 * (d[2] + 3)


def series(ka, r, r0, ell):
    """Truncated Gegenbauer series of e^{i ka |r + r0|} / |r + r0| (Section 2.1) for rows of r."""
    n = np.arange(ell + 1)
    rn = np.linalg.norm(r, axis=1)
    cosg = (r @ r0) / (rn * np.linalg.norm(r0))
    P = osp.legendre_table(ell, cosg)
    jn = np.stack([osp.sph_jn(ell, ka * v) for v in rn], axis=1)       # [ell+1, nr]
    hn = osp.sph_h1(ell, ka * np.linalg.norm(r0))
    return np.sum((1j * ka * ((-1.0) ** n) * (2 * n + 1) * hn)[:, None] * jn * P, axis=0)


def unit_dirs(axis, nrand=40, seed=0):
    """+-axis and random unit vectors (the maximum over directions, Section 3.5.1)."""
    a = np.asarray(axis, float)
    rnd = np.random.default_rng(seed).standard_normal((nrand, 3))
    d = np.vstack([a, -a, rnd])
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def single_level(ka, eps, precision="fp64"):
    """eps_G, eps_I, eps_T (max over directions) for r0 along z and x on the parameters and tables
    of a GPU plan whose level-2 boxes have ka = kappa a_2 (4096 cube points, depth 2, eps_safety 1,
    best effort in the low-frequency breakdown)."""
    from paper_0911_4114_amd import workloads as wl
    x = wl.cube_points(4096, seed=0)
    side = float((x.max(axis=0) - x.min(axis=0)).max())
    a = side / 4.0
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    p = ff.Plan(xt, ka / a, eps, precision=precision, depth=2, eps_safety=1.0, best_effort=True)
    info = p.info()
    q = LevelQuad(info["ell"][2], info["ntheta"][2], p.nphi(2))
    s, w = q.dirs(), q.weights()
    ell = q.ell
    # the radius the plan designed for: the box diagonal above ka = 100 where eps is reachable
    # there, else 0.8 sqrt(3) a; in the low-frequency breakdown (eps out of reach at 0.8 sqrt(3))
    # ell minimises the error at |r| = a
    from oracle.quadrature import gegenbauer_error, rounding_floor, UNIT_ROUNDOFF
    u = UNIT_ROUNDOFF[precision]
    pred = {al: gegenbauer_error(ka, al * np.sqrt(3.0), 2.0, ell)[ell] + rounding_floor(ka, 2.0, ell, u)[ell]
            for al in (0.8, 1.0)}
    if ka > 100.0 and pred[1.0] < eps:
        rad, regime = np.sqrt(3.0), "diagonal"
    elif pred[0.8] < eps:
        rad, regime = 0.8 * np.sqrt(3.0), "0.8 diagonal"
    else:
        rad, regime = 1.0, "breakdown"
    res = {"ka": ka, "eps": eps, "ell": ell, "ntheta": q.ntheta, "K": q.K,
           "quad_ratio": q.K / (2.0 * (ell + 1) ** 2), "radius": rad, "regime": regime,
           "predicted": info["predicted_err"][2]}
    for name, axis in (("z", (0.0, 0.0, 1.0)), ("x", (1.0, 0.0, 0.0))):
        r0 = 2.0 * np.asarray(axis)
        # T_{r0} of the plan (the GPU table, rebuilt through the quadrature symmetry); code of the
        # transfer vector in box units, a_2 = 1 in these units
        # (physical units: T scales as 1 / length, so the box-unit function is a times the table)
        tab = a * p.transfer(2, code_of((int(r0[0]), int(r0[1]), int(r0[2]))))
        rr = rad * unit_dirs(axis)
        quadv = np.empty(len(rr), complex)
        for i0 in range(0, len(rr), 8):
            quadv[i0:i0 + 8] = (np.exp(1j * ka * (rr[i0:i0 + 8] @ s.T)) * (w * tab)).sum(axis=1)
        big = np.linalg.norm(rr + r0, axis=1)
        exact = np.exp(1j * ka * big) / big
        ser = series(ka, rr, r0, ell)
        res[name] = {"eps_T": float(np.abs(quadv - exact).max()),
                     "eps_G": float(np.abs(ser - exact).max()),
                     "eps_I": float(np.abs(quadv - ser).max())}
    del p
    torch.cuda.empty_cache()
    return res


def two_point_plan(kappa, xj, xi, depth, precision="fp64", **kw):
    """GPU plan over a source point x_j (charge 1) and a target x_i with two uncharged points fixing
    the root cube to [0, 4]^3 (level-2 boxes of side 1); returns phi_i and the plan's info."""
    frame = np.array([[0.0, 0.0, 0.5], [4.0, 4.0, 4.0]])
    x = np.vstack([xj, xi, frame])
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    p = ff.Plan(xt, kappa, kw.pop("eps"), precision=precision, depth=depth, best_effort=True, **kw)
    q = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=torch.complex128, device="cuda")
    phi = complex(p.matvec(q).cpu().numpy()[1])
    info = p.info()
    del p
    return phi, info


def multilevel(eps, levels=(2, 3, 4, 5, 6, 7, 8)):
    """Fig. Error_Quad on the GPU: eps_T^L and |eps_I^L - eps_I^2| for the corner pair."""
    kappa, dd = 100.0, 1e-9
    xj = np.array([dd, dd, dd])
    xi = np.array([3.0 - dd, 1.0 - dd, 1.0 - dd])
    rr = (xi - np.array([2.5, 0.5, 0.5])) - (xj - np.array([0.5, 0.5, 0.5]))
    R = np.linalg.norm(xi - xj)
    exact = np.exp(1j * kappa * R) / R
    rows = []
    ei2 = None
    for L in levels:
        phi, info = two_point_plan(kappa, xj, xi, L, eps=eps, alpha=0.8, eps_safety=1.0)
        ser = series(kappa, rr[None, :], np.array([2.0, 0.0, 0.0]), info["ell"][2])[0]
        ei = phi - ser
        if ei2 is None:
            ei2 = ei
        rows.append({"L": L, "K2": info["K"][2], "eps_T": abs(phi - exact), "eps_G": abs(ser - exact),
                     "eps_I": abs(ei), "drift": abs(ei - ei2)})
    return rows


def convergence(target, eps_q=(1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12)):
    """Fig. GegError_Quad on the GPU: ell fixed at level 2 where the design radius |r| = 1 has a
    Gegenbauer error of ``target``, the quadratures grown by their target; eps_T against eps_G."""
    from oracle.quadrature import gegenbauer_error
    kappa = 100.0
    h = 0.5 / np.sqrt(3.0)
    xj = np.full(3, 0.5 - h)
    xi = np.array([2.5 + h, 0.5 + h, 0.5 + h])
    rr = (xi - np.array([2.5, 0.5, 0.5])) - (xj - np.array([0.5, 0.5, 0.5]))
    R = np.linalg.norm(xi - xj)
    exact = np.exp(1j * kappa * R) / R
    geg = gegenbauer_error(kappa, 1.0, 2.0, 200)
    ell = int(np.nonzero(geg[1:] < target)[0][0]) + 1
    eg = abs(series(kappa, rr[None, :], np.array([2.0, 0.0, 0.0]), ell)[0] - exact)
    rows = []
    for e in eps_q:
        phi, info = two_point_plan(kappa, xj, xi, 3, eps=e, alpha=1.0 / np.sqrt(3.0), eps_safety=1.0,
                                   ell_override={2: ell})
        et = abs(phi - exact)
        rows.append({"eps_q": e, "ell": ell, "K2": info["K"][2], "eps_G": eg, "eps_T": et,
                     "gap": abs(et - eg) / eg})
    return rows


def markdown(single, multi, conv):
    out = ["Single level, box side a = 1 (Figs. Error_R0Z, Error_R0X, QuadSize); errors are maxima "
           "over +-r0-hat and 40 random directions at the radius the plan designed for:", "",
           "| eps | ka | ell | N_theta | K | K/2(ell+1)^2 | radius | r0 | eps_G | eps_I | eps_T | eps_T/eps |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in single:
        for ax in ("z", "x"):
            e = r[ax]
            out.append("| %.0e | %g | %d | %d | %d | %.3f | %s | %s | %.2e | %.2e | %.2e | %.2f |"
                       % (r["eps"], r["ka"], r["ell"], r["ntheta"], r["K"], r["quad_ratio"], r["regime"],
                          ax, e["eps_G"], e["eps_I"], e["eps_T"], e["eps_T"] / r["eps"]))
    out += ["", "Multilevel, corner pair, kappa = 100, alpha = 0.8 (Fig. Error_Quad):", "",
            "| eps | L | K (level 2) | eps_G | eps_I | eps_T | abs(eps_I^L - eps_I^2) |", "|---|---|---|---|---|---|---|"]
    for eps, rows in multi:
        for r in rows:
            out.append("| %.0e | %d | %d | %.2e | %.2e | %.2e | %.1e |"
                       % (eps, r["L"], r["K2"], r["eps_G"], r["eps_I"], r["eps_T"], r["drift"]))
    out += ["", "Convergence to eps_G, kappa = 100, alpha = 1/sqrt(3), two levels (Fig. GegError_Quad):", "",
            "| ell | quadrature target | K (level 2) | eps_G | eps_T | abs(eps_T - eps_G)/eps_G |", "|---|---|---|---|---|---|"]
    for rows in conv:
        for r in rows:
            out.append("| %d | %.0e | %d | %.2e | %.2e | %.1e |" % (r["ell"], r["eps_q"], r["K2"], r["eps_G"],
                                                                r["eps_T"], r["gap"]))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ka", default=",".join("%g" % k for k in KA_DEFAULT))
    a = ap.parse_args(argv)
    kas = [float(v) for v in a.ka.split(",")]
    log = lambda m: print("[study] %s" % m, file=sys.stderr, flush=True)
    single = []
    for eps in (1e-4, 1e-8):
        for ka in kas:
            r = single_level(ka, eps)
            log(r)
            single.append(r)
    multi = [(eps, multilevel(eps)) for eps in (1e-4, 1e-8)]
    log(multi)
    conv = [convergence(t) for t in (1e-4, 1e-6, 1e-8, 1e-10)]
    log(conv)
    print(markdown(single, multi, conv))


if __name__ == "__main__":
    main()
