"""Accuracy across the leaf box size in wavelengths (the error-control study of Sections 3.3-3.5),
reduced: FP64 at eps 1e-4 and 1e-8, FP32 at 1e-4, ka from the breakdown region to 500. The
default design radius is the paper's 0.8 sqrt(3) a up to ka = 100 and the box diagonal above it
where eps is reachable there. Not covered: FP64 eps 1e-8 near ka = 100, where neither radius
reaches eps with one buffer box (measured 3e-7)."""
import numpy as np
import pytest

from _gpu_common import log
from accuracy_report import run

pytestmark = pytest.mark.gpu


def test_error_meets_eps_across_ka():
    rows = run(n=2048, kas=(1.0, 5.0, 20.0, 50.0, 500.0), log=log)
    for ka, prec, eps, err, pred, ell, K, setup in rows:
        log("ka %g %s eps %.0e: err %.2e predicted %.2e ell %d K %d" % (ka, prec, eps, err, pred, ell, K))
        if pred < eps:
            # outside the low-frequency breakdown the measured error stays below the target
            assert err < eps, (ka, prec, eps, err)
        else:
            # in the breakdown the plan reports what it can reach; the result stays near that
            assert err < 10 * pred, (ka, prec, eps, err, pred)


@pytest.mark.parametrize("by_parent", [1, 0])
def test_fp64_ka_1000_large_tables(by_parent):
    """Level-2 quadrature of ~4.2M directions in FP64 (ka = 1000): the transfer table of the 34
    representative vectors spans 2.3 GB, so table rows sit beyond 2^31 bytes from its start; both
    transfer-pass forms must read them (Section 3.5.1, the high-frequency end of the study)."""
    import torch
    from oracle import direct
    from paper_0911_4114_amd import workloads as wl
    import paper_0911_4114_amd as ff
    x = wl.cube_points(2048, seed=0)
    q = wl.complex_normal(len(x), seed=1)
    xt = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    side = float((x.max(axis=0) - x.min(axis=0)).max())
    kappa = 1000.0 / (side / 4)
    p = ff.Plan(xt, kappa, 1e-6, precision="fp64", depth=2)
    p.set_tuning(m2l_by_parent=by_parent)
    K = p.info()["K"][2]
    log("ka 1000 fp64: K %d, table %.2f GB" % (K, 34 * K * 16 / 1e9))
    assert 34 * K * 16 > 2 ** 31
    out = p.matvec(torch.as_tensor(q, dtype=torch.complex128, device="cuda")).cpu().numpy()
    ref = direct.matvec(x, q, kappa)
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    log("  by_parent %d rel err %.3e" % (by_parent, err))
    assert err < 1e-6
    del p
    torch.cuda.empty_cache()
