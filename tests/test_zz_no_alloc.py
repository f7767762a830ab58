"""The allocation-free matvec (ffmm_matvec_static, C-ABI through the binding) against ffmm_matvec:
the same kernels on workspaces in the library's static device array, so the results are the same
bits; two calls in a row, the second on a smaller plan and fewer right-hand sides, so that the
second call runs over what the first left in the array. Also the size limit and the direct
method."""
import numpy as np
import pytest
import torch

import paper_0911_4114_amd as ff
from paper_0911_4114_amd import workloads as wl
from oracle import direct
from _gpu_common import log, dev_points, dev_complex, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,eps", [("fp32", 1e-4), ("fp64", 1e-6)])
def test_static_matvec_equals_matvec_twice(prec, eps):
    assert torch.cuda.is_available()
    f32 = prec == "fp32"
    # the second call is the smaller one; workspaces 39 and 6 MiB (FP32), 48 and 20 MiB (FP64)
    cases = [(9000, 40.0, 2), (2500, 25.0, 1)] if f32 else [(6000, 30.0, 2), (2500, 25.0, 1)]
    for n, kappa, nrhs in cases:
        log("static matvec %s n=%d kappa=%g nrhs=%d" % (prec, n, kappa, nrhs))
        x = wl.sphere_points(n, seed=11)
        q = wl.complex_normal(n, seed=12, nrhs=nrhs)
        p = ff.Plan(dev_points(x), kappa, eps, precision=prec, max_rhs=nrhs)
        qt = dev_complex(q, f32)
        ref_lib = p.matvec(qt)
        out = torch.empty_like(ref_lib)
        got = p.matvec_static(qt, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        a = got.cpu().numpy()
        b = ref_lib.cpu().numpy()
        assert np.array_equal(a, b), "static workspace changed the result"
        tg = wl.subset(n, 600)
        ref = direct.matvec(x, q[0], kappa, targets=tg)
        err = rel_l2(a[0][tg].astype(complex), ref)
        log("  rel err vs direct sum %.3e" % err)
        assert err < eps
        # the plan's own entry point still gives the same bits after the static call
        assert np.array_equal(p.matvec(qt).cpu().numpy(), b)


def test_static_matvec_direct_method_and_limit():
    n = 3000
    x = wl.sphere_points(n, seed=13)
    q = wl.complex_normal(n, seed=14)
    pd = ff.Plan(dev_points(x), 30.0, 1e-4, precision="fp32", method="direct")
    qt = dev_complex(q, True)
    log("static matvec direct n=%d" % n)
    assert np.array_equal(pd.matvec_static(qt).cpu().numpy(), pd.matvec(qt).cpu().numpy())
    # workspace of 8 right-hand sides of 2^18 FP64 points: 3 x 32 MiB > the 64 MiB array
    nb = 1 << 18
    xb = wl.sphere_points(nb, seed=15)
    pb = ff.Plan(dev_points(xb), 20.0, 1e-6, precision="fp64", max_rhs=8)
    qb = dev_complex(wl.complex_normal(nb, seed=16, nrhs=8))
    log("static matvec size limit n=%d nrhs=8" % nb)
    with pytest.raises(ff.FfmmError) as ei:
        pb.matvec_static(qb)
    assert ei.value.status == -4 and "static array" in str(ei.value)
    # a call that fits still works afterwards, on the same plan
    one = pb.matvec_static(qb[0])
    assert np.array_equal(one.cpu().numpy(), pb.matvec(qb[0]).cpu().numpy())
