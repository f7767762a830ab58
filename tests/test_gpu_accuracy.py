"""Accuracy across the leaf box size in wavelengths (the error-control study of Sections 3.3-3.5),
reduced. With the default design radius (alpha = 0.8) the measured error meets eps up to ka ~ 100
at eps 1e-4 (pairs near opposite box corners exceed the radius the quadrature resolves beyond
that); with alpha = 1 it meets eps 1e-4 up to ka = 1000 (checked at 500)."""
import numpy as np
import pytest

from _gpu_common import log
from accuracy_report import run

pytestmark = pytest.mark.gpu


def test_error_meets_eps_across_ka():
    rows = run(n=2048, kas=(1.0, 5.0, 20.0, 50.0), log=log)
    rows += run(n=2048, kas=(500.0,), cases=(("fp64", 1e-4), ("fp32", 1e-4)), alpha=1.0, log=log)
    for ka, prec, eps, err, pred, ell, K, setup in rows:
        log("ka %g %s eps %.0e: err %.2e predicted %.2e ell %d K %d" % (ka, prec, eps, err, pred, ell, K))
        if pred < eps:
            # outside the low-frequency breakdown the measured error stays below the target
            assert err < eps, (ka, prec, eps, err)
        else:
            # in the breakdown the plan reports what it can reach; the result stays near that
            assert err < 10 * pred, (ka, prec, eps, err, pred)
