"""Per-level error contributions (tests/level_errors.py writes the full report): 2^16 sphere
points at kappa 44.25 and depth 4 (the leaf ka of the 2^20 benchmark), FP64 at eps 1e-6 and FP32
at eps 1e-4, against exact per-level sums on 384 sampled targets."""
import pytest

from _gpu_common import log
import level_errors as le

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,eps,split_tol", [("fp64", 1e-6, 1e-9), ("fp32", 1e-4, 1e-5)])
def test_level_contributions(prec, eps, split_tol):
    r = le.study(1 << 16, 44.25, eps, prec, depth=4, ntarget=384)
    for row in r["rows"]:
        log("%s level %d ka %.2f ell %d share %.3f predicted %.2e measured %.2e"
            % (prec, row["l"], row["ka"], row["ell"], row["share"], row["predicted"], row["err"]))
    log("%s total %.2e split %.1e" % (prec, r["total"], r["split"]))
    # the far field restricted to one level's transfer pass, summed over levels, is the far field
    assert r["split"] < split_tol
    # every level carries about a quarter to a third of phi on the sphere, and stays well inside eps
    assert all(0.2 < row["share"] < 0.4 for row in r["rows"])
    assert all(row["err"] < 0.5 * eps for row in r["rows"])
    assert r["total"] < eps
