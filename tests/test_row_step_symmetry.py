"""The half- and quarter-range forms of a phi row step (Section 3.4, steps 1 and 5), restated in
NumPy exactly as the resample kernels arrange them, against the oracle's 1-D Fourier resample.

A row step maps N uniform samples x_m (phi_m = 2 pi m / N) to M samples y_j by the band-limited
resample of Section 3.1.3, y = D^T x with D[m][j] = resample_1d(e_m, M)[j]. The kernels use two
symmetries of that operator (both N and M multiples of 4):
* half turn: sample m + N/2 lies pi from sample m, so u = x_m + x_{m+N/2} carries the even
  Fourier modes and v = x_m - x_{m+N/2} the odd ones; with De, Do = (D[m][j] +- D[m+N/2][j]) / 2
  over m < N/2, y_j = a_j + b_j and y_{j+M/2} = a_j - b_j for a = De^T u, b = Do^T v;
* reflection phi -> -phi, under which the operator is even: u and v split again over
  m = 0..N/4 (the samples 0 and N/4 are fixed, their operator rows halved) into four channels whose
  sums S, A, Mv, P give y_j, y_{j+M/2}, y_{M/2-j}, y_{M-j} for j = 0..M/4.
A dropped fixed-point weight, a wrong sign in the antiperiodic wrap of Do (Do at N/2 is -Do at 0)
or a swapped channel changes the result by O(1) on random data.
"""
import numpy as np
import pytest

from oracle.fourier import resample_1d

SIZES = [(4, 4), (4, 8), (8, 4), (8, 8), (12, 20), (20, 12), (16, 16), (44, 60), (60, 44),
         (96, 128), (128, 96)]


def operator(n, m):
    """D[k][j]: sample j of the resample of the k-th unit vector from n to m samples."""
    return np.real(resample_1d(np.eye(n), m, axis=-1))


def half_range(x, n, m):
    d = operator(n, m)
    h, hh = n // 2, m // 2
    de = 0.5 * (d[:h, :hh] + d[h:, :hh])
    do = 0.5 * (d[:h, :hh] - d[h:, :hh])
    u, v = x[:h] + x[h:], x[:h] - x[h:]
    a, b = de.T @ u, do.T @ v
    return np.concatenate([a + b, a - b])


def quarter_range(x, n, m):
    d = operator(n, m)
    h, q, hh, qq = n // 2, n // 4, m // 2, m // 4
    de = 0.5 * (d[:h, :hh] + d[h:, :hh])
    do = 0.5 * (d[:h, :hh] - d[h:, :hh])
    cs, ca, cm, cp = (np.zeros((q + 1, qq + 1)) for _ in range(4))
    for k in range(q + 1):
        r = (h - k) % h
        wt = 0.5 if k in (0, q) else 1.0
        e0, e1 = de[k, :qq + 1], de[r, :qq + 1]
        o0 = do[k, :qq + 1]
        o1 = -do[0, :qq + 1] if k == 0 else do[r, :qq + 1]
        cs[k], ca[k] = wt * 0.5 * (e0 + e1), wt * 0.5 * (e0 - e1)
        cm[k], cp[k] = wt * 0.5 * (o0 - o1), wt * 0.5 * (o0 + o1)
    k = np.arange(q + 1)
    x0, x1, x2, x3 = x[k], x[k + h], x[h - k], x[(n - k) % n]
    u, ub, v, vb = x0 + x1, x2 + x3, x0 - x1, x2 - x3
    s_, a_, mv, p_ = cs.T @ (u + ub), ca.T @ (u - ub), cm.T @ (v - vb), cp.T @ (v + vb)
    y = np.zeros(m, dtype=complex)
    j = np.arange(qq + 1)
    y[j] = s_ + a_ + mv + p_
    y[j + hh] = s_ + a_ - mv - p_
    inner = np.arange(1, qq)
    y[hh - inner] = (s_ - a_ + p_ - mv)[1:qq]
    y[m - inner] = (s_ - a_ - p_ + mv)[1:qq]
    return y


@pytest.mark.parametrize("n,m", SIZES)
def test_half_range_row_step_equals_resample(n, m):
    rng = np.random.default_rng(n * 1000 + m)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    ref = resample_1d(x, m)
    assert np.allclose(half_range(x, n, m), ref, rtol=0, atol=1e-12 * np.abs(x).sum())


@pytest.mark.parametrize("n,m", SIZES)
def test_quarter_range_row_step_equals_resample(n, m):
    rng = np.random.default_rng(n * 1000 + m + 7)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    ref = resample_1d(x, m)
    assert np.allclose(quarter_range(x, n, m), ref, rtol=0, atol=1e-12 * np.abs(x).sum())


def test_quarter_range_fixed_points_matter():
    """Dropping the half weight of the fixed rows, or the sign of the wrapped odd operator, breaks
    the identity: the pins above see those mistakes."""
    n, m = 16, 24
    rng = np.random.default_rng(3)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    ref = resample_1d(x, m)
    d = operator(n, m)
    h, q, hh, qq = n // 2, n // 4, m // 2, m // 4
    de = 0.5 * (d[:h, :hh] + d[h:, :hh])
    k = np.arange(q + 1)
    u = x[k] + x[k + h] + x[h - k] + x[(n - k) % n]
    # the symmetric even channel without the fixed-point halving
    cs = np.stack([0.5 * (de[i, :qq + 1] + de[(h - i) % h, :qq + 1]) for i in range(q + 1)])
    s_full = cs.T @ u
    s_ok = (cs * np.where((k == 0) | (k == q), 0.5, 1.0)[:, None]).T @ u
    assert np.abs(s_full - s_ok).max() > 1e-3 * np.abs(ref).max()
