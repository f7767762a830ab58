"""1D Fourier tools (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

Conventions (Table 1 and Section 3.1):
* A periodic function is f(x) = sum_n F_n e^{i n x}; on N uniform samples x_j = 2 pi j / N the
  coefficients are F_n = DFT(f)_n / N.
* Band limit. Every inter/anterpolation between N and N' samples keeps the frequencies
  |n| <= min(N, N')/2 - 1 and drops the Nyquist bin. The printed data of Fig. SINconv fixes this:
  the quadrature there has K = 2N + 2 points for the band |n| <= N (the caption's K = 2N + 1
  does not reproduce the printed numbers; the truncation |n| <= N_theta/2 - 1 of Section 3.2 and of
  the T^{s,LL} sums in Section 3.3.2 is the same convention).
"""
import numpy as np


def sin_abs_coeff(n):
    """Fourier coefficients of |sin t| (Section 3.1.3): ((-1)^n + 1) / (pi (1 - n^2)),
    which is 0 for odd n (including n = +-1) and 2/(pi (1 - n^2)) for even n."""
    n = np.asarray(n)
    out = np.zeros(n.shape, dtype=np.float64)
    even = (n % 2) == 0
    ne = n[even].astype(np.float64)
    out[even] = 2.0 / (np.pi * (1.0 - ne * ne))
    return out


def band(n_src, n_dst):
    """Highest frequency kept when resampling between n_src and n_dst samples."""
    return min(n_src, n_dst) // 2 - 1


def resample_1d(x, n_new, axis=-1):
    """Fourier interpolation (zero padding, n_new > N) or anterpolation (truncation, n_new < N)
    of the samples x along ``axis`` (Section 3.1.3). Keeps |k| <= min(N, n_new)/2 - 1."""
    x = np.asarray(x)
    x = np.moveaxis(x, axis, -1)
    n = x.shape[-1]
    coef = np.fft.fft(x, axis=-1) / n
    b = band(n, n_new)
    out = np.zeros(x.shape[:-1] + (n_new,), dtype=np.complex128)
    if b >= 0:
        out[..., : b + 1] = coef[..., : b + 1]
        if b >= 1:
            out[..., n_new - b:] = coef[..., n - b:]
    y = np.fft.ifft(out, axis=-1) * n_new
    return np.moveaxis(y, -1, axis)


def coeffs_symmetric(x):
    """Fourier coefficients F_n, n = -(N-1)/2..(N-1)/2, of N (odd) uniform samples."""
    n = x.shape[-1]
    assert n % 2 == 1
    c = np.fft.fft(x, axis=-1) / n
    h = (n - 1) // 2
    return np.concatenate([c[..., n - h:], c[..., : h + 1]], axis=-1)


def sin_filtered_quadrature(g, nband, k):
    """The toy problem of Section 3.1.2: integrate |sin t| g(t) over [0, 2 pi] with a uniform
    quadrature of k points after truncating the spectrum of |sin t| to |n| <= nband (eqn. fN)."""
    assert 2 * nband < k
    t = 2.0 * np.pi * np.arange(k) / k
    spec = np.zeros(k)
    n = np.arange(0, nband + 1)
    spec[n] = sin_abs_coeff(n)
    spec[k - n[1:]] = sin_abs_coeff(n[1:])
    f = np.real(np.fft.ifft(spec) * k)          # sum_{|n| <= nband} s_n e^{i n t}
    return 2.0 * np.pi / k * np.sum(f * g(t))


def trapezoid_quadrature(g, k):
    """Uniform (trapezoid) quadrature of |sin t| g(t) with k points (Fig. SINconv, squares)."""
    t = 2.0 * np.pi * np.arange(k) / k
    return 2.0 * np.pi / k * np.sum(np.abs(np.sin(t)) * g(t))
