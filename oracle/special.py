"""Special functions used by the oracle (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

Notation follows Table 1 of the paper: j_n, y_n spherical Bessel functions of the first and
second kind, h_n^(1) = j_n + i y_n the spherical Hankel function, P_n the Legendre polynomial,
J_n the Bessel function of the first kind (used for the plane-wave spectrum, eqn. PlaneWaveSpec).

The Bessel functions are taken from scipy.special (a library routine serving as a step); the
Legendre polynomials are the three-term recurrence written out.
"""
import numpy as np
from scipy import special as _sp


def sph_jn(nmax, x):
    """j_n(x) for n = 0..nmax (Table 1). Returns array [nmax+1] (+ x.shape)."""
    n = np.arange(nmax + 1)
    x = np.asarray(x, dtype=np.float64)
    return _sp.spherical_jn(n.reshape((-1,) + (1,) * x.ndim), x)


def sph_yn(nmax, x):
    """y_n(x) for n = 0..nmax (Table 1)."""
    n = np.arange(nmax + 1)
    x = np.asarray(x, dtype=np.float64)
    return _sp.spherical_yn(n.reshape((-1,) + (1,) * x.ndim), x)


def sph_h1(nmax, x):
    """Spherical Hankel function of the first kind h_n^(1)(x) = j_n(x) + i y_n(x), n = 0..nmax."""
    return sph_jn(nmax, x) + 1j * sph_yn(nmax, x)


def legendre_table(nmax, t):
    """P_n(t) for n = 0..nmax by the three-term recurrence
    (n+1) P_{n+1} = (2n+1) t P_n - n P_{n-1}. Returns [nmax+1] + t.shape."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty((nmax + 1,) + t.shape)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = t
    for n in range(1, nmax):
        out[n + 1] = ((2 * n + 1) * t * out[n] - n * out[n - 1]) / (n + 1)
    return out


def bessel_jn_abs(nmax, x):
    """|J_n(x)| for n = 0..nmax (integer order). |J_{-n}| = |J_n|, so this covers negative n too.
    Used for the plane-wave spectrum of eqn. PlaneWaveSpec / PlaneWaveSpecX."""
    n = np.arange(nmax + 1)
    return np.abs(_sp.jv(n, x))
