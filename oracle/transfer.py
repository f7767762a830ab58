"""Transfer function and band-limited modified transfer function
(TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

* eqn. TransferFn (Section 2):
      T_{ell,r0}(s) = (i kappa / 4 pi) sum_{n=0}^{ell} i^n (2n+1) h_n^(1)(kappa |r0|) P_n(s . r0/|r0|)
* eqn. modifiedIntegrand / FBFMM (Section 3): T^s(theta, phi) = 1/2 T(s) |sin theta| on the doubled
  sphere (theta in [0, 2 pi)), s = [cos phi sin theta, sin phi sin theta, cos theta].
* Alg. BMTF (Section 3.2): for every phi column, sample 1/2 T on 2 ell + 1 uniform theta points
  (T is a trigonometric polynomial of degree ell in theta), take its Fourier coefficients,
  convolve them with the |sin| coefficients, keep |n| <= N_theta/2 - 1 and evaluate on the
  theta_n = 2 pi n / N_theta grid.
* Section 3.3.2: each row theta_n is then Fourier anterpolated in phi from the full column count
  to N_phi(theta_n), giving T^{s,LL}.
"""
import numpy as np

from .special import sph_h1, legendre_table
from .fourier import sin_abs_coeff, coeffs_symmetric, resample_1d


def sphere_dirs(theta, phi):
    """s(theta, phi) = [cos phi sin theta, sin phi sin theta, cos theta] (Section 1)."""
    theta, phi = np.broadcast_arrays(np.asarray(theta, float), np.asarray(phi, float))
    st = np.sin(theta)
    return np.stack([np.cos(phi) * st, np.sin(phi) * st, np.cos(theta)], axis=-1)


def transfer_coeffs(kappa, r0norm, ell):
    """c_n = (i kappa / 4 pi) i^n (2n+1) h_n^(1)(kappa |r0|), n = 0..ell (eqn. TransferFn)."""
    n = np.arange(ell + 1)
    h = sph_h1(ell, kappa * r0norm)
    return (1j * kappa / (4.0 * np.pi)) * (1j ** n) * (2 * n + 1) * h


def transfer_eval(kappa, r0, ell, sdirs):
    """T_{ell,r0}(s) at unit vectors sdirs[..., 3] (eqn. TransferFn)."""
    r0 = np.asarray(r0, float)
    r0n = float(np.linalg.norm(r0))
    c = transfer_coeffs(kappa, r0n, ell)
    t = np.clip(sdirs @ (r0 / r0n), -1.0, 1.0)
    P = legendre_table(ell, t)
    return np.tensordot(c, P, axes=1)


def bmtf(kappa, r0, ell, ntheta, ncols, theta_rows=None):
    """Alg. BMTF: the band-limited modified transfer function T^{s,L}_{ell,r0} on the rows
    theta_n = 2 pi n / ntheta, n = 0..ntheta/2 (or at ``theta_rows`` if given) and the columns
    phi_m = 2 pi m / ncols. Returns complex [rows, ncols]."""
    nt = 2 * ell + 1
    thp = 2.0 * np.pi * np.arange(nt) / nt
    phi = 2.0 * np.pi * np.arange(ncols) / ncols
    s = sphere_dirs(thp[:, None], phi[None, :])
    half_t = 0.5 * transfer_eval(kappa, r0, ell, s)            # [nt, ncols]
    tt = coeffs_symmetric(half_t.T).T                          # [p = -ell..ell, ncols]
    kmax = ntheta // 2 - 1
    k = np.arange(-kmax, kmax + 1)
    p = np.arange(-ell, ell + 1)
    conv = sin_abs_coeff(k[:, None] - p[None, :])              # s~_{k-p}
    ts = conv @ tt                                             # [k, ncols]
    if theta_rows is None:
        theta_rows = 2.0 * np.pi * np.arange(ntheta // 2 + 1) / ntheta
    return np.exp(1j * np.outer(theta_rows, k)) @ ts


def full_phi_count(ell):
    """Column count used for T^{s,L} before the per-row anterpolation: the smallest multiple of 4
    that is >= 2 ell + 2, so the phi-band |m| <= ell of T is kept and the Nyquist bin is empty."""
    return 4 * ((2 * ell + 2 + 3) // 4)


def transfer_table(kappa, r0, quad):
    """T^{s,LL}_{ell,r0} sampled on a level quadrature (Section 3.2 + Section 3.3.2): BMTF on
    ntheta/2 + 1 rows and full_phi_count(ell) columns, then each row anterpolated in phi to
    N_phi(theta_n). Returns complex [K] in row-major (row n, then phi index) order."""
    ncols = full_phi_count(quad.ell)
    tl = bmtf(kappa, r0, quad.ell, quad.ntheta, ncols)
    return np.concatenate([resample_1d(tl[n], int(quad.nphi[n])) for n in range(quad.nrows)])
