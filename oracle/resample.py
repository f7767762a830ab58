"""Inter/anterpolation between two level quadratures (TEST INFRASTRUCTURE ONLY; see
oracle/__init__.py).

Section 3.4 describes five steps that move data sampled on a quadrature K (N_theta, N_phi(theta_n))
to a quadrature K' (N'_theta, N'_phi(theta'_n)) with FFTs only. NPhi denotes the largest row
length of either quadrature.
1. every row theta_n, 0 <= n <= N_theta/2: Fourier-resample in phi from N_phi(theta_n) to NPhi;
2. every column phi_m, 0 <= m < NPhi/2: build the theta-periodic sequence of length N_theta with
   the symmetry eqn. NumSphereSym, F(theta_n, phi_m) = F(theta_{N_theta - n}, phi_{m + NPhi/2});
3. resample each such sequence in theta from N_theta to N'_theta;
4. every row theta'_n, 0 <= n <= N'_theta/2: rebuild the phi-periodic sequence of length NPhi by the
   same symmetry;
5. resample each row in phi from NPhi to N'_phi(theta'_n).
Every resample keeps |k| <= min(N, N')/2 - 1 (see oracle/fourier.py).
"""
import numpy as np

from .fourier import resample_1d


def resample_sig(f, q_src, q_dst, nphi_all=None):
    """Five-step resample of signatures f [..., K_src] from q_src to q_dst. Returns [..., K_dst].

    nphi_all is the common phi length NPhi of steps 1-5 (default: the largest row length of either
    quadrature, as in Section 3.4). Tests pass other even lengths to check which of them give the
    same operator."""
    f = np.asarray(f, dtype=np.complex128)
    lead = f.shape[:-1]
    if nphi_all is None:
        nphi_all = max(int(q_src.nphi.max()), int(q_dst.nphi.max()))
    half = nphi_all // 2
    nt, nt2 = q_src.ntheta, q_dst.ntheta
    # step 1
    g1 = np.empty(lead + (q_src.nrows, nphi_all), dtype=np.complex128)
    for n in range(q_src.nrows):
        seg = f[..., q_src.row_off[n]:q_src.row_off[n + 1]]
        g1[..., n, :] = resample_1d(seg, nphi_all)
    # step 2
    circ = np.empty(lead + (half, nt), dtype=np.complex128)
    for t in range(nt):
        if t <= nt // 2:
            circ[..., :, t] = g1[..., t, :half]
        else:
            circ[..., :, t] = g1[..., nt - t, half:]
    # step 3
    circ2 = resample_1d(circ, nt2)
    # steps 4 and 5
    out = np.empty(lead + (q_dst.K,), dtype=np.complex128)
    for n in range(q_dst.nrows):
        row = np.concatenate([circ2[..., :, n], circ2[..., :, (nt2 - n) % nt2]], axis=-1)
        out[..., q_dst.row_off[n]:q_dst.row_off[n + 1]] = resample_1d(row, int(q_dst.nphi[n]))
    return out


def resample_sig_fourier_sym(f, q_src, q_dst, nphi_all=None):
    """The variant the paper mentions after the five steps (Section 3.4): use the symmetry of the
    Fourier coefficients, eqn. FourierSphereSym (f_{n,m} = (-1)^m f_{-n,m}), instead of the sample
    symmetry. Per phi column m < NPhi/2 the data split into u = (F_m + F_{m+NPhi/2})/2, which holds
    the even phi modes and is even in theta, and v = (F_m - F_{m+NPhi/2})/2, odd modes, odd in theta.
    Each is resampled in theta on the half range theta_0..theta_{N_theta/2} by the theta resample
    restricted to even or odd sequences; the destination rows are then F'_m = u' + v',
    F'_{m+NPhi/2} = u' - v'. Same steps 1 and 5 as resample_sig."""
    f = np.asarray(f, dtype=np.complex128)
    lead = f.shape[:-1]
    if nphi_all is None:
        nphi_all = max(int(q_src.nphi.max()), int(q_dst.nphi.max()))
    half = nphi_all // 2
    nt, nt2 = q_src.ntheta, q_dst.ntheta
    g1 = np.empty(lead + (q_src.nrows, nphi_all), dtype=np.complex128)
    for n in range(q_src.nrows):
        g1[..., n, :] = resample_1d(f[..., q_src.row_off[n]:q_src.row_off[n + 1]], nphi_all)
    u = 0.5 * (g1[..., :half] + g1[..., half:])      # [..., rows, half]
    v = 0.5 * (g1[..., :half] - g1[..., half:])
    # even / odd extension to the full theta circle, resample, keep rows 0..N'_theta/2
    t_idx = np.array([t if t <= nt // 2 else nt - t for t in range(nt)])
    sign = np.array([1.0 if t <= nt // 2 else -1.0 for t in range(nt)])
    ue = np.moveaxis(u[..., t_idx, :], -2, -1)                    # [..., half, nt]
    vo = np.moveaxis(v[..., t_idx, :] * sign[:, None], -2, -1)
    ur = resample_1d(ue, nt2)[..., : nt2 // 2 + 1]
    vr = resample_1d(vo, nt2)[..., : nt2 // 2 + 1]
    out = np.empty(lead + (q_dst.K,), dtype=np.complex128)
    for n in range(q_dst.nrows):
        row = np.concatenate([ur[..., :, n] + vr[..., :, n], ur[..., :, n] - vr[..., :, n]], axis=-1)
        out[..., q_dst.row_off[n]:q_dst.row_off[n + 1]] = resample_1d(row, int(q_dst.nphi[n]))
    return out
