"""Choice of the truncation ell and of the uniform quadrature (TEST INFRASTRUCTURE ONLY; see
oracle/__init__.py).

All selection is done in units of the box size (a_l = 1), so only the dimensionless wavenumber
ka = kappa a_l enters (Section 3.5.1 quotes its errors with box size a = 1). The representative
lengths are |r0| = 2 (the shortest transfer vector with one buffer box) and |r| = alpha sqrt(3)
(Section 3.3.3).

* ell (Section 2.1): the smallest ell whose Gegenbauer truncation error eps_G (eqn. eps_G),
  maximised over the angle between r and r0 on a 129-point grid of [0, pi], is below eps. This is
  the quantity the closed form eqn. CollinoError bounds; evaluating eps_G itself also stays valid
  for small |r| where that closed form does not.
* N_theta (Section 3.3.1, Alg. Ntheta, eqn. EpsITheta) with r, r0 along z.
* N_phi(theta_n) (Section 3.3.2, Alg. Nphi, eqn. EpsIPhi) with r, r0 along x; the smallest
  multiple of 4 that passes is taken, and rows theta_n, pi - theta_n get the larger of their two
  values so that the quadrature keeps the z = 0 reflection symmetry (Section 3.2).
"""
import numpy as np

from .special import sph_jn, sph_h1, legendre_table, bessel_jn_abs
from .fourier import coeffs_symmetric
from .transfer import bmtf

NGAMMA = 129


class LevelQuad:
    """One level's quadrature (Section 3.4): N_theta (even), rows n = 0..N_theta/2 at
    theta_n = 2 pi n / N_theta, row n holding N_phi(theta_n) (a multiple of 4) samples at
    phi_m = 2 pi m / N_phi(theta_n). Only half of the doubled sphere is stored (eqn. NumSphereSym)."""

    def __init__(self, ell, ntheta, nphi):
        self.ell = int(ell)
        self.ntheta = int(ntheta)
        self.nphi = np.asarray(nphi, dtype=np.int64)
        self.nrows = self.ntheta // 2 + 1
        assert self.ntheta % 2 == 0 and len(self.nphi) == self.nrows
        assert np.all(self.nphi % 4 == 0) and np.all(self.nphi >= 4)
        self.row_off = np.concatenate([[0], np.cumsum(self.nphi)]).astype(np.int64)
        self.K = int(self.row_off[-1])

    def row_theta(self):
        return 2.0 * np.pi * np.arange(self.nrows) / self.ntheta

    def angles(self):
        """(theta_k, phi_k) of every stored sample, row-major."""
        th = np.repeat(self.row_theta(), self.nphi)
        ph = np.concatenate([2.0 * np.pi * np.arange(m) / m for m in self.nphi])
        return th, ph

    def dirs(self):
        """Unit vectors s_k = [cos phi sin theta, sin phi sin theta, cos theta], [K, 3]."""
        th, ph = self.angles()
        st = np.sin(th)
        return np.stack([np.cos(ph) * st, np.sin(ph) * st, np.cos(th)], axis=-1)

    def weights(self):
        """Quadrature weights of eqn. eps_T, 4 pi^2 / (N_theta N_phi(theta_n)), folded onto the
        stored half: rows 0 < n < N_theta/2 stand for themselves and for row N_theta - n, so
        they count twice; the two pole rows count once."""
        w = 4.0 * np.pi ** 2 / (self.ntheta * self.nphi.astype(np.float64))
        mult = np.full(self.nrows, 2.0)
        mult[0] = 1.0
        mult[-1] = 1.0
        return np.repeat(w * mult, self.nphi)

    def __eq__(self, other):
        return (self.ell == other.ell and self.ntheta == other.ntheta
                and np.array_equal(self.nphi, other.nphi))

    def __repr__(self):
        return "LevelQuad(ell=%d, ntheta=%d, K=%d)" % (self.ell, self.ntheta, self.K)


def gegenbauer_error(ka, r, r0, ell_max, ngamma=NGAMMA):
    """max over gamma of |eps_G(ell)| for ell = 0..ell_max (eqn. eps_G), with |r| = r, |r0| = r0
    and cos(gamma) = rhat . r0hat on a uniform grid of [0, pi]. Box units, wavenumber ka."""
    gam = np.linspace(0.0, np.pi, ngamma)
    c = np.cos(gam)
    big_r = np.sqrt(r * r + r0 * r0 + 2.0 * r * r0 * c)
    exact = np.exp(1j * ka * big_r) / big_r
    n = np.arange(ell_max + 1)
    jn = sph_jn(ell_max, ka * r)
    hn = sph_h1(ell_max, ka * r0)
    P = legendre_table(ell_max, c)
    terms = (1j * ka * ((-1.0) ** n) * (2 * n + 1) * hn * jn)[:, None] * P
    partial = np.cumsum(terms, axis=0)
    return np.max(np.abs(exact[None, :] - partial), axis=1)


def ell_search_max(ka, r):
    """Upper end of the ell search: well beyond the excess-bandwidth formula (eqn. EBF)."""
    x = ka * r
    return int(np.ceil(x + 10.0 * max(x, 1.0) ** (1.0 / 3.0) + 40.0))


# Unit roundoff of the arithmetic the signatures are carried in.
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}
# The transfer-function part of the floor below is a coherent worst case; the oracle's measured
# breakdown at ka = pi in FP64 sits 5-8x under it, so a quarter of it is used.
FLOOR_SCALE = 0.25


def rounding_floor(ka, r0, ell_max, u):
    """Rounding floor of the low-frequency breakdown (Sections 2.1 and 3.5.1: for n > x the
    Hankel function diverges, the transfer function becomes huge and roundoff dominates), box
    units, for ell = 0..ell_max. Two parts:
    * evaluating T_ell (always in FP64) sums terms up to |c_n|, c_n = (i ka / 4 pi) i^n (2n+1) h_n;
      its error, integrated over the sphere, is at most u64 * ka * sum (2n+1) |h_n(ka |r0|)|
      (scaled by FLOOR_SCALE);
    * the signature arithmetic in the plan's precision u rounds every one of the ~(4/pi)(ell+1)^2
      quadrature terms independently; their random-walk sum is u * ka * sqrt(sum (2n+1) |h_n|^2 / K)
      (the L2 norm of T from the orthogonality of the P_n)."""
    n = np.arange(ell_max + 1)
    h = np.abs(sph_h1(ell_max, ka * r0))
    coherent = FLOOR_SCALE * UNIT_ROUNDOFF["fp64"] * ka * np.cumsum((2 * n + 1) * h)
    kq = (4.0 / np.pi) * (n + 1.0) ** 2
    walk = u * ka * np.sqrt(np.cumsum((2 * n + 1) * h * h) / kq)
    return coherent + walk


# Radius used to balance truncation against the rounding floor in the low-frequency breakdown:
# the box size, |r| = a (alpha = 1/sqrt(3), the value of Fig. GegError).
R_BREAKDOWN = 1.0


def select_ell(ka, r, r0, eps, u=UNIT_ROUNDOFF["fp64"]):
    """Section 2.1: the smallest ell whose predicted error max_gamma |eps_G(ell; r)| + rounding
    floor is below eps. If no ell reaches eps (low-frequency breakdown, Section 3.5.1), the
    achievable accuracy is set by roundoff: ell then minimises the truncation error at
    |r| = R_BREAKDOWN plus the floor. Returns (ell, predicted error)."""
    emax = ell_search_max(ka, r)
    floor = rounding_floor(ka, r0, emax, u)
    tot = gegenbauer_error(ka, r, r0, emax) + floor
    ok = np.nonzero(tot[1:] < eps)[0]
    if len(ok):
        ell = int(ok[0]) + 1
        return ell, float(tot[ell])
    low = gegenbauer_error(ka, min(r, R_BREAKDOWN), r0, emax) + floor
    ell = int(np.argmin(low[1:])) + 1
    return ell, float(low[ell])


def select_ntheta(ka, r, r0, ell, eps):
    """Alg. Ntheta (Section 3.3.1) with r0 = |r0| z: T^{s,L} sampled on N^max uniform theta
    points (N^max = 4 ell + 64), the magnitudes of its Fourier coefficients dotted with
    |J_{M(N_theta, n)}(ka |r|)| (eqn. EpsITheta); the first even N_theta >= 2 ell whose bound is
    below eps / 4 pi^2 is returned."""
    nmax = 4 * ell + 64
    th = 2.0 * np.pi * np.arange(nmax) / nmax
    vals = bmtf(ka, [0.0, 0.0, r0], ell, nmax, 1, theta_rows=th)[:, 0]
    coef = np.abs(np.fft.fft(vals) / nmax)
    j = np.arange(nmax)
    k = np.where(j <= nmax // 2, j, j - nmax)
    ak = np.abs(k)
    e = bessel_jn_abs(nmax, ka * r)
    tol = eps / (4.0 * np.pi ** 2)
    for nth in range(2 * ell, nmax + 1, 2):
        m = np.where(ak < nth // 2, nth - ak, ak)
        if np.sum(coef * e[m]) < tol:
            return nth
    return nmax


def select_nphi(ka, r, r0, ell, ntheta, eps):
    """Alg. Nphi (Section 3.3.2) with r0 = |r0| x: for every row theta_n, n = 0..N_theta/2, the
    phi-spectrum of T^{s,L} (2 ell + 1 samples) dotted with |J_{M(N_phi, m)}(ka |r| sin theta_n)|
    (eqn. EpsIPhi); the smallest multiple of 4 whose bound is below eps / 4 pi^2 is kept. Rows
    theta_n and pi - theta_n then take the larger of their two values."""
    nc = 2 * ell + 1
    tl = bmtf(ka, [r0, 0.0, 0.0], ell, ntheta, nc)
    coef = np.abs(coeffs_symmetric(tl))                    # [rows, m = -ell..ell]
    am = np.abs(np.arange(-ell, ell + 1))
    nphi_max = 4 * ((2 * ell + 2 + 64 + 3) // 4)
    tol = eps / (4.0 * np.pi ** 2)
    rows = ntheta // 2 + 1
    out = np.empty(rows, dtype=np.int64)
    for n in range(rows):
        st = abs(np.sin(2.0 * np.pi * n / ntheta))
        e = bessel_jn_abs(nphi_max, ka * r * st)
        out[n] = nphi_max
        for nphi in range(4, nphi_max + 1, 4):
            m = np.where(am < nphi // 2, nphi - am, am)
            if np.sum(coef[n] * e[m]) < tol:
                out[n] = nphi
                break
    return np.maximum(out, out[::-1])


# Above this box size in wavelength units (ka) the design radius widens to the box diagonal.
WIDE_KA = 100.0


def design_alpha(ka, alpha, eps, u=UNIT_ROUNDOFF["fp64"]):
    """The representative |r| = alpha sqrt(3) of Section 3.3.3 for one level. The paper's alpha
    (0.8) stands for the typical pair of interacting points; pairs near opposite corners reach
    |r| = sqrt(3). The truncation rule places ell just past ka|r| (Section 2.1), so for large ka
    an ell chosen at 0.8 sqrt(3) leaves those pairs short of it, and their error exceeds eps. So
    for ka > WIDE_KA the full diagonal (alpha = 1) is used whenever some ell reaches eps there;
    otherwise (and for alpha >= 1 as given) alpha is kept."""
    if not ka > WIDE_KA or alpha >= 1.0:
        return alpha
    r = np.sqrt(3.0)
    emax = ell_search_max(ka, r)
    tot = gegenbauer_error(ka, r, 2.0, emax) + rounding_floor(ka, 2.0, emax, u)
    return 1.0 if np.any(tot[1:] < eps) else alpha


def level_quadrature(ka, alpha, eps, ell=None, u=UNIT_ROUNDOFF["fp64"]):
    """Full parameter choice for one level in box units (Sections 2.1, 3.3):
    |r| = design_alpha(...) sqrt(3), |r0| = 2. Returns (LevelQuad, info dict with the predicted
    error and the design alpha)."""
    alpha = design_alpha(ka, alpha, eps, u)
    r = alpha * np.sqrt(3.0)
    r0 = 2.0
    if ell is None:
        ell, eg = select_ell(ka, r, r0, eps, u)
    else:
        eg = float(gegenbauer_error(ka, r, r0, ell)[ell] + rounding_floor(ka, r0, ell, u)[ell])
    nth = select_ntheta(ka, r, r0, ell, eps)
    nphi = select_nphi(ka, r, r0, ell, nth, eps)
    q = LevelQuad(ell, nth, nphi)
    return q, {"predicted": eg, "ka": ka, "alpha": alpha}
