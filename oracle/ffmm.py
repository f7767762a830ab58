"""The multilevel Fourier-basis FMM matvec, stage by stage, in FP64
(TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

It approximates sigma_i = sum_{j != i} e^{i kappa |x_i - x_j|} / |x_i - x_j| psi_j
(eqn. HelmholtzMatrixVector) by the steps of Section 2, with the Fourier-basis quadrature,
the band-limited modified transfer function and the FFT inter/anterpolation of Section 3:

* P2M (Initialization):  M^L_a(s) = sum_{x_i in B_a} psi_i e^{i kappa s.(x_i - c_a)}
* M2M (Upward pass):      M^{l-1}_a = sum_children R_{l->l-1}(M^l_b) e^{i kappa s.(c_b - c_a)},
                          l = L..3; the child signature is first resampled to the parent grid
                          (Section 3.4) and translated there.
* M2L (Transfer pass):    I^l_a = sum_{b in I(B_a)} M^l_b T^{s,LL}_{c_b - c_a}, l = L..2.
* L2L (Downward pass):    L^{l+1}_a = R_{l->l+1}(L^l_b e^{i kappa s.(c_b - c_a)}) + I^{l+1}_a, with
                          L^2 = I^2; the translation is applied on the parent grid and the result
                          anterpolated to the child grid (Section 3.1.3).
* L2P + P2P (eqn. FMM_FinalStep): sigma_i = sum_k w_k L^L_a(s_k) e^{i kappa s_k.(c_a - x_i)} +
                          sum over the neighbour list, j != i.

Readings: pairs at distance exactly 0 are skipped like j = i; the signatures and T^{s,LL} hold
function values and the quadrature weights (eqn. eps_T) are applied once, in L2P.

Levels use parameters chosen in box units (oracle/quadrature.py) with ka_l = kappa a_l,
|r| = alpha sqrt(3) a_l and |r0| = 2 a_l, or integer parameters given by the caller.
"""
import numpy as np

from .tree import Tree, OCT8, auto_depth
from .quadrature import level_quadrature, select_ell, UNIT_ROUNDOFF
from .transfer import transfer_table
from .resample import resample_sig

ALPHA_DEFAULT = 0.8
EPS_SAFETY_DEFAULT = 0.1


def leaf_feasible(kappa, a_leaf, alpha, eps, u):
    """Whether the leaf level can reach eps at all: the smallest predicted error (truncation +
    rounding floor) over ell must be below eps (Section 3.5.1, low-frequency breakdown)."""
    _, pred = select_ell(kappa * a_leaf, alpha * np.sqrt(3.0), 2.0, 0.0, u)
    return pred < eps


def kernel(kappa, r):
    """e^{i kappa r} / r (eqn. HelmholtzMatrixVector)."""
    return np.exp(1j * kappa * r) / r


class Plan:
    """Tree, per-level quadratures and tables for one point set."""

    def __init__(self, x, kappa, eps, depth=None, max_leaf=64, alpha=ALPHA_DEFAULT,
                 quads=None, eps_levels=None, precision="fp64", eps_safety=EPS_SAFETY_DEFAULT):
        """Parameters per level l = 2..depth: ka_l = kappa a_l; ell, N_theta, N_phi chosen for
        eps_int = eps_safety * eps with the rounding floor of ``precision``. With depth=None the
        depth is the smallest one whose leaves hold <= max_leaf points, reduced while the leaf
        level cannot reach eps (low-frequency breakdown)."""
        self.kappa = float(kappa)
        self.precision = precision
        u = UNIT_ROUNDOFF[precision]
        x = np.ascontiguousarray(x, dtype=np.float64)
        if depth is None:
            depth = auto_depth(x, max_leaf)
            lo = x.min(axis=0)
            side = float((x.max(axis=0) - lo).max()) or 1.0
            while depth > 2 and eps is not None and not leaf_feasible(
                    self.kappa, side / 2 ** depth, alpha, eps, u):
                depth -= 1
        self.tree = Tree(x, depth=depth, max_leaf=max_leaf)
        self.depth = self.tree.depth
        self.alpha = alpha
        self.quads = {}
        self.predicted = {}
        for l in range(2, self.depth + 1):
            if quads is not None:
                self.quads[l] = quads[l]
            else:
                e = eps * eps_safety if eps_levels is None else eps_levels[l]
                ka = self.kappa * self.tree.levels[l].a
                self.quads[l], info = level_quadrature(ka, alpha, e, u=u)
                self.predicted[l] = info["predicted"]
        self._tables = {}

    # --- precompute ------------------------------------------------------------------------
    def table(self, l):
        """T^{s,LL} for all 343 offset codes of level l (rows of inner codes are zero)."""
        if l not in self._tables:
            q = self.quads[l]
            a = self.tree.levels[l].a
            tab = np.zeros((343, q.K), dtype=np.complex128)
            for code in range(343):
                d = np.array([code % 7 - 3, (code // 7) % 7 - 3, code // 49 - 3])
                if np.max(np.abs(d)) <= 1:
                    continue
                tab[code] = transfer_table(self.kappa, d * a, q)
            self._tables[l] = tab
        return self._tables[l]

    def translation(self, l_grid, l_child, sign=1.0):
        """e^{i sign kappa s.(c_child - c_parent)} on the level-l_grid quadrature for the 8
        octants; c_child - c_parent = (oct - 1/2) a_{l_child}. Returns [8, K]."""
        s = self.quads[l_grid].dirs()
        d = (OCT8 - 0.5) * self.tree.levels[l_child].a
        return np.exp(1j * sign * self.kappa * (d @ s.T))

    # --- stages ----------------------------------------------------------------------------
    def p2m(self, q_sorted):
        """Initialization (Section 2) at the leaf level. q_sorted [N] in tree order."""
        t = self.tree
        L = self.depth
        lev = t.levels[L]
        s = self.quads[L].dirs()
        M = np.zeros((lev.n, self.quads[L].K), dtype=np.complex128)
        for b0 in range(0, lev.n, 512):
            b1 = min(lev.n, b0 + 512)
            p0, p1 = t.leaf_start[b0], t.leaf_start[b1 - 1] + t.leaf_count[b1 - 1]
            rel = t.xs[p0:p1] - lev.centers[t.point_box[p0:p1]]
            ph = np.exp(1j * self.kappa * (rel @ s.T)) * q_sorted[p0:p1, None]
            M[b0:b1] = np.add.reduceat(ph, t.leaf_start[b0:b1] - p0, axis=0)
        return M

    def m2m(self, M_leaf):
        """Upward pass (Section 2, Section 3.4). Returns {l: M^l}."""
        t = self.tree
        M = {self.depth: M_leaf}
        for l in range(self.depth, 2, -1):
            par = t.parent[l]
            oct_ = t.levels[l].ijk - 2 * t.levels[l - 1].ijk[par]
            code = oct_[:, 0] + 2 * oct_[:, 1] + 4 * oct_[:, 2]
            E = self.translation(l - 1, l, +1.0)
            R = resample_sig(M[l], self.quads[l], self.quads[l - 1]) * E[code]
            P = np.zeros((t.levels[l - 1].n, self.quads[l - 1].K), dtype=np.complex128)
            np.add.at(P, par, R)
            M[l - 1] = P
        return M

    def m2l(self, M):
        """Transfer pass (Section 2). Returns {l: I^l}."""
        t = self.tree
        I = {}
        for l in range(2, self.depth + 1):
            tab = self.table(l)
            (ptr, src), off = t.ilist[l], t.ioff[l]
            out = np.zeros_like(M[l])
            for b in range(t.levels[l].n):
                sl = slice(ptr[b], ptr[b + 1])
                if ptr[b + 1] > ptr[b]:
                    out[b] = np.sum(M[l][src[sl]] * tab[off[sl]], axis=0)
            I[l] = out
        return I

    def l2l(self, I):
        """Downward pass (Section 2, Section 3.4). Returns {l: L^l}."""
        t = self.tree
        Lf = {2: I[2]}
        for l in range(2, self.depth):
            par = t.parent[l + 1]
            oct_ = t.levels[l + 1].ijk - 2 * t.levels[l].ijk[par]
            code = oct_[:, 0] + 2 * oct_[:, 1] + 4 * oct_[:, 2]
            E = self.translation(l, l + 1, -1.0)
            Lf[l + 1] = resample_sig(Lf[l][par] * E[code], self.quads[l], self.quads[l + 1]) + I[l + 1]
        return Lf

    def l2p(self, L_leaf):
        """Far part of eqn. FMM_FinalStep. Returns [N] in tree order."""
        t = self.tree
        lev = t.levels[self.depth]
        qd = self.quads[self.depth]
        s = qd.dirs()
        w = qd.weights()
        out = np.zeros(t.n, dtype=np.complex128)
        for p0 in range(0, t.n, 4096):
            p1 = min(t.n, p0 + 4096)
            box = t.point_box[p0:p1]
            rel = lev.centers[box] - t.xs[p0:p1]
            ph = np.exp(1j * self.kappa * (rel @ s.T))
            out[p0:p1] = np.sum(ph * (L_leaf[box] * w[None, :]), axis=1)
        return out

    def p2p(self, q_sorted):
        """Near part of eqn. FMM_FinalStep: sources in N(B), j != i, R = 0 skipped."""
        t = self.tree
        ptr, nb = t.neighbors[self.depth]
        out = np.zeros(t.n, dtype=np.complex128)
        for b in range(t.levels[self.depth].n):
            i0, i1 = t.leaf_start[b], t.leaf_start[b] + t.leaf_count[b]
            js = np.concatenate([np.arange(t.leaf_start[c], t.leaf_start[c] + t.leaf_count[c])
                                 for c in nb[ptr[b]:ptr[b + 1]]])
            d = t.xs[i0:i1, None, :] - t.xs[None, js, :]
            r = np.sqrt(np.sum(d * d, axis=-1))
            ok = r > 0.0
            g = np.where(ok, np.exp(1j * self.kappa * r) / np.where(ok, r, 1.0), 0.0)
            out[i0:i1] = g @ q_sorted[js]
        return out

    # --- whole matvec ----------------------------------------------------------------------
    def stages(self, q):
        """All intermediates for one right-hand side q [N] (user order)."""
        qs = np.asarray(q, dtype=np.complex128)[self.tree.perm]
        M = self.m2m(self.p2m(qs))
        I = self.m2l(M)
        Lf = self.l2l(I)
        far = self.l2p(Lf[self.depth])
        near = self.p2p(qs)
        return {"M": M, "I": I, "L": Lf, "far": far, "near": near}

    def matvec(self, q):
        """sigma = A q in user order. q [N] or [nrhs, N]."""
        q = np.asarray(q)
        if q.ndim == 2:
            return np.stack([self.matvec(r) for r in q])
        st = self.stages(q)
        out = np.empty(self.tree.n, dtype=np.complex128)
        out[self.tree.perm] = st["far"] + st["near"]
        return out
