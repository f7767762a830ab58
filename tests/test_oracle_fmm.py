"""Pins of the oracle's tree, direct sum and whole FMM (brute force, invariants, the definition)."""
import numpy as np
import pytest

from oracle import direct, tree as otree
from oracle.ffmm import Plan
from oracle.quadrature import level_quadrature
from oracle.resample import resample_sig, resample_sig_fourier_sym


def _cube(n, seed=0):
    return np.random.default_rng(seed).random((n, 3))


def _sphere(n, seed=0):
    g = np.random.default_rng(seed).standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _charges(n, seed=1):
    r = np.random.default_rng(seed)
    return r.standard_normal(n) + 1j * r.standard_normal(n)


# --- direct sum (the definition) ----------------------------------------------------------

def test_direct_two_points_closed_form():
    x = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.2]])
    q = np.array([1.0 + 2.0j, -0.5 + 0.25j])
    k = 5.0
    d = 1.3
    g = np.exp(1j * k * d) / d
    assert np.allclose(direct.matvec(x, q, k), [g * q[1], g * q[0]], rtol=1e-15)


def test_direct_brute_force_and_symmetry():
    x = _cube(60)
    x[7] = x[3]                      # a coincident pair is skipped
    q = _charges(60)
    k = 11.0
    r = np.linalg.norm(x[:, None] - x[None], axis=-1)
    a = np.where(r > 0, np.exp(1j * k * r) / np.where(r > 0, r, 1), 0)
    assert np.allclose(direct.matvec(x, q, k), a @ q, rtol=1e-13)
    assert np.allclose(a, a.T)
    sub = np.array([5, 7, 59])
    assert np.allclose(direct.matvec(x, q, k, targets=sub), (a @ q)[sub], rtol=1e-13)


def test_direct_gradient_finite_difference():
    x = _cube(40, seed=4)
    q = _charges(40, seed=5)
    k = 7.0
    f = direct.gradient(x, q, k)
    h = 1e-6
    for i in (0, 17):
        for a in range(3):
            xp = x.copy(); xp[i, a] += h
            xm = x.copy(); xm[i, a] -= h
            fd = (direct.matvec(xp, q, k, targets=[i]) - direct.matvec(xm, q, k, targets=[i])) / (2 * h)
            assert abs(fd[0] - f[i, a]) < 1e-6 * abs(f[i, a]) + 1e-7


# --- octree -------------------------------------------------------------------------------

def test_morton_small_example():
    idx = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 2, 1], [5, 6, 7]])
    keys = otree.morton(idx, 3)
    assert list(keys[:3]) == [1, 2, 4]
    # x=011, y=010, z=001 -> bits (b0: x1 y0 z1)(b1: x1 y1 z0)(b2: 0 0 0)
    assert keys[3] == 0b000_011_101
    assert np.array_equal(otree.demorton(keys, 3), idx)


def test_quantize_and_stable_sort():
    x = np.array([[0.0, 0, 0], [1.0, 1, 1], [0.5, 0.5, 0.5], [0.0, 0, 0], [0.99999, 0.2, 0.7]])
    t = otree.Tree(x, depth=2)
    assert np.array_equal(t.idx[1], [3, 3, 3])           # the max corner is clamped
    assert np.array_equal(t.idx[2], [2, 2, 2])
    assert t.perm[0] == 0 and t.perm[1] == 3              # ties keep the input order


def test_interaction_list_counts_dense_grid():
    """Section 3.2: 316 distinct transfer vectors per level; a box has at most 189 interaction
    boxes and at most 27 neighbours (itself included)."""
    g = (np.stack(np.meshgrid(*[np.arange(16)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / 16
    t = otree.Tree(g, depth=4)
    offs = set()
    for l in (3, 4):
        (ptr, _), codes = t.ilist[l], t.ioff[l]
        assert np.diff(ptr).max() == 189
        offs |= set(codes.tolist())
        nptr, _ = t.neighbors[l]
        assert np.diff(nptr).max() == 27
    assert len(offs) == 316
    semi = [d for d in (np.array([c % 7 - 3, (c // 7) % 7 - 3, c // 49 - 3]) for c in offs)
            if d[0] >= 0 and d[1] >= 0 and d[2] >= 0 and d[0] >= d[1]]
    assert len(semi) == 34


def test_interaction_list_definition_brute_force():
    x = _sphere(700, seed=2)
    t = otree.Tree(x, depth=4)
    for l in (2, 3, 4):
        lev, par = t.levels[l], t.levels[l - 1]
        (ptr, src), codes = t.ilist[l], t.ioff[l]
        for b in range(lev.n):
            want = []
            for c in range(lev.n):
                near = np.max(np.abs(lev.ijk[c] - lev.ijk[b])) <= 1
                pnear = np.max(np.abs(par.ijk[t.parent[l][c]] - par.ijk[t.parent[l][b]])) <= 1
                if pnear and not near:
                    want.append(c)
            assert list(src[ptr[b]:ptr[b + 1]]) == want
            d = lev.ijk[src[ptr[b]:ptr[b + 1]]] - lev.ijk[b]
            assert np.array_equal(codes[ptr[b]:ptr[b + 1]], otree.offset_code(d))


def test_every_pair_counted_once():
    """The near field (leaf neighbours) and the interaction lists of all levels together cover
    every ordered pair of distinct boxes exactly once (Section 2)."""
    x = _cube(600, seed=9)
    t = otree.Tree(x, depth=4)
    L = t.depth
    leaf = t.levels[L]
    cover = np.zeros((leaf.n, leaf.n), dtype=int)
    nptr, nb = t.neighbors[L]
    for b in range(leaf.n):
        cover[b, nb[nptr[b]:nptr[b + 1]]] += 1
    anc = {L: np.arange(leaf.n)}
    for l in range(L, 2, -1):
        anc[l - 1] = t.parent[l][anc[l]]
    for l in range(2, L + 1):
        (ptr, src), _ = t.ilist[l], t.ioff[l]
        for b in range(leaf.n):
            B = anc[l][b]
            s = set(src[ptr[B]:ptr[B + 1]].tolist())
            cover[b] += np.isin(anc[l], list(s)).astype(int)
    assert np.all(cover == 1)


# --- symmetric transfer storage (Fig. SemiOctant) ---------------------------------------------

def _sym_index(g, n, m, q):
    """Direction index of g^{-1}(s) for s = (theta_n, phi_m) on quadrature q; g = swap x <-> y
    (bit 0) then reflections of x, y, z (bits 1-3), so g^{-1} reflects first and swaps last."""
    npn = int(q.nphi[n])
    if g & 8:
        n = q.ntheta // 2 - n
    if g & 2:
        m = npn // 2 - m
    if g & 4:
        m = -m
    if g & 1:
        m = npn // 4 - m
    return int(q.row_off[n]) + m % npn


def test_transfer_symmetry_34_representatives():
    """The 316 transfer vectors fall into 34 classes under the quadrature's symmetries (x <-> y,
    reflections of x, y, z: 16 maps), and T_{g r0}(s) = T_{r0}(g^{-1} s) on the grid, so 34 tables
    and a direction permutation give all 316. Checked on the oracle's own tables."""
    from oracle.transfer import transfer_table
    ka = 6.0
    q, _ = level_quadrature(ka, 0.8, 1e-8)
    reps = {}
    for code in range(343):
        d = np.array([code % 7 - 3, (code // 7) % 7 - 3, code // 49 - 3])
        if np.max(np.abs(d)) <= 1:
            continue
        ax, ay, az = np.abs(d)
        key = (max(ax, ay), min(ax, ay), az)
        g = (1 if ax < ay else 0) | (2 if d[0] < 0 else 0) | (4 if d[1] < 0 else 0) | (8 if d[2] < 0 else 0)
        reps.setdefault(key, []).append((d, g))
    assert len(reps) == 34 and sum(len(v) for v in reps.values()) == 316
    rng = np.random.default_rng(0)
    keys = sorted(reps)
    for key in [keys[i] for i in rng.choice(34, 8, replace=False)] + [(3, 3, 3), (2, 0, 0)]:
        t_rep = transfer_table(ka / 1.0, np.array(key, dtype=float), q)
        for d, g in reps[key]:
            t = transfer_table(ka, d.astype(float), q)
            perm = np.array([_sym_index(g, n, m, q) for n in range(q.nrows) for m in range(int(q.nphi[n]))])
            assert np.max(np.abs(t - t_rep[perm])) < 1e-12 * np.max(np.abs(t)), (key, tuple(d), g)


# --- five-step resample ---------------------------------------------------------------------

@pytest.mark.parametrize("ka_pair", [(2.0, 4.0), (4.0, 2.0), (7.5, 15.0), (15.0, 7.5)])
def test_five_step_common_length_min_equals_max(ka_pair):
    """The common phi length may be the smaller of the two largest row lengths: upward the source
    rows already fit on it, downward the destination rows keep no mode it lacks, and the theta
    step acts on each phi mode separately (the mirror multiplies mode p by (-1)^p). So the
    five-step operator with NPhi = min equals the one with NPhi = max on data with the symmetry of
    the doubled sphere (eqn. NumSphereSym), i.e. on every signature: the rows theta = 0 and
    theta = pi are their own mirror images, so F(theta, phi) = F(theta, phi + pi) there."""
    q1, _ = level_quadrature(ka_pair[0], 0.8, 1e-6)
    q2, _ = level_quadrature(ka_pair[1], 0.8, 1e-6)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2, q1.K)) + 1j * rng.standard_normal((2, q1.K))
    for n in (0, q1.nrows - 1):   # project the self-mirrored rows onto pi-periodic data
        a, b = q1.row_off[n], q1.row_off[n + 1]
        row = f[:, a:b]
        f[:, a:b] = 0.5 * (row + np.roll(row, (b - a) // 2, axis=-1))
    n_lo = min(int(q1.nphi.max()), int(q2.nphi.max()))
    n_hi = max(int(q1.nphi.max()), int(q2.nphi.max()))
    assert n_lo < n_hi
    ref = resample_sig(f, q1, q2)
    got = resample_sig(f, q1, q2, nphi_all=n_lo)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # a common length below both maxima drops modes the destination keeps
    bad = resample_sig(f, q1, q2, nphi_all=n_lo - 8)
    assert np.max(np.abs(bad - ref)) > 1e-3 * np.max(np.abs(ref))


def test_five_step_resample_plane_wave():
    """Section 3.4: a plane wave e^{i ka s.d} with small |d| is band-limited well below both
    grids, so the five steps reproduce its samples on the other quadrature."""
    q1, _ = level_quadrature(6.0, 1 / np.sqrt(3), 1e-10)
    q2, _ = level_quadrature(12.0, 1 / np.sqrt(3), 1e-10)
    d = np.array([0.3, -0.2, 0.25])
    f1 = np.exp(1j * 6.0 * q1.dirs() @ d)
    f2 = np.exp(1j * 6.0 * q2.dirs() @ d)
    assert np.allclose(resample_sig(f1, q1, q2), f2, atol=1e-10)
    assert np.allclose(resample_sig(f2, q2, q1), f1, atol=1e-10)


@pytest.mark.parametrize("ka_pair", [(2.0, 4.0), (4.0, 2.0), (7.5, 15.0), (15.0, 7.5)])
def test_fourier_sym_variant_equals_five_steps(ka_pair):
    """The variant built on eqn. FourierSphereSym (even/odd theta parts of the phi columns, each
    resampled on the half range) gives the five-step result on data with the sphere symmetry,
    with the smaller common phi length too."""
    q1, _ = level_quadrature(ka_pair[0], 0.8, 1e-6)
    q2, _ = level_quadrature(ka_pair[1], 0.8, 1e-6)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((2, q1.K)) + 1j * rng.standard_normal((2, q1.K))
    for n in (0, q1.nrows - 1):
        a, b = q1.row_off[n], q1.row_off[n + 1]
        f[:, a:b] = 0.5 * (f[:, a:b] + np.roll(f[:, a:b], (b - a) // 2, axis=-1))
    ref = resample_sig(f, q1, q2)
    for na in (None, min(int(q1.nphi.max()), int(q2.nphi.max()))):
        got = resample_sig_fourier_sym(f, q1, q2, nphi_all=na)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), na


def test_five_step_resample_uniform_rows_roundtrip():
    """With every row of equal length the five steps are tensor-product Fourier resamples, so
    interpolating up and anterpolating back is the identity (Section 3.1.3)."""
    from oracle.quadrature import LevelQuad
    q1 = LevelQuad(5, 12, [12] * 7)
    q2 = LevelQuad(9, 20, [20] * 11)
    # data with the spherical symmetry and a band inside the coarse grid
    d = np.array([0.2, 0.1, -0.3])
    g = np.exp(1j * 2.0 * q1.dirs() @ d) + 0.5 * q1.dirs()[:, 2] ** 2
    back = resample_sig(resample_sig(g, q1, q2), q2, q1)
    assert np.allclose(back, resample_sig(g, q1, q1), atol=1e-13)


# --- whole matvec -----------------------------------------------------------------------------

def test_fmm_cube_fp64_meets_eps():
    """Volumetric workload (N = 4096 in the unit cube, kappa = 8 pi, depth 3, eps 1e-6)
    against the full direct sum."""
    x = _cube(4096)
    q = _charges(4096)
    k = 8 * np.pi
    p = Plan(x, k, 1e-6, depth=3)
    out = p.matvec(q)
    ref = direct.matvec(x, q, k)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-6


def test_fmm_error_falls_with_eps():
    x = _sphere(3000)
    q = _charges(3000)
    k = 30.0
    ref = direct.matvec(x, q, k)
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        out = Plan(x, k, eps, depth=4).matvec(q)
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-4 and errs[2] < 1e-6


def test_fmm_multilevel_matches_single_level():
    """Adding levels (more M2M/L2L passes) leaves the result within eps of the direct sum."""
    x = _cube(1500, seed=3)
    q = _charges(1500, seed=4)
    k = 12.0
    ref = direct.matvec(x, q, k)
    for depth in (2, 3, 4):
        out = Plan(x, k, 1e-5, depth=depth).matvec(q)
        assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-5, depth


# --- multilevel accuracy with two points (Section 3.5.2) ----------------------------------------

def _two_point_plan(kappa, xj, xi, depth, **kw):
    """Plan over a source point x_j (charge 1) and a target x_i (charge 0) in level-2 boxes of side
    1 whose centres differ by r0 = (2, 0, 0) (one buffer box), with two uncharged points fixing
    the root cube to [0, 4]^3. The pair meets only through the level-2 transfer pass; the
    transfer functions of every other offset (which only carry zero charges here) are left zero,
    so only T_{(-2,0,0)} at level 2 is built. Returns the plan and phi_i."""
    from oracle.transfer import transfer_table
    frame = np.array([[0.0, 0.0, 0.5], [4.0, 4.0, 4.0]])
    x = np.vstack([xj, xi, frame])
    p = Plan(x, kappa, kw.pop("eps", None), depth=depth, **kw)
    for l in range(2, depth + 1):
        p._tables[l] = np.zeros((343, p.quads[l].K), dtype=np.complex128)
    code = (-2 + 3) + 7 * 3 + 49 * 3        # source minus target = (-2, 0, 0) box sides
    p._tables[2][code] = transfer_table(kappa, np.array([-2.0, 0.0, 0.0]), p.quads[2])
    return p, p.matvec(np.array([1.0, 0.0, 0.0, 0.0], dtype=np.complex128))[1]


def _gegenbauer_value(kappa, r, r0, ell):
    """The truncated addition theorem (Section 2.1, eqn. eps_G's series) for r and r0."""
    from oracle import special as osp
    n = np.arange(ell + 1)
    cg = float(r @ r0) / (np.linalg.norm(r) * np.linalg.norm(r0))
    P = osp.legendre_table(ell, np.array([cg]))[:, 0]
    jn = osp.sph_jn(ell, kappa * np.linalg.norm(r))
    hn = osp.sph_h1(ell, kappa * np.linalg.norm(r0))
    return complex(np.sum(1j * kappa * ((-1.0) ** n) * (2 * n + 1) * hn * jn * P))


def test_multilevel_interpolation_error_independent_of_depth():
    """Fig. Error_Quad (Section 3.5.2): two points at opposite corners of their level-2 boxes
    (|r| = sqrt(3)), kappa = 100, alpha = 0.8, a_2 = 1, transfer at level 2 and L = 2..8 levels in
    all. eps_G^L is one series for every L; eps_I^L = phi^L - series differs from eps_I^2 (one
    level, no interpolation) by far less than the target: the up- and downward passes add almost
    nothing. A wrong translation, resample or level chain makes the L > 2 results drift."""
    kappa, dd = 100.0, 1e-9
    xj = np.array([dd, dd, dd])
    xi = np.array([3.0 - dd, 1.0 - dd, 1.0 - dd])
    rr = (xi - np.array([2.5, 0.5, 0.5])) - (xj - np.array([0.5, 0.5, 0.5]))
    exact = np.exp(1j * kappa * np.linalg.norm(xi - xj)) / np.linalg.norm(xi - xj)
    for eps in (1e-3, 1e-6):
        ei = {}
        for L in (2, 3, 5, 8):
            p, phi = _two_point_plan(kappa, xj, xi, L, eps=eps, alpha=0.8, eps_safety=1.0)
            series = _gegenbauer_value(kappa, rr, np.array([2.0, 0.0, 0.0]), p.quads[2].ell)
            ei[L] = phi - series
            assert abs(abs(phi - exact) - abs(ei[2] + series - exact)) < 0.01 * eps
        drift = max(abs(ei[L] - ei[2]) for L in (3, 5, 8))
        assert drift < 0.01 * eps, (eps, drift)


def test_quadrature_converges_to_gegenbauer_error():
    """Fig. GegError_Quad (Section 3.5.2): kappa = 100, alpha = 1/sqrt(3), a_2 = 1, two active
    levels (the transfer at level 2, interpolation and anterpolation to level 3). With ell held
    where the Gegenbauer error of the design radius |r| = 1 is 1e-6 or 1e-10, and the quadrature
    grown by lowering its own target, the total error becomes the truncation error: eps_T ->
    eps_G. The level-2 quadrature sizes fall in the figure's range (14 000 .. 28 000)."""
    from oracle.quadrature import level_quadrature, gegenbauer_error
    kappa = 100.0
    h = 0.5 / np.sqrt(3.0)
    xj = np.full(3, 0.5 - h)
    xi = np.array([2.5 + h, 0.5 + h, 0.5 + h])
    rr = (xi - np.array([2.5, 0.5, 0.5])) - (xj - np.array([0.5, 0.5, 0.5]))   # |r| = 1
    exact = np.exp(1j * kappa * np.linalg.norm(xi - xj)) / np.linalg.norm(xi - xj)
    geg = gegenbauer_error(kappa * 1.0, 1.0, 2.0, 200)
    alpha = 1.0 / np.sqrt(3.0)
    for target in (1e-6, 1e-10):
        ell = int(np.nonzero(geg[1:] < target)[0][0]) + 1
        eg = abs(_gegenbauer_value(kappa, rr, np.array([2.0, 0.0, 0.0]), ell) - exact)
        gap = []
        for eps_q in (1e-2, 1e-6, 1e-12):
            q2, _ = level_quadrature(kappa, alpha, eps_q, ell=ell)
            q3, _ = level_quadrature(kappa / 2.0, alpha, eps_q)
            assert 14000 <= q2.K <= 28000
            _, phi = _two_point_plan(kappa, xj, xi, 3, alpha=alpha, quads={2: q2, 3: q3})
            gap.append(abs(abs(phi - exact) - eg) / eg)
        assert gap[-1] < 0.05 and gap[0] > 10.0 * gap[-1], (target, gap)
