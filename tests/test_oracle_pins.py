"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own arithmetic.

Each pin is chosen so that a plausible slip inside the oracle (a dropped
term, a wrong sign or index, a transposed operand, a wrong list) fails at
least one of them:

* paper counts (golden fixture, Sec. 2.1, 2.2, 4),
* derivative tensors against sympy's symbolic derivatives, the harmonic trace
  identity and the on-axis closed form,
* exact polynomial identities of P2M/M2M/L2L/L2P,
* convergence of M2L+L2P and M2P to the direct 1/r sum as p grows,
* the near/intermediate/far fields partitioning every source-target pair,
* the full solve against an O(N^2) direct sum, its cube symmetries,
  linearity, zero net force and closed-form Plummer / single-cell fields,
* the adjoint's dot-product identity, finite differences and the direct-sum
  gradient.
"""
import json
import math
import os

import numpy as np
import pytest

import fmm_inputs as fi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# --------------------------------------------------------------------------
# counts printed in the paper
# --------------------------------------------------------------------------
def test_paper_counts(orc):
    g = json.load(open(GOLDEN))
    assert orc.nterms(2) == g["multipole_terms_order2"]["value"]
    assert orc.nterms(3) == g["local_terms_order3"]["value"]
    assert 8 * orc.nterms(2) == g["multipole_terms_per_oct_order2"]["value"]
    # interior interaction lists have 6^3 - 3^3 members for every parity
    for k in (4, 5):
        for par in range(8):
            c = 6 + ((par >> 2) & 1), 6 + ((par >> 1) & 1), 6 + (par & 1)
            assert orc.list_size(k, *c) == g["list_octs"]["value"]
    # near field of an interior unigrid cell: 27 FMM cells x 8 unigrid cells
    n = 32
    u = (14 * n + 17) * n + 15
    row = orc.pair_pass_row(n, u)
    assert int((row == -1).sum()) == g["near_cells_delta1"]["value"]
    assert 27 - 1 == g["near_octs"]["value"]
    # a corner cell's list is clipped by the isolated boundary
    assert orc.list_size(4, 0, 0, 0) < 189


@pytest.mark.parametrize("n", [8, 16])
def test_fields_partition_every_pair(orc, n):
    """Near field + M2P list + M2L lists of all levels cover every source
    exactly once (Sec. 2.2: the fields partition the domain)."""
    F = int(math.log2(n)) - 1
    for u in range(n ** 3):
        row = orc.pair_pass_row(n, u)
        assert (row >= -1).all(), (u, np.unique(row))
        assert set(np.unique(row)) <= set([-1] + list(range(2, F + 1)))


def test_fields_partition_sampled_32(orc):
    n = 32
    rng = np.random.default_rng(7)
    for u in rng.choice(n ** 3, 48, replace=False):
        row = orc.pair_pass_row(n, int(u))
        assert (row >= -1).all()
        # at n = 32 all four passes occur for an interior target
    u = (15 * n + 16) * n + 17
    assert set(np.unique(orc.pair_pass_row(n, u))) == {-1, 2, 3, 4}


# --------------------------------------------------------------------------
# derivative tensors
# --------------------------------------------------------------------------
def test_dtensor_matches_sympy(orc):
    sp = pytest.importorskip("sympy")
    x, y, z = sp.symbols("x y z", real=True)
    f = -1 / sp.sqrt(x * x + y * y + z * z)
    P = 7
    pt = {x: sp.Rational(3, 7), y: sp.Rational(-5, 11), z: sp.Rational(2, 3)}
    R = np.array([3 / 7, -5 / 11, 2 / 3])
    mi = orc.multi_index(P)
    D = orc.dtensor(R, P)
    cache = {(0, 0, 0): f}

    def deriv(e):
        e = tuple(int(v) for v in e)
        if e in cache:
            return cache[e]
        for d, var in enumerate((x, y, z)):
            if e[d] > 0:
                lo = list(e)
                lo[d] -= 1
                cache[e] = sp.diff(deriv(lo), var)
                return cache[e]

    for t, e in enumerate(mi):
        exact = float(sp.N(deriv(e).subs(pt), 30))
        assert D[t] == pytest.approx(exact, rel=1e-12, abs=1e-12 * max(1.0, abs(exact))), tuple(e)


def test_dtensor_harmonic_trace(orc):
    """d^g(1/r) is harmonic: sum_i D[g + 2 e_i] = 0 for r > 0."""
    P = 9
    mi = orc.multi_index(P)
    index = {tuple(e): t for t, e in enumerate(mi)}
    rng = np.random.default_rng(3)
    for _ in range(5):
        R = rng.uniform(-2, 2, 3)
        D = orc.dtensor(R, P)
        scale = np.abs(D).max()
        for e in mi:
            if e.sum() + 2 > P:
                continue
            s = sum(D[index[tuple(e + 2 * np.eye(3, dtype=int)[i])]] for i in range(3))
            assert abs(s) < 1e-12 * scale


def test_dtensor_on_axis_closed_form(orc):
    """On the positive x axis d^n/dx^n (-1/x) = -(-1)^n n! / x^(n+1)."""
    P = 9
    mi = orc.multi_index(P)
    index = {tuple(e): t for t, e in enumerate(mi)}
    for xv in (0.37, 1.0, 2.75):
        for axis in range(3):
            R = np.zeros(3)
            R[axis] = xv
            D = orc.dtensor(R, P)
            for nn in range(P + 1):
                e = [0, 0, 0]
                e[axis] = nn
                want = -((-1) ** nn) * math.factorial(nn) / xv ** (nn + 1)
                assert D[index[tuple(e)]] == pytest.approx(want, rel=1e-13)


# --------------------------------------------------------------------------
# upward-pass identities
# --------------------------------------------------------------------------
def test_p2m_monopole_and_m2m_equals_p2m(orc):
    rng = np.random.default_rng(11)
    nmax = 6
    child_c = np.array([0.3, 0.55, 0.7])
    parent_c = child_c + np.array([0.0625, -0.0625, 0.0625])
    pos = child_c + rng.uniform(-0.06, 0.06, (20, 3))
    m = rng.uniform(0.1, 2.0, 20)
    Mc = orc.op_p2m(nmax, m, pos, child_c)
    assert Mc[0] == pytest.approx(m.sum(), rel=1e-15)
    shifted = orc.op_m2m(nmax, child_c - parent_c, Mc)
    direct = orc.op_p2m(nmax, m, pos, parent_c)
    assert rel(shifted, direct) < 1e-13


def test_origin_moments_then_shift_equals_centred(orc):
    """The paper accumulates moments about the origin and then shifts them to
    the cell centre with eq. (M2M) (Sec. 2.1); for the quadrupole order it
    uses this equals the centred moments the oracle forms directly."""
    rng = np.random.default_rng(12)
    c = np.array([0.40625, 0.59375, 0.84375])
    pos = c + rng.uniform(-1 / 64, 1 / 64, (8, 3))
    m = rng.uniform(0.5, 1.5, 8)
    M0 = orc.op_p2m(2, m, pos, np.zeros(3))
    shifted = orc.op_m2m(2, -c, M0)  # d = origin - centre
    assert rel(shifted, orc.op_p2m(2, m, pos, c)) < 1e-10


def test_l2l_is_exact_recentring(orc):
    rng = np.random.default_rng(13)
    p = 6
    Lp = rng.standard_normal(orc.nterms(p))
    a = np.array([0.03, -0.02, 0.05])
    Lc = orc.op_l2l(p, a, Lp)
    for _ in range(5):
        v = rng.uniform(-0.05, 0.05, 3)
        assert rel(orc.op_l2p(p, v - a, Lc), orc.op_l2p(p, v, Lp)) < 1e-12


def _cloud(rng, centre, half, k):
    return centre + rng.uniform(-half, half, (k, 3)), rng.uniform(0.2, 1.0, k)


def _direct_points(src, m, x):
    r = x - src
    d = np.linalg.norm(r, axis=1)
    return -(m / d).sum(), -(m[:, None] * r / d[:, None] ** 3).sum(0)


def test_m2l_l2p_converges_to_direct(orc):
    """Source cell of size h, target child cell of size h/2 at the closest
    list distance: M2L + L2P tends to the direct sum as p grows (and a wrong
    sign of R in eq. (M2L) would not)."""
    rng = np.random.default_rng(21)
    h = 0.125
    cs = np.array([0.5, 0.5, 0.5]) + 0.5 * h
    ct = cs + np.array([1.75, 0.25, -0.25]) * h  # R-hat of the nearest list member
    src, m = _cloud(rng, cs, 0.5 * h, 30)
    tgt = ct + rng.uniform(-0.25 * h, 0.25 * h, (10, 3))
    errs = []
    for p in range(1, 9):
        M = orc.op_p2m(p, m, src, cs)
        L = orc.op_m2l(p, p, ct - cs, M)
        e = []
        for x in tgt:
            phi_d, g_d = _direct_points(src, m, x)
            out = orc.op_l2p(p, x - ct, L)
            e.append(abs(out[0] - phi_d) / abs(phi_d))
        errs.append(max(e))
    assert errs[-1] < 2e-4
    assert all(errs[i + 2] < errs[i] for i in range(len(errs) - 2))


def test_m2p_converges_to_direct(orc):
    rng = np.random.default_rng(22)
    h = 1 / 64
    cs = np.array([0.25, 0.25, 0.25]) + 0.5 * h
    src, m = _cloud(rng, cs, 0.5 * h, 25)
    x = cs + np.array([2.25, -0.25, 0.25]) * h
    phi_d, g_d = _direct_points(src, m, x)
    errs = []
    for p in range(1, 9):
        out = orc.op_m2p(p, x - cs, orc.op_p2m(p, m, src, cs))
        errs.append((abs(out[0] - phi_d) / abs(phi_d), np.linalg.norm(out[1:] - g_d) / np.linalg.norm(g_d)))
    assert errs[-1][0] < 1e-5 and errs[-1][1] < 1e-4
    assert all(errs[i + 2][0] < errs[i][0] for i in range(len(errs) - 2))


# --------------------------------------------------------------------------
# full solve
# --------------------------------------------------------------------------
def _plummer(n, k=None, seed=None):
    if k is None:
        return fi.plummer_density(n, fi.single_plummer())
    return fi.plummer_density(n, fi.multi_plummer_params(k, seed))


@pytest.mark.parametrize("n", [8, 16, 32])
def test_solve_matches_direct_sum_and_improves_with_p(orc, n):
    rho = _plummer(n, 16, 100 + n)
    pd, gd = orc.direct(rho)
    errs = []
    for p in range(1, 9):
        phi, g = orc.solve(rho, p)
        errs.append((rel(phi, pd), rel(g, gd)))
    assert errs[5][0] < 1e-4 and errs[5][1] < 2e-3      # p = 6
    for i in range(len(errs) - 2):
        assert errs[i + 2][0] < errs[i][0] and errs[i + 2][1] < errs[i][1], errs


def test_single_massive_cell_closed_form(orc):
    """A single occupied cell: the discrete answer is exactly -m/|r| (and
    -m/dx at the cell itself); the FMM reaches it to its truncation error."""
    n = 32
    rho = np.zeros((n, n, n))
    c = (9, 20, 13)
    rho[c] = 5.0
    dx = 1 / n
    m = 5.0 * dx ** 3
    x = fi.cell_centres(n)
    r = np.stack(np.meshgrid(x - x[c[0]], x - x[c[1]], x - x[c[2]], indexing="ij"))
    d = np.sqrt((r ** 2).sum(0))
    d[c] = 1.0
    phi_exact = -m / d
    phi_exact[c] = -m / dx
    g_exact = -m * r / d ** 3
    g_exact[:, c[0], c[1], c[2]] = 0.0
    phi, g = orc.solve(rho, 6)
    assert rel(phi, phi_exact) < 1e-4
    assert rel(g, g_exact) < 1e-3
    assert phi[c] == pytest.approx(-m / dx, rel=1e-12)  # near field is exact


def test_linearity(orc):
    n = 16
    r1 = _plummer(n, 4, 1)
    r2 = np.random.default_rng(2).standard_normal((n, n, n))
    a, b = 0.7, -1.3
    p1, g1 = orc.solve(r1, 4)
    p2, g2 = orc.solve(r2, 4)
    p3, g3 = orc.solve(a * r1 + b * r2, 4)
    assert rel(p3, a * p1 + b * p2) < 1e-13
    assert rel(g3, a * g1 + b * g2) < 1e-13


def _cube_map(arr, perm, flips):
    out = np.transpose(arr, perm)
    for ax, f in enumerate(flips):
        if f:
            out = np.flip(out, ax)
    return out


@pytest.mark.parametrize("n", [8, 16])
def test_cube_symmetries(orc, n):
    """The oct hierarchy is invariant under the 48 symmetries of the cube, so
    transforming rho transforms phi as a scalar and g as a vector."""
    import itertools
    rho = np.random.default_rng(5).uniform(0, 1, (n, n, n))
    phi, g = orc.solve(rho, 4)
    syms = [(perm, flips) for perm in itertools.permutations(range(3))
            for flips in itertools.product((0, 1), repeat=3)]
    if n > 8:
        syms = syms[::7]
    for perm, flips in syms:
        phi_t, g_t = orc.solve(np.ascontiguousarray(_cube_map(rho, perm, flips)), 4)
        assert rel(phi_t, _cube_map(phi, perm, flips)) < 1e-13
        want = np.stack([(-1 if flips[j] else 1) * _cube_map(g[perm[j]], perm, flips) for j in range(3)])
        assert rel(g_t, want) < 1e-12, (perm, flips)


def test_net_force(orc):
    n = 16
    rho = _plummer(n, 8, 9)
    m = rho / n ** 3
    pd, gd = orc.direct(rho)
    tot = np.abs(m[None] * gd).sum()
    assert np.abs((m[None] * gd).sum(axis=(1, 2, 3))).max() / tot < 1e-13
    phi, g = orc.solve(rho, 6)
    # the FMM breaks action = reaction only at its truncation level
    assert np.abs((m[None] * g).sum(axis=(1, 2, 3))).max() / tot < 1e-4


def test_plummer_closed_form(orc):
    """One Plummer sphere (M = 1, a = 0.1, centred): discretisation-limited
    agreement with phi = -M/sqrt(r^2 + a^2), improving with resolution."""
    errs = []
    for n in (16, 32):
        rho = _plummer(n)
        x = fi.cell_centres(n) - 0.5
        r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
        phi_exact = -1.0 / np.sqrt(r2 + 0.01)
        phi, g = orc.solve(rho, 4)
        errs.append(rel(phi, phi_exact))
    assert errs[0] < 0.05 and errs[1] < errs[0]


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,p", [(8, 3), (16, 4), (16, 6)])
def test_adjoint_dot_product(orc, n, p):
    rng = np.random.default_rng(n + p)
    rho = rng.standard_normal((n, n, n))
    wphi = rng.standard_normal((n, n, n))
    wg = rng.standard_normal((3, n, n, n))
    phi, g = orc.solve(rho, p)
    lhs = (phi * wphi).sum() + (g * wg).sum()
    rhs = (rho * orc.adjoint(wphi, wg, p)).sum()
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(phi * wphi).sum() + np.abs(g * wg).sum())


def test_adjoint_finite_differences(orc):
    """Central differences of a quadratic loss are exact up to rounding."""
    n, p = 16, 4
    rho = _plummer(n, 6, 5001)
    phi_t, _ = orc.solve(_plummer(n, 6, 5002), p)
    phi, _ = orc.solve(rho, p)
    grad = orc.adjoint(2 * (phi - phi_t), None, p)
    eps = 1e-3 * rho.max()
    for c in fi.fd_cells(n, 6):
        idx = np.unravel_index(c, rho.shape)
        rp, rm = rho.copy(), rho.copy()
        rp[idx] += eps
        rm[idx] -= eps
        lp = ((orc.solve(rp, p)[0] - phi_t) ** 2).sum()
        lm = ((orc.solve(rm, p)[0] - phi_t) ** 2).sum()
        fd = (lp - lm) / (2 * eps)
        assert fd == pytest.approx(grad[idx], rel=1e-6, abs=1e-9 * abs(grad).max())


def test_adjoint_close_to_direct_sum_gradient(orc):
    """With the exact (symmetric) Green's matrix G the gradient of
    sum (phi - phi_t)^2 is 2 dx^3 G (phi - phi_t); the FMM adjoint agrees to
    its truncation error."""
    n, p = 16, 6
    rho = _plummer(n, 6, 5001)
    phi_t = orc.direct(_plummer(n, 6, 5002))[0]
    phi = orc.direct(rho)[0]
    grad_direct = 2 * orc.direct(phi - phi_t)[0]
    phi_f = orc.solve(rho, p)[0]
    grad_fmm = orc.adjoint(2 * (phi_f - phi_t), None, p)
    assert rel(grad_fmm, grad_direct) < 1e-4


# --------------------------------------------------------------------------
# multipoles truncated at nmax < p (Sec. 2.1: separate multipole and local
# orders; the paper's own pair is p = 3, nmax = 2)
# --------------------------------------------------------------------------
def test_truncated_multipoles_are_the_leading_terms(orc):
    """M2M only maps child terms of degree <= |a| to parent term a, so the
    multipoles kept at nmax are exactly the leading terms of the order-p
    multipoles at every level; the truncation drops, never alters."""
    n, p, nmax = 16, 5, 2
    rho = fi.plummer_density(n, fi.multi_plummer_params(6, 41))
    nt = (nmax + 1) * (nmax + 2) * (nmax + 3) // 6
    for level in (2, 3):
        full = orc.expansions(rho, p, "M", level)
        cut = orc.expansions(rho, p, "M", level, nmax=nmax)
        assert cut.shape[1] == nt
        assert rel(cut, full[:, :nt]) < 1e-14


def test_m2l_with_nmax_sums_only_the_kept_terms(orc):
    """eq. (M2L) with nmax < p is the order-p M2L of a multipole whose terms
    above nmax are zero."""
    rng = np.random.default_rng(43)
    p, nmax = 4, 2
    nt_p = (p + 1) * (p + 2) * (p + 3) // 6
    nt_m = (nmax + 1) * (nmax + 2) * (nmax + 3) // 6
    M = rng.standard_normal(nt_p)
    Mz = M.copy()
    Mz[nt_m:] = 0.0
    R = np.array([0.31, -0.27, 0.44])
    assert rel(orc.op_m2l(p, nmax, R, M[:nt_m]), orc.op_m2l(p, p, R, Mz)) < 1e-14
    # and dropping terms changes the result
    assert rel(orc.op_m2l(p, nmax, R, M[:nt_m]), orc.op_m2l(p, p, R, M)) > 1e-6
