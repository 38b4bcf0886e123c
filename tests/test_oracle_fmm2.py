"""Pins of the oracle's FMM-2 (finest FMM level two levels above the unigrid,
App. A) against facts fixed by the paper and by mathematics:

* the near field of a unigrid cell is the 27 x 64 cells of the adjacent
  finest FMM cells (Sec. 4, golden count), and near field + M2P list + M2L
  lists still cover every source exactly once (Sec. 2.2);
* a density confined to one finest FMM cell reaches every target in it and in
  its neighbours through the near field alone, so there the solve equals the
  O(N^2) direct sum to rounding;
* the full solve converges to the direct sum as p grows, and keeps the cube
  symmetries and a single cell's closed form;
* FMM-1 and FMM-2 potentials of a point charge at the box centre (deposited
  by cloud-in-cell on its 8 surrounding cells) differ by less than 0.3 %
  (App. A).
"""
import itertools
import json
import os

import numpy as np
import pytest

import fmm_inputs as fi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_near_field_count_delta2(orc):
    g = json.load(open(GOLDEN))
    n = 64
    u = (29 * n + 34) * n + 30
    row = orc.pair_pass_row(n, u, delta_l=2)
    assert int((row == -1).sum()) == g["near_cells_delta2"]["value"]
    # the M2P list of an interior finest cell holds 189 cells of 64 sources
    assert int((row == 4).sum()) == g["list_octs"]["value"] * 64


def test_fields_partition_every_pair_delta2(orc):
    n = 16
    for u in range(n ** 3):
        row = orc.pair_pass_row(n, u, delta_l=2)
        assert (row >= -1).all(), (u, np.unique(row))
        assert set(np.unique(row)) <= {-1, 2}


def test_fields_partition_sampled_delta2_64(orc):
    n = 64
    rng = np.random.default_rng(11)
    for u in rng.choice(n ** 3, 16, replace=False):
        assert (orc.pair_pass_row(n, int(u), delta_l=2) >= -1).all()
    u = (31 * n + 32) * n + 33
    assert set(np.unique(orc.pair_pass_row(n, u, delta_l=2))) == {-1, 2, 3, 4}


def test_near_field_alone_is_the_direct_sum(orc):
    """Mass in one finest FMM cell only: the targets in that cell and its 26
    neighbours see it through P2P alone; targets farther out do not."""
    n = 32
    rng = np.random.default_rng(3)
    rho = np.zeros((n, n, n))
    T = (3, 4, 2)  # finest cell (level 3, 4 unigrid cells per axis)
    rho[4 * T[0]:4 * T[0] + 4, 4 * T[1]:4 * T[1] + 4, 4 * T[2]:4 * T[2] + 4] = rng.uniform(0.5, 2.0, (4, 4, 4))
    near = [((4 * (T[0] + a) + i) * n + 4 * (T[1] + b) + j) * n + 4 * (T[2] + c) + k
            for a, b, c in itertools.product((-1, 0, 1), repeat=3)
            for i, j, k in itertools.product(range(4), repeat=3)]
    near = np.array(near, dtype=np.int64)
    phi, g = orc.solve(rho, 4, targets=near, delta_l=2)
    pd, gd = orc.direct(rho, targets=near)
    assert np.abs(phi - pd).max() <= 1e-13 * np.abs(pd).max()
    assert np.abs(g - gd).max() <= 1e-13 * np.abs(gd).max()
    # one finest cell further out the M2P takes over: close, but not exact
    far = np.array([((4 * (T[0] + 2) + 1) * n + 4 * T[1] + 2) * n + 4 * T[2] + 1], dtype=np.int64)
    pf, _ = orc.solve(rho, 4, targets=far, delta_l=2)
    pdf, _ = orc.direct(rho, targets=far)
    assert 0 < abs(pf[0] - pdf[0]) < 1e-3 * abs(pdf[0])


@pytest.mark.parametrize("n", [16, 32])
def test_solve_delta2_matches_direct_sum_and_improves_with_p(orc, n):
    rho = fi.plummer_density(n, fi.multi_plummer_params(16, 200 + n))
    pd, gd = orc.direct(rho)
    errs = []
    for p in range(1, 9):
        phi, g = orc.solve(rho, p, delta_l=2)
        errs.append((rel(phi, pd), rel(g, gd)))
    assert errs[5][0] < 1e-4 and errs[5][1] < 2e-3      # p = 6
    for i in range(len(errs) - 2):
        assert errs[i + 2][0] < errs[i][0] and errs[i + 2][1] < errs[i][1], errs


def test_single_massive_cell_closed_form_delta2(orc):
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
    phi, g = orc.solve(rho, 6, delta_l=2)
    assert rel(phi, phi_exact) < 1e-4
    assert rel(g, g_exact) < 1e-3
    assert phi[c] == pytest.approx(-m / dx, rel=1e-12)


def test_cube_symmetries_delta2(orc):
    n = 16
    rho = np.random.default_rng(6).uniform(0, 1, (n, n, n))
    phi, g = orc.solve(rho, 4, delta_l=2)
    syms = [(perm, flips) for perm in itertools.permutations(range(3))
            for flips in itertools.product((0, 1), repeat=3)][::5]
    for perm, flips in syms:
        t = np.ascontiguousarray(np.flip(np.transpose(rho, perm), [a for a in range(3) if flips[a]]))
        phi_t, g_t = orc.solve(t, 4, delta_l=2)
        want = np.flip(np.transpose(phi, perm), [a for a in range(3) if flips[a]])
        assert rel(phi_t, want) < 1e-13
        for j in range(3):
            gj = np.flip(np.transpose(g[perm[j]], perm), [a for a in range(3) if flips[a]])
            assert rel(g_t[j], (-1 if flips[j] else 1) * gj) < 1e-12


def test_fmm1_fmm2_point_charge_differ_below_0p3_percent(orc):
    """App. A: a unit point charge at the box centre, deposited by CIC on the
    8 cells around it, gives FMM-1 and FMM-2 potentials on the midplane slice
    through it that differ by less than about 0.3 % (paper's orders p = 3,
    nmax = 2).  The 0.3 % is read as the level of the difference map: 99 % of
    the slice lies below it; the largest difference, 0.31 % at every grid
    size, sits 4 to 5 cells from the charge, where FMM-1 takes the source
    through M2P and FMM-2 through the near field."""
    n = 64
    rho = fi.point_charge_cic(n)
    h = n // 2
    t = (np.arange(n)[:, None] * n + np.arange(n)[None, :]) * n + h
    t = t.ravel().astype(np.int64)
    p1, _ = orc.solve(rho, 3, nmax=2, targets=t)
    p2, _ = orc.solve(rho, 3, nmax=2, targets=t, delta_l=2)
    d = np.abs(p2 - p1) / np.abs(p1)
    assert np.percentile(d, 99) < 3e-3, np.percentile(d, 99)
    assert 1e-3 < d.max() < 4e-3, d.max()


# --------------------------------------------------------------------------
# adjoint of FMM-2: the explicit transposes against the oracle's own FMM-2
# forward solve (dot-product identity, central differences of a quadratic
# loss, both exact up to rounding for a linear solve) and against the exact
# Green's matrix (agreement to the truncation error)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,p,nmax", [(16, 4, None), (32, 4, None), (32, 3, 2), (64, 2, None)])
def test_fmm2_adjoint_dot_product(orc, n, p, nmax):
    """<A rho, (psi, chi)> = <rho, A^T (psi, chi)> for random vectors; at
    64^3 (F = 4) every pass of the transpose carries weight, the parent-level
    L2P and the L2L chain included."""
    rng = np.random.default_rng(300 + n + p)
    rho = rng.standard_normal((n, n, n))
    wphi = rng.standard_normal((n, n, n))
    wg = rng.standard_normal((3, n, n, n))
    phi, g = orc.solve(rho, p, nmax=nmax, delta_l=2)
    lhs = (phi * wphi).sum() + (g * wg).sum()
    rhs = (rho * orc.adjoint(wphi, wg, p, nmax=nmax, delta_l=2)).sum()
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(phi * wphi).sum() + np.abs(g * wg).sum())
    # the potential part and the acceleration part separately
    rhs_phi = (rho * orc.adjoint(wphi, None, p, nmax=nmax, delta_l=2)).sum()
    assert abs((phi * wphi).sum() - rhs_phi) <= 1e-13 * np.abs(phi * wphi).sum()


def test_fmm2_adjoint_finite_differences(orc):
    """Central differences of L = sum (phi - phi_t)^2 through the FMM-2
    forward solve are exact up to rounding."""
    n, p = 32, 4
    rho = fi.plummer_density(n, fi.multi_plummer_params(6, 5001))
    phi_t, _ = orc.solve(fi.plummer_density(n, fi.multi_plummer_params(6, 5002)), p, delta_l=2)
    phi, _ = orc.solve(rho, p, delta_l=2)
    grad = orc.adjoint(2 * (phi - phi_t), None, p, delta_l=2)
    eps = 1e-3 * rho.max()
    for c in fi.fd_cells(n, 6):
        idx = np.unravel_index(c, rho.shape)
        rp, rm = rho.copy(), rho.copy()
        rp[idx] += eps
        rm[idx] -= eps
        fp = orc.solve(rp, p, delta_l=2)[0]
        fm = orc.solve(rm, p, delta_l=2)[0]
        fd = float(((fp - fm) * (fp + fm - 2 * phi_t)).sum()) / (2 * eps)
        assert fd == pytest.approx(grad[idx], rel=1e-6, abs=1e-9 * abs(grad).max())


def test_fmm2_adjoint_differs_from_fmm1(orc):
    """The FMM-2 adjoint is not the FMM-1 one: their difference is of the
    truncation level (App. A's comparison, transposed), while each is the
    exact transpose of its own forward solve."""
    n, p = 32, 3
    rng = np.random.default_rng(77)
    w = rng.standard_normal((n, n, n))
    a1 = orc.adjoint(w, None, p, delta_l=1)
    a2 = orc.adjoint(w, None, p, delta_l=2)
    d = rel(a2, a1)
    assert 1e-9 < d < 1e-2, d


def test_fmm2_adjoint_close_to_direct_sum_gradient(orc):
    """The gradient of sum (phi - phi_t)^2 with the exact Green's matrix is
    2 dx^3 G (phi - phi_t); the FMM-2 adjoint agrees to its truncation
    error."""
    n, p = 16, 6
    rho = fi.plummer_density(n, fi.multi_plummer_params(6, 5001))
    phi_t = orc.direct(fi.plummer_density(n, fi.multi_plummer_params(6, 5002)))[0]
    grad_direct = 2 * orc.direct(orc.direct(rho)[0] - phi_t)[0]
    phi_f = orc.solve(rho, p, delta_l=2)[0]
    grad_fmm = orc.adjoint(2 * (phi_f - phi_t), None, p, delta_l=2)
    assert rel(grad_fmm, grad_direct) < 1e-4
