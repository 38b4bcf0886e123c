"""Pins of the oracle's finite-difference force (App. C: the host code takes
the force from phi with a 5-point stencil) against the calculus it must
reproduce: exact derivatives of every polynomial of degree <= 4 along each
axis, at every cell including the two one-sided layers at each wall; fourth
order convergence on a smooth field; and not exact at degree 5."""
import numpy as np

import fmm_inputs as fi


def _grid(n):
    c = fi.cell_centres(n)
    return np.meshgrid(c, c, c, indexing="ij")


def test_exact_on_quartics_everywhere(orc):
    n = 16
    X, Y, Z = _grid(n)
    rng = np.random.default_rng(8)
    C = rng.uniform(-1, 1, (5, 5, 5))
    phi = sum(C[a, b, c] * X ** a * Y ** b * Z ** c for a in range(5) for b in range(5) for c in range(5))
    gx = -sum(a * C[a, b, c] * X ** (a - 1) * Y ** b * Z ** c for a in range(1, 5) for b in range(5) for c in range(5))
    gy = -sum(b * C[a, b, c] * X ** a * Y ** (b - 1) * Z ** c for a in range(5) for b in range(1, 5) for c in range(5))
    gz = -sum(c * C[a, b, c] * X ** a * Y ** b * Z ** (c - 1) for a in range(5) for b in range(5) for c in range(1, 5))
    f = orc.fd_force(phi)
    want = np.stack([gx, gy, gz])
    assert np.abs(f - want).max() < 1e-10 * np.abs(want).max()


def test_fourth_order_convergence(orc):
    errs = []
    for n in (16, 32, 64):
        X, Y, Z = _grid(n)
        phi = np.sin(2 * np.pi * X) * np.cos(np.pi * Y) * np.exp(Z)
        gx = -2 * np.pi * np.cos(2 * np.pi * X) * np.cos(np.pi * Y) * np.exp(Z)
        gy = np.pi * np.sin(2 * np.pi * X) * np.sin(np.pi * Y) * np.exp(Z)
        gz = -phi
        e = np.abs(orc.fd_force(phi) - np.stack([gx, gy, gz]))
        errs.append((e[:, 2:-2, 2:-2, 2:-2].max(), e.max()))
    for k in range(2):
        assert errs[k][0] / errs[k + 1][0] > 12, errs   # interior
        assert errs[k][1] / errs[k + 1][1] > 10, errs   # walls included (16 asymptotically)


def test_not_exact_at_degree_five(orc):
    n = 16
    X, _, _ = _grid(n)
    f = orc.fd_force(X ** 5)
    err = np.abs(f[0] + 5 * X ** 4)
    assert err[2:-2].max() > 1e-6 and err.max() > 1e-5
    assert np.abs(f[1]).max() == 0 and np.abs(f[2]).max() == 0
