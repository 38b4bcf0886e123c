"""The seeded inputs and the exact fields the tests compare against
(fmm_inputs.py): the two-sphere potential obeys Poisson's equation and is
continuous at the surfaces, its force is minus its gradient, the particles
fill the spheres with their masses, the CIC point charge holds unit mass, and
cell_order sorts by cell."""
import math

import numpy as np

import fmm_inputs as fi


def test_two_spheres_potential_solves_poisson():
    rng = np.random.default_rng(1)
    h = 1e-3
    for (c, r) in fi.TWO_SPHERES:
        rho = 1.0
        for inside in (True, False):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            x = np.asarray(c) + d * (0.5 * r if inside else 1.5 * r)
            # the other sphere is far enough that its field is smooth here
            lap = sum((fi.two_spheres_potential([x + h * e])[0] - 2 * fi.two_spheres_potential([x])[0]
                       + fi.two_spheres_potential([x - h * e])[0]) / h ** 2 for e in np.eye(3))
            want = 4 * math.pi * rho if inside else 0.0
            assert abs(lap - want) < 1e-3 * 4 * math.pi, (c, inside, lap)
        # continuous across the surface
        d = np.array([0.0, 1.0, 0.0])
        a = fi.two_spheres_potential([np.asarray(c) + d * r * (1 - 1e-9)])[0]
        b = fi.two_spheres_potential([np.asarray(c) + d * r * (1 + 1e-9)])[0]
        assert abs(a - b) < 1e-8 * abs(a)


def test_two_spheres_force_is_minus_the_gradient():
    rng = np.random.default_rng(2)
    pts = rng.uniform(0.2, 0.8, (20, 3))
    h = 1e-5
    g = fi.two_spheres_force(pts)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        num = -(fi.two_spheres_potential(pts + e) - fi.two_spheres_potential(pts - e)) / (2 * h)
        assert np.abs(num - g[d]).max() < 1e-5 * np.abs(g).max()


def test_two_spheres_particles_fill_the_spheres():
    pos, m = fi.two_spheres_particles(1 << 14, seed=3)
    inside = np.zeros(len(pos), bool)
    for c, r in fi.TWO_SPHERES:
        inside |= np.linalg.norm(pos - np.asarray(c), axis=1) <= r
    assert inside.all()
    total = sum(4.0 / 3.0 * math.pi * r ** 3 for _, r in fi.TWO_SPHERES)
    assert abs(m.sum() - total) < 1e-12 * total


def test_point_charge_and_cell_order():
    n = 16
    rho = fi.point_charge_cic(n)
    assert rho.sum() / n ** 3 == 1.0 and np.count_nonzero(rho) == 8
    rng = np.random.default_rng(4)
    pos = rng.uniform(0.0, 1.0, (500, 3))
    order = fi.cell_order(pos, n)
    assert sorted(order.tolist()) == list(range(500))
    lo = np.floor(pos[order] * n - 0.5).astype(int)
    keys = [tuple(v) for v in lo]
    assert keys == sorted(keys)
