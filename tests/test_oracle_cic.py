"""Pins of the oracle's cloud-in-cell deposition (the step before the solve,
Sec. 3) against what fixes the tent weights: a particle on a cell centre
stays in that cell, one on the corner shared by 8 cells gives each 1/8 (the
paper's central point charge), and an interior particle's deposit keeps its
mass and its centre of mass exactly -- on each axis the two weights that sum
to 1 and reproduce the position are the tent weights and nothing else.
Shares that leave the isolated box are dropped by the tent's closed form."""
import numpy as np

import fmm_inputs as fi


def _moments(orc, n, x, m=1.0):
    rho = orc.deposit_cic(n, np.array([x]), np.array([m]))
    dx = 1.0 / n
    c = fi.cell_centres(n)
    w = rho * dx ** 3
    first = np.array([(w.sum(axis=(1, 2)) * c).sum(), (w.sum(axis=(0, 2)) * c).sum(), (w.sum(axis=(0, 1)) * c).sum()])
    return rho, w.sum(), first


def test_particle_on_a_cell_centre_stays_there(orc):
    n = 16
    c = fi.cell_centres(n)
    rho, mass, _ = _moments(orc, n, (c[3], c[9], c[14]), 2.5)
    assert np.count_nonzero(rho) == 1 and rho[3, 9, 14] == 2.5 * n ** 3


def test_point_on_the_shared_corner_splits_in_eight(orc):
    n = 32
    rho = orc.deposit_cic(n, np.array([[0.5, 0.5, 0.5]]), np.array([1.0]))
    assert np.array_equal(rho, fi.point_charge_cic(n))


def test_mass_and_centre_of_mass_are_kept(orc):
    n = 16
    rng = np.random.default_rng(4)
    for x in rng.uniform(1.0 / n, 1 - 1.0 / n, (40, 3)):
        rho, mass, first = _moments(orc, n, x, 1.0)
        assert abs(mass - 1.0) < 1e-14
        assert np.abs(first - x).max() < 1e-14
        # the support is the 2^3 cells around x
        nz = np.argwhere(rho > 0)
        assert len(nz) <= 8 and (np.ptp(nz, axis=0) <= 1).all()
        assert (np.abs((nz + 0.5) / n - x).max(axis=1) < 1.0 / n).all()


def test_share_outside_the_box_is_dropped(orc):
    n = 16
    dx = 1.0 / n
    c = fi.cell_centres(n)
    # a quarter cell from the wall: the tent gives 1/4 to the missing cell
    _, mass, _ = _moments(orc, n, (dx / 4, c[5], c[7]))
    assert abs(mass - 0.75) < 1e-15
    # outside a corner by a quarter cell on each axis: (1/4)^3 of it is left
    _, mass, _ = _moments(orc, n, (1 + dx / 4, 1 + dx / 4, -dx / 4))
    assert abs(mass - 0.25 ** 3) < 1e-15
    _, mass, _ = _moments(orc, n, (1.5, 0.5, 0.5))
    assert mass == 0.0


def test_deposit_is_linear(orc):
    n = 8
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, 1, (50, 3))
    m = rng.uniform(0.1, 1, 50)
    whole = orc.deposit_cic(n, pos, m)
    parts = sum(orc.deposit_cic(n, pos[i:i + 1], m[i:i + 1]) for i in range(50))
    assert np.abs(whole - parts).max() < 1e-12 * np.abs(whole).max()
