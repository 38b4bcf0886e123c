"""The finite-difference force (``fmm_fd_force``, App. C) on the GPU against
the oracle's, and App. C's check on the paper's two spheres: inside them,
where the density is non-zero, 90 % of the cells hold a force magnitude
within one percent of the exact one.

Bar: the GPU force matches the oracle to 1e-13 of its largest component (the
same stencils, summed in another order)."""
import os
import sys

import numpy as np
import pytest

import fmm_inputs as fi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2606_13793_amd import fmm
    assert os.path.exists(fmm.LIB_PATH), "libfmm.so must be built before the GPU tests"
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return fmm


@pytest.mark.parametrize("n", [8, 16, 64])
def test_fd_force_matches_oracle(F, orc, n):
    import torch
    _say(f"case fd force n={n}")
    phi = np.random.default_rng(n).standard_normal((n, n, n))
    f = F.fd_force(torch.as_tensor(phi).cuda()).cpu().numpy()
    want = orc.fd_force(phi)
    assert np.abs(f - want).max() <= 1e-13 * np.abs(want).max()


def test_fd_force_of_a_solved_potential_matches_oracle(F, orc):
    import torch
    n = 32
    _say("case fd force of a solve n=32")
    rho = fi.plummer_density(n, fi.multi_plummer_params(8, 77))
    phi, _ = F.Plan(n, 4, "fp64").solve(torch.as_tensor(rho).cuda(), want_g=False)
    f = F.fd_force(phi).cpu().numpy()
    want = orc.fd_force(orc.solve(rho, 4)[0])
    assert np.abs(f - want).max() <= 1e-11 * np.abs(want).max()


def _inside_cells(n):
    """Flat indices and centres of the cells whose centres lie inside a sphere."""
    c = fi.cell_centres(n)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    inside = np.zeros(len(pts), bool)
    for cc, r in fi.TWO_SPHERES:
        inside |= np.linalg.norm(pts - np.asarray(cc), axis=1) < r
    idx = np.nonzero(inside)[0]
    return idx, pts[idx]


@pytest.mark.parametrize("source", ["cells", "particles"])
def test_two_spheres_force_inside_within_one_percent_256(F, source):
    """App. C at the paper's 256^3, p = 3, nmax = 2: inside the spheres the
    90th percentile of the relative force-magnitude error is below 1 %, for
    the finite-difference force and for the solve's own g, with FMM-1 and
    FMM-2.  "cells": the spheres sampled at the cell centres (density 1
    inside).  "particles": 16M particles deposited by CIC, over the cells
    whose centres lie inside; over every cell the deposit reaches (the CIC
    halo just outside the surfaces included) the percentile is about 1.5 %,
    held here below 2 %."""
    import torch
    n = 256
    _say(f"case two spheres force n=256 from {source}")
    if source == "cells":
        rho = torch.as_tensor(sum(fi.uniform_sphere_density(n, c, r) for c, r in fi.TWO_SPHERES)).cuda()
    else:
        pos, m = fi.two_spheres_particles(1 << 24)
        rho = F.deposit_cic(n, torch.as_tensor(pos).cuda(), torch.as_tensor(m).cuda())
        del pos, m
    idx, pts = _inside_cells(n)
    sets = [(torch.as_tensor(idx).cuda(), np.linalg.norm(fi.two_spheres_force(pts), axis=0), 1e-2)]
    if source == "particles":
        flat = torch.nonzero(rho.reshape(-1) > 0).flatten()
        f = flat.cpu().numpy()
        c = fi.cell_centres(n)
        pts_nz = np.stack([c[f // (n * n)], c[(f // n) % n], c[f % n]], 1)
        sets.append((flat, np.linalg.norm(fi.two_spheres_force(pts_nz), axis=0), 2e-2))
    for dl in (1, 2):
        phi, g = F.Plan(n, 3, "fp64", nmax=2, delta_l=dl).solve(rho)
        for name, force in (("fd", F.fd_force(phi)), ("g", g)):
            for cells, exact, bar in sets:
                mag = torch.linalg.vector_norm(force.reshape(3, -1)[:, cells], dim=0).cpu().numpy()
                err = np.abs(mag - exact) / exact
                assert np.percentile(err, 90) < bar, (dl, name, len(exact), np.percentile(err, 90))
