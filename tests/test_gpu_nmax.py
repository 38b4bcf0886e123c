"""Multipoles truncated at n_max < p (Sec. 2.1: the multipole order n_max and
the local order p are separate; the paper's own configuration is p = 3,
n_max = 2), through the C ABI, against the FP64 oracle run with the same
n_max.

Bars: FP64 relative L2 <= 1e-12 for phi, g, the multipole grids and the
adjoint; FP32 phi <= 1e-5, g <= 1e-4 against the oracle of the float-rounded
input.
"""
import math
import sys

import numpy as np
import pytest

import fmm_inputs as fi

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2606_13793_amd import fmm
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return fmm


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solve(F, rho, p, nmax, precision="fp64"):
    import torch
    n = rho.shape[0]
    plan = F.Plan(n, p, precision, nmax=nmax)
    dt = torch.float64 if precision == "fp64" else torch.float32
    phi, g = plan.solve(torch.as_tensor(rho).to("cuda", dt).contiguous())
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), g.double().cpu().numpy(), plan


@pytest.mark.parametrize("n,p,nmax", [(16, 3, 2), (32, 3, 2), (32, 6, 4), (16, 2, 0), (64, 3, 2)])
def test_truncated_multipoles_match_oracle(F, orc, n, p, nmax):
    _say(f"case nmax fp64 n={n} p={p} nmax={nmax}")
    rho = fi.plummer_density(n, fi.multi_plummer_params(16, 700 + n + p))
    phi, g, _ = _solve(F, rho, p, nmax)
    phi_o, g_o = orc.solve(rho, p, nmax=nmax)
    e1, e2 = rel(phi, phi_o), rel(g, g_o)
    _say(f"  phi {e1:.2e} g {e2:.2e}")
    assert e1 < TOL64 and e2 < TOL64, (e1, e2)
    # the truncation changes the answer: it is not the n_max = p solve
    phi_p, _ = orc.solve(rho, p)
    assert rel(phi_o, phi_p) > 1e-9


def test_truncated_multipole_grids(F, orc):
    """The kept multipole terms at every level equal the oracle's (the
    dropped ones are not reported)."""
    n, p, nmax = 32, 3, 2
    _say("case nmax expansions n=32 p=3 nmax=2")
    rho = fi.plummer_density(n, fi.multi_plummer_params(8, 91))
    _, _, plan = _solve(F, rho, p, nmax)
    # the oracle's physical multipoles in the kernels' scaled form and term
    # order: Mhat[a] = (-1)^|a| M[a] / (a! h^|a| dx^3)
    mi_o = [tuple(e) for e in orc.multi_index(nmax)]
    mi_g = [tuple(e) for e in F.multi_index(nmax)]
    col = [mi_o.index(e) for e in mi_g]
    deg = np.array([sum(e) for e in mi_g])
    fact = np.array([math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2]) for e in mi_g], float)
    dx = 1.0 / n
    finest = n.bit_length() - 2  # F = log2(n) - 1
    for level in range(2, finest + 1):
        h = 2.0 ** -level
        got = plan.expansions("M", level)
        ref = orc.expansions(rho, p, "M", level, nmax=nmax)[:, col] * ((-1.0) ** deg) / (fact * h ** deg * dx ** 3)
        assert got.shape == ref.shape
        assert rel(got, ref) < TOL64, level


def test_truncated_adjoint_matches_oracle(F, orc):
    import torch
    n, p, nmax = 16, 3, 2
    _say("case nmax adjoint n=16 p=3 nmax=2")
    rng = np.random.default_rng(17)
    dphi, dg = rng.standard_normal((n, n, n)), rng.standard_normal((3, n, n, n))
    plan = F.Plan(n, p, nmax=nmax)
    got = plan.backward(torch.as_tensor(dphi, device="cuda"), torch.as_tensor(dg, device="cuda"))
    torch.cuda.synchronize()
    ref = orc.adjoint(dphi, dg, p, nmax=nmax)
    assert rel(got.cpu().numpy(), ref) < TOL64


def test_truncated_fp32(F, orc):
    n, p, nmax = 64, 3, 2
    _say("case nmax fp32 n=64 p=3 nmax=2")
    rho = fi.plummer_density(n, fi.multi_plummer_params(16, 93)).astype(np.float32)
    phi, g, _ = _solve(F, rho, p, nmax, "fp32")
    phi_o, g_o = orc.solve(rho.astype(np.float64), p, nmax=nmax)
    e1, e2 = rel(phi, phi_o), rel(g, g_o)
    _say(f"  phi {e1:.2e} g {e2:.2e}")
    assert e1 < 1e-5 and e2 < 1e-4, (e1, e2)
