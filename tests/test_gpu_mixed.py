"""Mixed-precision solves (FP32 / BF16 matrix-core operands, FP32
accumulation) against the FP64 oracle.

The oracle solves the same input the GPU sees: the density rounded to FP32
and widened back.  Bars, each as a relative L2 error over the grid (or the
sampled cells) and as a per-cell bound max|err| / max|ref|:
    FP32   phi <= 1e-5   g <= 1e-4
    BF16   phi <= 5e-3   g <= 5e-2
(the per-cell bound follows from rounding each matrix-core operand once:
about 2u times the sum of a cell's term magnitudes, which for phi is close
to |phi| and for g reaches several times max|g|).
Levels at or below ``coarse_fp64_levels`` (default 4) keep FP64; small grids
are run with that threshold lowered so the low-precision kernels carry every
level.
"""
import math
import sys

import numpy as np
import pytest

import fmm_inputs as fi

pytestmark = pytest.mark.gpu

BARS = {"fp32": (1e-5, 1e-4), "bf16": (5e-3, 5e-2)}


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


def cell_max(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _solve(F, rho32, p, precision, coarse):
    import torch
    n = rho32.shape[0]
    plan = F.Plan(n, p, precision, coarse_fp64_levels=coarse)
    phi, g = plan.solve(torch.as_tensor(rho32).cuda())
    torch.cuda.synchronize()
    assert phi.dtype == torch.float32 and g.dtype == torch.float32
    return phi.double().cpu().numpy(), g.double().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n,p,coarse", [(16, 4, 0), (32, 6, 0), (64, 6, 0), (64, 6, 2), (32, 8, 0)])
def test_mixed_full_grid(F, orc, precision, n, p, coarse):
    _say(f"case {precision} full n={n} p={p} coarse_fp64_levels={coarse}")
    rho32 = fi.plummer_density(n, fi.multi_plummer_params(32, 700 + n + p)).astype(np.float32)
    phi, g = _solve(F, rho32, p, precision, coarse)
    phi_o, g_o = orc.solve(rho32.astype(np.float64), p)
    ep, eg = rel(phi, phi_o), rel(g, g_o)
    cp, cg = cell_max(phi, phi_o), cell_max(g, g_o)
    _say(f"  rel L2 phi {ep:.3e} g {eg:.3e}; per cell phi {cp:.3e} g {cg:.3e}")
    bp, bg = BARS[precision]
    assert ep <= bp and eg <= bg, (ep, eg)
    assert cp <= bp and cg <= bg, (cp, cg)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_coarse_levels_stay_fp64(F, orc, precision):
    """With every level at or below the FP64 threshold the solve is the FP64
    path with float I/O: only the output rounding remains."""
    _say(f"case {precision} all-fp64 levels n=32 p=6")
    rho32 = fi.plummer_density(32, fi.multi_plummer_params(16, 41)).astype(np.float32)
    phi, g = _solve(F, rho32, 6, precision, 8)
    phi_o, g_o = orc.solve(rho32.astype(np.float64), 6)
    assert rel(phi, phi_o) < 2e-7 and rel(g, g_o) < 2e-7, (rel(phi, phi_o), rel(g, g_o))
    # float output rounding only: half an FP32 ulp of each value
    # (plus the FP64 solve's own rounding, far below it)
    assert np.all(np.abs(phi - phi_o) <= 1.001 * 2.0 ** -24 * np.abs(phi_o) + 1e-13 * np.abs(phi_o).max())
    assert np.all(np.abs(g - g_o) <= 1.001 * 2.0 ** -24 * np.abs(g_o) + 1e-13 * np.abs(g_o).max())


def test_error_ordering(F, orc):
    """BF16 operands lose more than FP32 operands, which lose more than FP64."""
    _say("case error ordering n=32 p=6")
    rho32 = fi.plummer_density(32, fi.multi_plummer_params(32, 43)).astype(np.float32)
    phi_o, g_o = orc.solve(rho32.astype(np.float64), 6)
    err = {}
    for prec in ("fp32", "bf16"):
        phi, g = _solve(F, rho32, 6, prec, 0)
        err[prec] = (rel(phi, phi_o), rel(g, g_o))
    assert err["bf16"][0] > err["fp32"][0] and err["bf16"][1] > err["fp32"][1], err


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [128, 256])
def test_mixed_full_size_sampled(F, orc, precision, n):
    """128^3 and 256^3 (where the finest level's locals stay in the compute
    type), p = 6, default policy (levels <= 4 in FP64), sampled cells."""
    import torch
    p = 6
    _say(f"case {precision} sampled n={n} p={p}")
    rho_t = fi.plummer_density(n, fi.multi_plummer_params(32, 128), device="cuda").float()
    plan = F.Plan(n, p, precision)
    phi, g = plan.solve(rho_t)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    cells = np.unique(np.concatenate([[0, n ** 3 - 1], rng.choice(n ** 3, 48, replace=False)]))
    idx = torch.as_tensor(cells, device="cuda")
    phi_s = phi.reshape(-1)[idx].double().cpu().numpy()
    g_s = g.reshape(3, -1)[:, idx].double().cpu().numpy()
    phi_o, g_o = orc.solve(rho_t.double().cpu().numpy(), p, targets=cells)
    ep, eg = rel(phi_s, phi_o), rel(g_s, g_o)
    cp, cg = cell_max(phi_s, phi_o), cell_max(g_s, g_o)
    _say(f"  rel L2 phi {ep:.3e} g {eg:.3e}; per cell phi {cp:.3e} g {cg:.3e}")
    bp, bg = BARS[precision]
    assert ep <= bp and eg <= bg, (ep, eg)
    assert cp <= bp and cg <= bg, (cp, cg)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_finest_level_kept_in_compute_type(F, orc, precision):
    """A low-precision bottom keeps the finest level's multipoles and M2L
    locals in its compute type only, so their FP64 export is refused; the
    level below, formed from the density in FP64, matches the oracle's
    multipoles to 1e-12."""
    import torch
    # (below 256^3 the finest M2L launch is small enough to split its offset
    # sums, whose FP64 partial sums keep the locals in FP64)
    n, p = 256, 6
    _say(f"case {precision} finest-level storage n={n} p={p}")
    rho32 = fi.plummer_density(n, fi.multi_plummer_params(8, 47)).astype(np.float32)
    plan = F.Plan(n, p, precision)
    plan.solve(torch.as_tensor(rho32).cuda())
    torch.cuda.synchronize()
    lev = plan.finest_level
    for which in ("M", "L"):
        with pytest.raises(F.FmmError) as ei:
            plan.expansions(which, lev)
        assert ei.value.code == F.FMM_ERR_UNSUPPORTED
    # the oracle's physical multipoles in the kernels' scaled form and order:
    # Mhat[a] = (-1)^|a| M[a] / (a! h^|a| dx^3)
    level = lev - 1
    mi_o = [tuple(e) for e in orc.multi_index(p)]
    mi_g = [tuple(e) for e in F.multi_index(p)]
    col = [mi_o.index(e) for e in mi_g]
    deg = np.array([sum(e) for e in mi_g])
    fact = np.array([math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2]) for e in mi_g], float)
    dx, h = 1.0 / n, 2.0 ** -level
    want = orc.expansions(rho32.astype(np.float64), p, "M", level)[:, col] * ((-1.0) ** deg) / (fact * h ** deg * dx ** 3)
    got = plan.expansions("M", level)
    assert rel(got, want) < 1e-12, rel(got, want)
