"""FMM-2 (delta_l = 2, App. A) on the GPU against the FP64 oracle's FMM-2.

Same bar as FMM-1: relative L2 error <= 1e-12 for phi and g (the two sides
differ only in rounding order).  Covers several tiles and ragged tails
(n = 16 .. 64 full grids), the paper's orders (p = 3, nmax = 2), the
benchmark size (256^3, sampled cells evaluated by the oracle one by one),
the FMM-1 vs FMM-2 point-charge difference of App. A at the paper's 256^3,
and the combinations the plan rejects.
"""
import os
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
    assert os.path.exists(fmm.LIB_PATH), "libfmm.so must be built before the GPU tests"
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return fmm


def rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def solve2(F, rho, p, nmax=None):
    import torch
    n = rho.shape[0]
    plan = F.Plan(n, p, "fp64", nmax=nmax, delta_l=2)
    r = torch.as_tensor(rho).to(device="cuda", dtype=torch.float64).contiguous()
    phi, g = plan.solve(r)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), g.cpu().numpy(), plan


@pytest.mark.parametrize("n,p,nmax", [(16, 4, None), (16, 1, None), (32, 6, None), (32, 3, 2),
                                      (64, 6, None), (64, 8, None)])
def test_fmm2_full_grid_matches_oracle(F, orc, n, p, nmax):
    _say(f"case fmm2 full n={n} p={p} nmax={nmax}")
    rho = fi.plummer_density(n, fi.multi_plummer_params(32, 300 + n))
    phi, g, plan = solve2(F, rho, p, nmax)
    assert plan.finest_level == int(np.log2(n)) - 2
    phi_o, g_o = orc.solve(rho, p, nmax=nmax, delta_l=2)
    assert rel(phi, phi_o) < TOL64, rel(phi, phi_o)
    assert rel(g, g_o) < TOL64, rel(g, g_o)


def test_fmm2_random_density_every_cell(F, orc):
    """A density with no structure, so every table entry and every near-field
    offset carries weight; checked cell by cell."""
    _say("case fmm2 random n=32 p=5")
    rho = np.random.default_rng(21).uniform(-1.0, 1.0, (32, 32, 32))
    phi, g, _ = solve2(F, rho, 5)
    phi_o, g_o = orc.solve(rho, 5, delta_l=2)
    assert np.abs(phi - phi_o).max() <= 1e-12 * np.abs(phi_o).max()
    assert np.abs(g - g_o).max() <= 1e-12 * np.abs(g_o).max()


@pytest.mark.parametrize("n", [256, 512])
def test_fmm2_full_size_sampled(F, orc, n):
    """256^3 and 512^3, p = 6: the benchmark's FMM-2 launch and a larger
    one, at sampled cells."""
    import torch
    p = 6
    _say(f"case fmm2 sampled n={n} p={p}")
    rho_t = fi.plummer_density(n, fi.multi_plummer_params(256, 256), device="cuda")
    plan = F.Plan(n, p, "fp64", delta_l=2)
    phi, g = plan.solve(rho_t)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    corners = [0, n - 1, (n - 1) * n * n, n ** 3 - 1, ((n // 2) * n + n // 2) * n + n // 2, n * n - 1]
    cells = np.unique(np.concatenate([corners, rng.choice(n ** 3, 40, replace=False)]))
    idx = torch.as_tensor(cells, device="cuda")
    phi_s = phi.reshape(-1)[idx].cpu().numpy()
    g_s = g.reshape(3, -1)[:, idx].cpu().numpy()
    rho = rho_t.cpu().numpy()
    del phi, g
    phi_o, g_o = orc.solve(rho, p, targets=cells, delta_l=2)
    assert rel(phi_s, phi_o) < TOL64, rel(phi_s, phi_o)
    assert rel(g_s, g_o) < TOL64, rel(g_s, g_o)
    assert np.max(np.abs(phi_s - phi_o) / np.abs(phi_o)) < 1e-11


def test_fmm1_fmm2_point_charge_256(F):
    """App. A at the paper's 256^3 with its orders (p = 3, nmax = 2): the
    midplane potentials of FMM-1 and FMM-2 differ by about 0.3 % at most
    (99 % of the slice below 0.3 %, the largest 0.31 %, as in the oracle)."""
    import torch
    n = 256
    _say("case fmm1 vs fmm2 point charge n=256 p=3 nmax=2")
    rho = torch.as_tensor(fi.point_charge_cic(n)).cuda()
    p1, _ = F.Plan(n, 3, "fp64", nmax=2).solve(rho, want_g=False)
    p2, _ = F.Plan(n, 3, "fp64", nmax=2, delta_l=2).solve(rho, want_g=False)
    s1, s2 = p1[:, :, n // 2].cpu().numpy(), p2[:, :, n // 2].cpu().numpy()
    d = np.abs(s2 - s1) / np.abs(s1)
    assert np.percentile(d, 99) < 3e-3, np.percentile(d, 99)
    assert 1e-3 < d.max() < 4e-3, d.max()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n,p,coarse", [(32, 6, 0), (64, 6, 0), (64, 4, 2)])
def test_fmm2_mixed_precision_matches_oracle(F, orc, precision, n, p, coarse):
    """FMM-2 with FP32 / BF16 operands against the FP64 oracle's FMM-2 of the
    same float-rounded density, at the mixed-precision bars of FMM-1."""
    import torch
    _say(f"case fmm2 {precision} n={n} p={p} coarse_fp64_levels={coarse}")
    bars = {"fp32": (1e-5, 1e-4), "bf16": (5e-3, 5e-2)}
    rho32 = fi.plummer_density(n, fi.multi_plummer_params(32, 900 + n + p)).astype(np.float32)
    plan = F.Plan(n, p, precision, coarse_fp64_levels=coarse, delta_l=2)
    phi, g = plan.solve(torch.as_tensor(rho32).cuda())
    torch.cuda.synchronize()
    assert phi.dtype == torch.float32
    phi_o, g_o = orc.solve(rho32.astype(np.float64), p, delta_l=2)
    phi, g = phi.double().cpu().numpy(), g.double().cpu().numpy()
    ep, eg = rel(phi, phi_o), rel(g, g_o)
    # per cell as well: max |err| / max |ref| (operand rounding bounds each
    # cell's error by about 2u times the sum of its term magnitudes)
    cp = float(np.abs(phi - phi_o).max() / np.abs(phi_o).max())
    cg = float(np.abs(g - g_o).max() / np.abs(g_o).max())
    _say(f"  rel L2 phi {ep:.2e} g {eg:.2e}; per cell phi {cp:.2e} g {cg:.2e}")
    bp, bg = bars[precision]
    assert ep <= bp and eg <= bg, (ep, eg)
    assert cp <= bp and cg <= bg, (cp, cg)


def test_fmm2_rejections(F):
    _say("case fmm2 rejections")
    with pytest.raises(F.FmmError):
        F.Plan(8, 4, "fp64", delta_l=2)          # needs n >= 16
    with pytest.raises(F.FmmError):
        F.Plan(32, 4, "fp64", delta_l=3)
    with pytest.raises(F.FmmError):
        F.Plan(32, 4, "fp64", delta_l=2, bottom_tile=8)


# --------------------------------------------------------------------------
# the backward pass of FMM-2 plans
# --------------------------------------------------------------------------
def _cot(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n, n)), rng.standard_normal((3, n, n, n))


def _gpu_bwd(F, n, p, dphi, dg, precision="fp64", nmax=None, coarse=4):
    import torch
    plan = F.Plan(n, p, precision, nmax=nmax, coarse_fp64_levels=coarse, delta_l=2)
    dt = torch.float64 if precision == "fp64" else torch.float32
    a = torch.as_tensor(dphi).to("cuda", dt).contiguous()
    b = None if dg is None else torch.as_tensor(dg).to("cuda", dt).contiguous()
    out = plan.backward(a, b)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


@pytest.mark.parametrize("n,p,nmax", [(16, 4, None), (32, 6, None), (32, 3, 2), (64, 6, None), (64, 2, None),
                                      (32, 8, None)])
def test_fmm2_adjoint_matches_oracle(F, orc, n, p, nmax):
    """Every cell against the oracle's explicit transposes of FMM-2: 16^3
    (no locals), 32^3 (locals at one level) and 64^3 (parent-level L2P and
    the L2L chain)."""
    _say(f"case fmm2 adjoint fp64 n={n} p={p} nmax={nmax}")
    dphi, dg = _cot(n, 500 + n + p)
    got = _gpu_bwd(F, n, p, dphi, dg, nmax=nmax)
    ref = orc.adjoint(dphi, dg, p, nmax=nmax, delta_l=2)
    e, c = rel(got, ref), float(np.abs(got - ref).max() / np.abs(ref).max())
    _say(f"  rel L2 {e:.2e}, per cell {c:.2e}")
    assert e <= TOL64 and c <= TOL64, (e, c)
    got = _gpu_bwd(F, n, p, dphi, None, nmax=nmax)
    assert rel(got, orc.adjoint(dphi, None, p, nmax=nmax, delta_l=2)) <= TOL64


@pytest.mark.parametrize("n", [128, 256])
def test_fmm2_adjoint_dot_product(F, n):
    """<A rho, (psi, chi)> = <rho, A^T (psi, chi)> with the GPU's own FMM-2
    forward solve, at the sizes the benchmark runs (exact up to rounding)."""
    import torch
    _say(f"case fmm2 dot product fp64 n={n} p=6")
    plan = F.Plan(n, 6, "fp64", delta_l=2)
    rho = fi.plummer_density(n, fi.multi_plummer_params(16, 9 + n), device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(n)
    psi = torch.randn((n, n, n), dtype=torch.float64, device="cuda", generator=gen)
    chi = torch.randn((3, n, n, n), dtype=torch.float64, device="cuda", generator=gen)
    phi, g = plan.solve(rho)
    lhs = float((phi * psi).sum() + (g * chi).sum())
    rhs = float((rho * plan.backward(psi, chi)).sum())
    scale = float(phi.norm() * psi.norm() + g.norm() * chi.norm())
    _say(f"  |lhs - rhs| / scale = {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("precision,bar", [("fp32", 1e-4), ("bf16", 5e-2)])
def test_fmm2_adjoint_mixed(F, orc, precision, bar):
    """Low-precision FMM-2 adjoint on every level (threshold 0) against the
    oracle, relative L2 and per cell."""
    _say(f"case fmm2 adjoint {precision} n=64 p=6")
    dphi, dg = _cot(64, 41)
    d32, g32 = dphi.astype(np.float32), dg.astype(np.float32)
    got = _gpu_bwd(F, 64, 6, d32, g32, precision, coarse=0)
    ref = orc.adjoint(d32.astype(np.float64), g32.astype(np.float64), 6, delta_l=2)
    e, c = rel(got, ref), float(np.abs(got - ref).max() / np.abs(ref).max())
    _say(f"  rel L2 {e:.2e}, per cell {c:.2e}")
    assert e < bar and c < bar, (e, c)


def test_fmm2_autograd(F, orc):
    """torch.autograd through an FMM-2 plan: the gradient of sum (phi - phi_t)^2
    is the oracle's FMM-2 adjoint of 2 (phi - phi_t)."""
    import torch
    n, p = 32, 4
    _say("case fmm2 autograd n=32 p=4")
    rho = fi.plummer_density(n, fi.multi_plummer_params(16, 5001))
    phi_t, _ = orc.solve(fi.plummer_density(n, fi.multi_plummer_params(16, 5002)), p, delta_l=2)
    plan = F.Plan(n, p, delta_l=2)
    x = torch.as_tensor(rho, device="cuda").requires_grad_(True)
    phi, g = F.solve(plan, x)
    ((phi - torch.as_tensor(phi_t, device="cuda")) ** 2).sum().backward()
    r = phi.detach().cpu().numpy() - phi_t
    assert rel(x.grad.cpu().numpy(), orc.adjoint(2 * r, None, p, delta_l=2)) < TOL64
