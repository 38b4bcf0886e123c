"""Parity of the launch configurations the benchmark times, at full size.

* The 16-deep bottom tiles (k_bottom<..., 16, 1>) run wherever a bottom site
  has at least one tile per compute unit, i.e. from 128^3 up; smaller grids
  take 8-deep tiles.  Here the 16-deep kernel is compared with the oracle on
  every cell: forced (option bottom_tile = 16) at 32^3 and 64^3 in every
  precision policy, and in its natural configuration at 128^3, p = 6 (the
  dense oracle solve takes about 40 s on 16 host threads).
* The benchmark's own slab check at 256^3, p = 6: 16 central unigrid planes
  (1,048,576 cells) against the oracle's downward pass for them.
* The 96-field batch of the uneven-batch workload (55 x 32^3, 27 x 64^3,
  14 x 128^3, FP32) at p = 4 and p = 6: sampled cells of every field
  against the oracle of that field's float-rounded density.

Bars (the SURVEY's tolerance table), each as a relative L2 error AND as a
per-cell bound max|err| / max|ref| over the compared cells:
    FP64   phi 1e-12   g 1e-12
    FP32   phi 1e-5    g 1e-4
    BF16   phi 5e-3    g 5e-2
The per-cell bounds follow from the operand rounding: every matrix-core
product rounds both operands once (unit roundoff u = 2^-24 for FP32, 2^-9
for BF16), so a cell's error is at most about 2u times the sum of the
magnitudes of its terms.  For phi of a positive density the terms share
their sign (the sum is within a few percent of |phi|); for g they cancel,
and the sum of magnitudes reaches several times max|g|, hence the wider g
bar.  FP32 accumulation over the ~16k products of a cell adds a random-walk
term of order sqrt(16k) u, still far below the FP32 bars.
"""
import sys

import numpy as np
import pytest

import fmm_inputs as fi

pytestmark = pytest.mark.gpu

BARS = {"fp64": (1e-12, 1e-12), "fp32": (1e-5, 1e-4), "bf16": (5e-3, 5e-2)}


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
    """max |a - b| / max |b| over the compared cells (and components)."""
    a, b = np.ravel(a), np.ravel(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def check(precision, phi, g, phi_o, g_o, label=""):
    bp, bg = BARS[precision]
    e = (rel(phi, phi_o), rel(g, g_o), cell_max(phi, phi_o), cell_max(g, g_o))
    _say(f"  {label} rel L2 phi {e[0]:.2e} g {e[1]:.2e}; per cell phi {e[2]:.2e} g {e[3]:.2e}")
    assert e[0] <= bp and e[2] <= bp, (label, e)
    assert e[1] <= bg and e[3] <= bg, (label, e)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,p", [(32, 6), (64, 6), (64, 3)])
def test_forced_16_deep_bottom_full_grid(F, orc, precision, n, p):
    """k_bottom<..., 16, 1> on every cell of grids too small to select it by
    itself (ragged z tiles at 32^3: a 16-deep tile over 16 level-F cells);
    every level in the plan's precision (coarse_fp64_levels = 0)."""
    import torch
    _say(f"case forced 16-deep bottom {precision} n={n} p={p}")
    rho = fi.plummer_density(n, fi.multi_plummer_params(32, 1600 + n + p))
    if precision != "fp64":
        rho = rho.astype(np.float32).astype(np.float64)
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = F.Plan(n, p, precision, coarse_fp64_levels=0, bottom_tile=16)
    phi, g = plan.solve(torch.as_tensor(rho).to("cuda", dt))
    torch.cuda.synchronize()
    phi_o, g_o = orc.solve(rho, p)
    check(precision, phi.double().cpu().numpy(), g.double().cpu().numpy(), phi_o, g_o)


def test_forced_8_deep_bottom_at_128(F, orc):
    """The other direction: 8-deep tiles forced where 16 would be chosen."""
    import torch
    n, p = 128, 4
    _say(f"case forced 8-deep bottom fp64 n={n} p={p}")
    rho_t = fi.plummer_density(n, fi.multi_plummer_params(32, 128), device="cuda")
    a = F.Plan(n, p, "fp64", bottom_tile=8)
    b = F.Plan(n, p, "fp64")
    pa, ga = a.solve(rho_t)
    pb, gb = b.solve(rho_t)
    torch.cuda.synchronize()
    # the same sums per cell; only their order differs (each block starts
    # its offset walk at a rotation of its own)
    pa, ga, pb, gb = (t.cpu().numpy() for t in (pa, ga, pb, gb))
    assert cell_max(pa, pb) < 1e-13 and cell_max(ga, gb) < 1e-13
    cells = _batch_cells(n, 0)
    phi_o, g_o = orc.solve(rho_t.cpu().numpy(), p, targets=cells)
    check("fp64", pa.reshape(-1)[cells], ga.reshape(3, -1)[:, cells], phi_o, g_o)


def test_fp64_dense_128_p6(F, orc):
    """Every cell of the 128^3, p = 6 FP64 solve (the CPU-baseline workload,
    32 Plummer spheres, seed 128), where the 16-deep bottom tiles and the
    unsplit M2L launch run as in the benchmark."""
    import torch
    n, p = 128, 6
    _say(f"case fp64 dense n={n} p={p} (oracle on the full grid)")
    rho_t = fi.plummer_density(n, fi.multi_plummer_params(32, 128), device="cuda")
    plan = F.Plan(n, p, "fp64")
    phi, g = plan.solve(rho_t)
    torch.cuda.synchronize()
    phi, g = phi.cpu().numpy(), g.cpu().numpy()
    rho = rho_t.cpu().numpy()
    del rho_t
    phi_o, g_o = orc.solve(rho, p)
    check("fp64", phi, g, phi_o, g_o)


def test_fp64_slab_256_p6(F, orc):
    """The benchmark's workload (256^3, p = 6, 256 spheres, seed 256) on the
    16 central unigrid planes, against the oracle's full upward pass and its
    downward pass for those 1,048,576 cells."""
    import torch
    n, p, planes = 256, 6, 16
    _say(f"case fp64 slab n={n} p={p} planes={planes}")
    rho_t = fi.plummer_density(n, fi.multi_plummer_params(256, 256), device="cuda")
    plan = F.Plan(n, p, "fp64")
    phi, g = plan.solve(rho_t)
    torch.cuda.synchronize()
    i0 = n // 2 - planes // 2
    cells = np.arange(i0 * n * n, (i0 + planes) * n * n, dtype=np.int64)
    phi_s = phi.reshape(-1)[i0 * n * n:(i0 + planes) * n * n].cpu().numpy()
    g_s = g.reshape(3, -1)[:, i0 * n * n:(i0 + planes) * n * n].cpu().numpy()
    rho = rho_t.cpu().numpy()
    del phi, g, rho_t, plan
    phi_o, g_o = orc.solve(rho, p, targets=cells)
    check("fp64", phi_s, g_s, phi_o, g_o)


def _batch_cells(n, f, count=24):
    rng = np.random.default_rng(9000 + f)
    corners = [0, n - 1, (n - 1) * n * n, n ** 3 - 1, ((n // 2) * n + n // 2) * n + n // 2]
    return np.unique(np.concatenate([corners, rng.choice(n ** 3, count, replace=False)]))


@pytest.mark.parametrize("p", [4, 6])
def test_uneven_batch_96_fields_fp32(F, orc, p):
    """The 96-field FP32 batch as the benchmark runs it (autotuned, graph
    replay), every field checked at sampled cells against the oracle."""
    import torch
    sizes = fi.batch_sizes()
    assert len(sizes) == 96 and sorted(set(sizes)) == [32, 64, 128]
    _say(f"case uneven batch 96 fields fp32 p={p}")
    rhos = [fi.plummer_density(m, fi.batch_field_params(f), device="cuda").float() for f, m in enumerate(sizes)]
    B = F.Batch(sizes, p, "fp32")
    phis, gs = B.solve(rhos)
    phis, gs = B.solve(rhos)  # a graph replay
    torch.cuda.synchronize()
    worst = [0.0] * 4
    for f, n in enumerate(sizes):
        cells = _batch_cells(n, f)
        idx = torch.as_tensor(cells, device="cuda")
        phi_s = phis[f].reshape(-1)[idx].double().cpu().numpy()
        g_s = gs[f].reshape(3, -1)[:, idx].double().cpu().numpy()
        phi_o, g_o = orc.solve(rhos[f].double().cpu().numpy(), p, targets=cells)
        e = (rel(phi_s, phi_o), rel(g_s, g_o), cell_max(phi_s, phi_o), cell_max(g_s, g_o))
        worst = [max(w, x) for w, x in zip(worst, e)]
        bp, bg = BARS["fp32"]
        assert e[0] <= bp and e[2] <= bp and e[1] <= bg and e[3] <= bg, (f, n, e)
    _say(f"  worst field: rel L2 phi {worst[0]:.2e} g {worst[1]:.2e}; per cell phi {worst[2]:.2e} g {worst[3]:.2e}")
