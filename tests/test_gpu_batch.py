"""Batch plans (fmm_batch_plan_create / fmm_batch_solve): every field of an
uneven batch against the FP64 oracle, against single-field plans, across
graph replays and buffer changes, and the autotuner's report.

Bars: FP64 relative L2 <= 1e-12 against the oracle; FP32 phi <= 1e-5 and
g <= 1e-4 against the oracle of the float-rounded input.
"""
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


def _fields(sizes, dtype):
    import torch
    return [torch.as_tensor(fi.plummer_density(n, fi.batch_field_params(f))).to("cuda", dtype).contiguous()
            for f, n in enumerate(sizes)]


@pytest.mark.parametrize("p", [4, 6])
def test_fp64_batch_matches_oracle_and_single_plans(F, orc, p):
    import torch
    sizes = [16, 8, 32, 16, 64, 8, 32]
    _say(f"case batch fp64 p={p} sizes={sizes}")
    B = F.Batch(sizes, p, "fp64")
    info = B.info()
    assert info["count"] == len(sizes)
    assert info["bottom_tile"] in (8, 16) and info["m2l_grouping"] in (0, 1)
    assert all(t > 0 for t in info["tune_ms"])
    rhos = _fields(sizes, torch.float64)
    phis, gs = B.solve(rhos)
    torch.cuda.synchronize()
    for f, n in enumerate(sizes):
        rho = rhos[f].cpu().numpy()
        phi_o, g_o = orc.solve(rho, p)
        e1, e2 = rel(phis[f].cpu().numpy(), phi_o), rel(gs[f].cpu().numpy(), g_o)
        assert e1 < TOL64 and e2 < TOL64, (f, n, e1, e2)
        single = F.Plan(n, p)
        ps, g1 = single.solve(rhos[f])
        torch.cuda.synchronize()
        assert rel(phis[f].cpu().numpy(), ps.cpu().numpy()) < 1e-14
        assert rel(gs[f].cpu().numpy(), g1.cpu().numpy()) < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fmm2_batch_matches_single_plans(F, orc, precision):
    """FMM-2 (delta_l = 2) fields in one batch: each equals its single-field
    FMM-2 plan, and the FP64 ones the oracle's FMM-2."""
    import torch
    sizes = [32, 16, 64, 16, 32]
    _say(f"case batch fmm2 {precision} sizes={sizes}")
    dt = torch.float64 if precision == "fp64" else torch.float32
    B = F.Batch(sizes, 4, precision, delta_l=2)
    rhos = _fields(sizes, dt)
    phis, gs = B.solve(rhos)
    torch.cuda.synchronize()
    for f, n in enumerate(sizes):
        ps, g1 = F.Plan(n, 4, precision, delta_l=2).solve(rhos[f])
        torch.cuda.synchronize()
        assert rel(phis[f].double().cpu().numpy(), ps.double().cpu().numpy()) < 1e-6
        assert rel(gs[f].double().cpu().numpy(), g1.double().cpu().numpy()) < 1e-6
        if precision == "fp64":
            assert rel(phis[f].cpu().numpy(), ps.cpu().numpy()) < 1e-14
            phi_o, g_o = orc.solve(rhos[f].cpu().numpy(), 4, delta_l=2)
            assert rel(phis[f].cpu().numpy(), phi_o) < TOL64 and rel(gs[f].cpu().numpy(), g_o) < TOL64


def test_graph_replays_and_buffer_changes(F):
    """Replays of the captured graph, with eager work between them and new
    buffers on the third call, give the eager (profiled, directly launched)
    result every time."""
    import torch
    sizes = [32, 16, 64]
    _say("case batch graph replays")
    B = F.Batch(sizes, 5, "fp64", autotune=False)
    rhos = _fields(sizes, torch.float64)
    B.profile(True)
    ref, ref_g = B.solve(rhos)  # direct launches
    torch.cuda.synchronize()
    B.profile_read()
    B.profile(False)
    phis = [torch.empty_like(r) for r in rhos]
    gs = [torch.empty((3,) + tuple(r.shape), dtype=r.dtype, device="cuda") for r in rhos]
    for rep in range(4):
        if rep == 2:  # new buffers: the I/O table is uploaded again
            phis = [torch.empty_like(r) for r in rhos]
            gs = [torch.empty((3,) + tuple(r.shape), dtype=r.dtype, device="cuda") for r in rhos]
        for t in phis + gs:
            t.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()  # eager work between replays
        B.solve_into(rhos, phis, gs)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for f in range(len(sizes)):
            assert torch.equal(phis[f], ref[f]), (rep, f)
            assert torch.equal(gs[f], ref_g[f]), (rep, f)


def test_batch_without_some_accelerations(F, orc):
    import torch
    sizes = [16, 32]
    _say("case batch partial g")
    B = F.Batch(sizes, 4, "fp64", autotune=False)
    rhos = _fields(sizes, torch.float64)
    phis = [torch.empty_like(r) for r in rhos]
    g1 = torch.empty((3, 32, 32, 32), dtype=torch.float64, device="cuda")
    B.solve_into(rhos, phis, [None, g1])
    torch.cuda.synchronize()
    for f in range(2):
        phi_o, g_o = orc.solve(rhos[f].cpu().numpy(), 4)
        assert rel(phis[f].cpu().numpy(), phi_o) < TOL64
    assert rel(g1.cpu().numpy(), g_o) < TOL64


def test_fp32_batch(F, orc):
    """FP32 batch with the default policy: the 32^3 field keeps an FP64
    bottom (F = 4), the others run the FP32 matrix-core kernels."""
    import torch
    sizes = [32, 64, 128, 64]
    p = 4
    _say("case batch fp32 p=4")
    B = F.Batch(sizes, p, "fp32")
    rhos = _fields(sizes, torch.float32)
    phis, gs = B.solve(rhos)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for f, n in enumerate(sizes):
        rho = rhos[f].double().cpu().numpy()
        if n <= 64:
            phi_o, g_o = orc.solve(rho, p)
            phi_s, g_s = phis[f].double().cpu().numpy(), gs[f].double().cpu().numpy()
        else:
            cells = rng.choice(n ** 3, 40, replace=False)
            phi_o, g_o = orc.solve(rho, p, targets=cells)
            idx = torch.as_tensor(cells, device="cuda")
            phi_s = phis[f].reshape(-1)[idx].double().cpu().numpy()
            g_s = gs[f].reshape(3, -1)[:, idx].double().cpu().numpy()
        e1, e2 = rel(phi_s, phi_o), rel(g_s, g_o)
        c1 = float(np.abs(phi_s - phi_o).max() / np.abs(phi_o).max())
        c2 = float(np.abs(g_s - g_o).max() / np.abs(g_o).max())
        _say(f"  field {f} n={n}: phi {e1:.2e} g {e2:.2e}; per cell {c1:.2e} {c2:.2e}")
        assert e1 < 1e-5 and e2 < 1e-4, (f, n, e1, e2)
        assert c1 < 1e-5 and c2 < 1e-4, (f, n, c1, c2)


def test_single_and_batch_entry_points_are_distinct(F):
    import torch
    B = F.Batch([16], 3, "fp64", autotune=False)
    x = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    rc = F.lib().fmm_solve(B.ptr, x.data_ptr(), y.data_ptr(), None, None)
    assert rc == F.FMM_ERR_INVALID_ARG
    with pytest.raises(F.FmmError):
        B.solve_into([x], [x])  # rho and phi alias


def test_autotune_cache_round_trip(F, tmp_path):
    """opt.autotune_cache: the first plan times the candidates and appends
    its choice; a second plan with the same key reads it back without
    timing (same figures, no new line); a hand-written entry is obeyed; a
    different batch adds its own line."""
    import torch
    path = str(tmp_path / "tune.txt")
    sizes = [32, 64, 16]
    _say("case batch autotune cache")
    B1 = F.Batch(sizes, 4, "fp32", autotune_cache=path)
    i1 = B1.info()
    lines = open(path).read().splitlines()
    assert len(lines) == 1, lines
    key, rest = lines[0].split(" ", 1)
    assert "/p4/" in key and key.endswith("/n32,64,16")
    bz, grp = (int(x) for x in rest.split()[:2])
    assert (bz, grp) == (i1["bottom_tile"], i1["m2l_grouping"])
    B2 = F.Batch(sizes, 4, "fp32", autotune_cache=path)
    i2 = B2.info()
    assert len(open(path).read().splitlines()) == 1
    assert (i2["bottom_tile"], i2["m2l_grouping"]) == (bz, grp)
    assert np.allclose(i2["tune_ms"], i1["tune_ms"], rtol=0, atol=1e-6)
    # a hand-written choice for the key wins (the last line with the key)
    with open(path, "a") as fh:
        fh.write(f"{key} 8 1 9.5 9.5 9.5 9.5\n")
    B3 = F.Batch(sizes, 4, "fp32", autotune_cache=path)
    i3 = B3.info()
    assert (i3["bottom_tile"], i3["m2l_grouping"], i3["tune_ms"]) == (8, 1, [9.5] * 4)
    rhos = _fields(sizes, torch.float32)
    p1, g1 = B1.solve(rhos)
    p3, g3 = B3.solve(rhos)
    torch.cuda.synchronize()
    for f in range(len(sizes)):
        assert rel(p3[f].double().cpu().numpy(), p1[f].double().cpu().numpy()) < 1e-6
        assert rel(g3[f].double().cpu().numpy(), g1[f].double().cpu().numpy()) < 1e-6
    F.Batch([32, 32], 4, "fp32", autotune_cache=path)
    assert len(open(path).read().splitlines()) == 3


def test_fmm2_batch_times_only_its_tile_depth(F):
    """FMM-2 fields always run 16-deep bottom tiles: the autotuner times
    only those candidates and reports 16."""
    B = F.Batch([32, 16], 3, "fp64", delta_l=2)
    info = B.info()
    assert info["bottom_tile"] == 16
    assert info["tune_ms"][0] > 0 and info["tune_ms"][1] > 0
    assert info["tune_ms"][2] == 0 and info["tune_ms"][3] == 0


def test_per_field_completion_times(F):
    """fmm_batch_timestamps: each field's completion time lies inside the
    batch solve's own span, fields are reported in both graph replays and
    direct launches, and recording does not change the results."""
    import torch
    sizes = [32, 64, 16, 128, 32]
    _say("case batch per-field timestamps")
    B = F.Batch(sizes, 4, "fp32")
    rhos = _fields(sizes, torch.float32)
    ref, ref_g = B.solve(rhos)
    B.timestamps(True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for rep in range(3):  # the first captures a new graph
        a.record()
        phis, gs = B.solve(rhos)
        b.record()
    torch.cuda.synchronize()
    span = a.elapsed_time(b)
    ms = B.field_ms()
    _say(f"  batch {span:.3f} ms; fields {['%.3f' % x for x in ms]}")
    assert len(ms) == len(sizes) and all(0.0 < x <= span * 1.05 + 0.05 for x in ms), (ms, span)
    for f in range(len(sizes)):
        assert torch.equal(phis[f], ref[f]) and torch.equal(gs[f], ref_g[f])
    B.timestamps(False)
    with pytest.raises(F.FmmError):
        B.field_ms()
    single = F.Plan(16, 4)
    assert F.lib().fmm_batch_timestamps(single.ptr, 1) == F.FMM_ERR_INVALID_ARG
