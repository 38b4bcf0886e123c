"""fmm_solve_backward_noalloc (the backward pass in the library's static
workspace) against fmm_solve_backward, through the C ABI.

Two calls in a row, the second on a smaller plan (so it finds the first
call's contents in the static array), in FP64 (bar: relative L2 and per-cell
max|err|/max|ref| <= 1e-12, the FP64 tolerance; the two entry points differ
only in the rounding order of the transposed M2L's sums), one FP32 plan (the
FP32 adjoint bar, 1e-4), an FMM-2 plan, and a plan too large for the array,
which must be rejected before anything is enqueued.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2606_13793_amd import fmm
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return fmm


def _cmp(got, ref):
    got, ref = got.double().cpu().numpy().ravel(), ref.double().cpu().numpy().ravel()
    return (float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            float(np.abs(got - ref).max() / np.abs(ref).max()))


def _both(F, n, p, precision, seed, coarse=4, delta_l=1):
    """(noalloc result, regular result) for one plan and seeded cotangents."""
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = F.Plan(n, p, precision, coarse_fp64_levels=coarse, delta_l=delta_l)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    dphi = torch.randn((n, n, n), dtype=dt, device="cuda", generator=gen)
    dg = torch.randn((3, n, n, n), dtype=dt, device="cuda", generator=gen)
    out = torch.full((n, n, n), float("nan"), dtype=dt, device="cuda")
    L = F.lib()
    stream = torch.cuda.current_stream().cuda_stream
    rc = L.fmm_solve_backward_noalloc(plan.ptr, dphi.data_ptr(), dg.data_ptr(), out.data_ptr(), stream)
    assert rc == F.FMM_OK, F.last_error()
    ref = plan.backward(dphi, dg)
    torch.cuda.synchronize()
    return out, ref, plan


def test_noalloc_matches_backward_two_calls(F):
    _say("case noalloc fp64 n=64 p=6, then n=32 p=4")
    out, ref, _ = _both(F, 64, 6, "fp64", 1)
    e = _cmp(out, ref)
    _say(f"  n=64 p=6: rel L2 {e[0]:.2e}, per cell {e[1]:.2e}")
    assert e[0] <= 1e-12 and e[1] <= 1e-12, e
    # the second call, on a smaller plan, starts from the first call's contents
    out, ref, _ = _both(F, 32, 4, "fp64", 2)
    e = _cmp(out, ref)
    _say(f"  n=32 p=4: rel L2 {e[0]:.2e}, per cell {e[1]:.2e}")
    assert e[0] <= 1e-12 and e[1] <= 1e-12, e


def test_noalloc_fp32(F):
    _say("case noalloc fp32 n=32 p=6 (every level FP32)")
    out, ref, _ = _both(F, 32, 6, "fp32", 3, coarse=0)
    e = _cmp(out, ref)
    _say(f"  rel L2 {e[0]:.2e}, per cell {e[1]:.2e}")
    assert e[0] <= 1e-4 and e[1] <= 1e-4, e


def test_noalloc_fmm2(F):
    _say("case noalloc fp64 FMM-2 n=64 p=6")
    out, ref, _ = _both(F, 64, 6, "fp64", 4, delta_l=2)
    e = _cmp(out, ref)
    _say(f"  rel L2 {e[0]:.2e}, per cell {e[1]:.2e}")
    assert e[0] <= 1e-12 and e[1] <= 1e-12, e


def test_noalloc_rejects_plans_too_large(F):
    import torch
    _say("case noalloc rejects n=128 p=6")
    n = 128
    plan = F.Plan(n, 6, "fp64")
    x = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    y = torch.full((n, n, n), 7.0, dtype=torch.float64, device="cuda")
    rc = F.lib().fmm_solve_backward_noalloc(plan.ptr, x.data_ptr(), None, y.data_ptr(), None)
    assert rc == F.FMM_ERR_INVALID_ARG
    assert "static workspace" in F.last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())  # nothing ran
    assert F.lib().fmm_solve_backward_noalloc(None, None, None, None, None) == F.FMM_ERR_INVALID_ARG
