#!/usr/bin/env python
"""Benchmark of the unigrid FMM solve on one MI355X.

Workload (default): 256^3 unigrid, isolated BC, p = 6, FP64; density = sum
of 256 seeded Plummer spheres (seed 256).  A step is one full solve (upward
pass, M2L/L2L over all levels, near field + L2P, M2P) producing phi and g,
with the density already resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
  value         grid cells per second (n^3 x steps / timed seconds)
  roofline      the dominant kernel (M2P) against the FP64 matrix-core peak,
                from HIP events recorded on the solve's stream
  cpu_baseline  the FP64 CPU oracle on this host, on a bounded sample (full
                upward pass + downward pass for a slab of cells), scaled to
                cells per second of a full solve
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid cells/s per FMM solve at 256^3 p=6 (FP64 vs mixed); M2L MFMA util"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0


PROFILE = os.path.join(ROOT, "profiles", "k_bottom_256cubed_p6_fp64.md")
KERNEL_SOURCES = ["fmm_impl.h", "fmm_mfma.h", "fmm_internal.h", "fmm_types.h"]


def profiled_traffic(n: int, p: int, prec: str, delta_l: int = 1):
    """HBM bytes per launch of the bottom kernel from the committed rocprofv3
    byte-counter summary, or None when it does not describe the current
    kernel sources or this workload."""
    import hashlib
    if (n, p, prec, delta_l) != (256, 6, "fp64", 1) or not os.path.exists(PROFILE):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        path = os.path.join(ROOT, "paper_2606_13793_amd", "csrc", f)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as fh:
            h.update(fh.read())
    fields = {}
    with open(PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", "#", " ")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    return int(fields["traffic_bytes_per_launch"])


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--p", type=int, default=6)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--delta-l", type=int, default=1, choices=[1, 2],
                    help="levels between the finest FMM level and the unigrid (2 = FMM-2)")
    ap.add_argument("--spheres", type=int, default=256)
    ap.add_argument("--seed", type=int, default=256)
    ap.add_argument("--cpu-planes", type=int, default=16,
                    help="unigrid planes of the oracle's downward-pass sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, equal-accuracy, adjoint and batch sections")
    ap.add_argument("--section", default=None,
                    choices=["mixed", "fmm2", "particles", "adjoint", "batch", "large", "huge", "cpu"],
                    help="run only this extra section (for profiling) and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one plain device-to-device copy of BYTES bytes (a known-size "
                         "reference dispatch for hardware byte counters)")
    return ap.parse_args()


def _event_ms(fn, steps: int, warmup: int) -> float:
    """Mean device milliseconds of fn() over `steps` calls on the current
    stream (HIP events), after `warmup` untimed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / steps


def _rel(a, b):
    import numpy as np
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cell_max(a, b):
    """Largest per-cell error relative to the largest reference value."""
    import numpy as np
    a, b = np.ravel(a), np.ravel(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def run_large(fi, fmm, costs, n: int = 512, p: int = 6) -> dict:
    """The same 256-sphere field at 512^3 (or 1024^3): solve time per policy
    and, at 4096 sampled cells, phi and g of the mixed policies against the
    FP64 solve and (up to 512^3, where the oracle's upward pass takes about
    15 s and 13 GB of host memory) every policy against the FP64 oracle, as
    relative L2 norms and as per-cell bounds max|err| / max|ref|.  At 1024^3
    a plan holds about 196 GiB and the FP64 input and outputs 40 GiB, so the
    density's temporaries are released first."""
    import numpy as np
    import torch
    log(f"extras: {n}^3 density")
    rho64 = fi.plummer_density(n, fi.multi_plummer_params(256, 256), device="cuda")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    N = n ** 3
    cells = np.sort(np.random.default_rng(11).choice(N, 4096, replace=False))
    idx = torch.as_tensor(cells, device="cuda")
    out = {"n": n, "p": p, "sampled_cells": len(cells)}
    phi_o = g_o = None
    if n <= 512:
        import oracle
        log(f"extras: {n}^3 oracle at {len(cells)} sampled cells")
        phi_o, g_o = oracle.solve(rho64.cpu().numpy(), p, targets=cells)
    ref = None
    for prec in ("fp64", "fp32", "bf16"):
        log(f"extras: {n}^3 {prec} plan")
        plan = fmm.Plan(n, p, prec)
        rho = rho64 if prec == "fp64" else rho64.float()
        phi = torch.empty((n, n, n), dtype=plan.io_dtype, device="cuda")
        g = torch.empty((3, n, n, n), dtype=plan.io_dtype, device="cuda")
        ms = _event_ms(lambda: plan.solve_into(rho, phi, g), 3, 1)
        ps = phi.reshape(-1)[idx].double().cpu().numpy()
        gs = g.reshape(3, -1)[:, idx].double().cpu().numpy()
        rec = {"ms_per_solve": ms, "cells_per_s": N / (ms * 1e-3),
               "useful_tflops": costs.solve_flops(n, p)["total"] / (ms * 1e-3) / 1e12}
        if prec == "fp64":
            ref = (ps, gs)
        else:
            rec["phi_rel_l2_vs_fp64"] = _rel(ps, ref[0])
            rec["g_rel_l2_vs_fp64"] = _rel(gs, ref[1])
            rec["phi_cell_max_vs_fp64"] = _cell_max(ps, ref[0])
            rec["g_cell_max_vs_fp64"] = _cell_max(gs, ref[1])
        if phi_o is not None:
            rec["phi_rel_l2_vs_oracle"] = _rel(ps, phi_o)
            rec["g_rel_l2_vs_oracle"] = _rel(gs, g_o)
            rec["phi_cell_max_vs_oracle"] = _cell_max(ps, phi_o)
            rec["g_cell_max_vs_oracle"] = _cell_max(gs, g_o)
        out[prec] = rec
        log(f"extras: {n}^3 {prec}: {ms:.1f} ms ({N / (ms * 1e-3):.3e} cells/s)"
            + (f", vs oracle phi {rec['phi_rel_l2_vs_oracle']:.2e} g {rec['g_rel_l2_vs_oracle']:.2e}"
               if phi_o is not None else ""))
        del plan, phi, g
        torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def run_cpu_oracle(fi, fmm, n: int = 128, p: int = 6) -> dict:
    """The CPU baseline workload (128^3, p = 6, FP64, 32 spheres, seed 128):
    the oracle's full solve on all host threads (measured, not
    extrapolated), a bounded sample on one thread (the full upward pass and
    the downward pass for 2 central planes), and the GPU solve of the same
    input beside them, compared with the oracle on every cell."""
    import numpy as np
    import torch
    import oracle
    rho = fi.plummer_density(n, fi.multi_plummer_params(32, 128))
    nthr = oracle.threads()
    log(f"cpu oracle: full {n}^3 p={p} solve on {nthr} threads")
    t0 = time.perf_counter()
    phi_o, g_o = oracle.solve(rho, p)
    t_all = time.perf_counter() - t0
    planes = 2
    i0 = n // 2 - planes // 2
    cells = np.arange(i0 * n * n, (i0 + planes) * n * n, dtype=np.int64)
    oracle.set_threads(1)
    try:
        log(f"cpu oracle: one thread, upward pass + {planes} planes")
        _, _, t_up1, t_down1, _ = oracle.solve_timed(rho, p, cells)
    finally:
        oracle.set_threads(nthr)
    t_one = t_up1 + t_down1 * n ** 3 / len(cells)
    plan = fmm.Plan(n, p, "fp64")
    r = torch.as_tensor(rho, device="cuda")
    phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    g = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    for _ in range(3):
        plan.solve_into(r, phi, g)
    for a, b in evs:
        a.record()
        plan.solve_into(r, phi, g)
        b.record()
    torch.cuda.synchronize()
    gpu_ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
    ph, gg = phi.cpu().numpy(), g.cpu().numpy()
    out = {
        "workload": f"{n}^3 unigrid, p={p}, FP64, phi+g, 32 Plummer spheres (seed 128)",
        "cpu_model": cpu_model(),
        "all_threads": {"threads": nthr, "seconds": t_all, "cells_per_s": n ** 3 / t_all,
                        "sample": "the full solve, measured"},
        "one_thread": {"threads": 1, "seconds_estimated": t_one, "cells_per_s": n ** 3 / t_one,
                       "sample": f"full upward pass ({t_up1:.2f} s) + downward pass for {planes} central planes "
                                 f"({len(cells)} cells, {t_down1:.2f} s), scaled to the full grid"},
        "thread_speedup": t_one / t_all,
        "gpu_fp64_ms_median": gpu_ms,
        "gpu_cells_per_s": n ** 3 / (gpu_ms * 1e-3),
        "gpu_vs_cpu_all_threads": t_all / (gpu_ms * 1e-3),
        "dense_parity": {"phi_rel_l2": _rel(ph, phi_o), "g_rel_l2": _rel(gg, g_o),
                         "phi_max_over_max": float(np.abs(ph - phi_o).max() / np.abs(phi_o).max()),
                         "g_max_over_max": float(np.abs(gg - g_o).max() / np.abs(g_o).max())},
    }
    log(f"cpu oracle: {t_all:.1f} s on {nthr} threads, ~{t_one:.0f} s on one; GPU {gpu_ms:.2f} ms; "
        f"dense parity phi {out['dense_parity']['phi_rel_l2']:.2e}")
    return out


def paper_flop_table(costs) -> dict:
    """The paper's per-operator counts (Sec. 4, p = 3, nmax = 2) beside this
    library's counting of the same operators."""
    ours = costs.operator_counts(3, 2)
    tab = {}
    for op, paper in costs.PAPER_SEC4.items():
        v = ours[op]
        tab[op] = {"paper": paper, "ours_phi_only": v[0] if isinstance(v, tuple) else v,
                   "ours_phi_and_g": v[1] if isinstance(v, tuple) else v}
    return tab


def run_extras(args, rho64, fi, fmm, costs,
               sections=("mixed", "fmm2", "particles", "adjoint", "batch", "large", "cpu")) -> dict:
    """The other measured rows at the same workload: mixed precision (with
    the equal-accuracy comparison against FP64 at lower order), the adjoint,
    and the uneven 96-field batch against a loop of single solves."""
    import numpy as np
    import torch
    import oracle
    n, P = args.n, args.p
    N = n ** 3
    out = {}
    # sampled cells for errors against the FP64 oracle and the direct sum
    cells = np.sort(np.random.default_rng(7).choice(N, 64, replace=False))
    idx = torch.as_tensor(cells, device="cuda")
    rho_host = rho64.cpu().numpy()
    phi_d = None
    if "mixed" in sections or "fmm2" in sections:
        log("extras: direct sum at 64 sampled cells")
        phi_d, _ = oracle.direct(rho_host, targets=cells)

    def sampled(plan, rho):
        phi = torch.empty((n, n, n), dtype=plan.io_dtype, device="cuda")
        g = torch.empty((3, n, n, n), dtype=plan.io_dtype, device="cuda")
        plan.solve_into(rho, phi, g)
        torch.cuda.synchronize()
        return phi.reshape(-1)[idx].double().cpu().numpy(), g.reshape(3, -1)[:, idx].double().cpu().numpy()

    # FP64 at orders 1..P: time and truncation error against the direct sum
    fp64 = {}
    for q in (range(1, P + 1) if "mixed" in sections else ()):
        plan = fmm.Plan(n, q, "fp64")
        phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        g = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        ms = _event_ms(lambda: plan.solve_into(rho64, phi, g), 5, 2)
        ps, _ = sampled(plan, rho64)
        fp64[q] = {"ms_per_solve": ms, "phi_err_vs_direct": _rel(ps, phi_d)}
        del plan, phi, g
        log(f"extras: fp64 p={q}: {ms:.2f} ms, error vs direct {fp64[q]['phi_err_vs_direct']:.3e}")
    if fp64:
        out["fp64_by_order"] = fp64
    # the paper's own expansion orders: locals p = 3, multipoles nmax = 2
    if "mixed" in sections and P >= 3:
        plan = fmm.Plan(n, 3, "fp64", nmax=2)
        phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        g = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        ms = _event_ms(lambda: plan.solve_into(rho64, phi, g), 5, 2)
        ps, _ = sampled(plan, rho64)
        out["paper_orders"] = {"p": 3, "nmax": 2, "ms_per_solve": ms, "phi_err_vs_direct": _rel(ps, phi_d)}
        del plan, phi, g
        log(f"extras: fp64 p=3 nmax=2: {ms:.2f} ms, error vs direct {out['paper_orders']['phi_err_vs_direct']:.3e}")
    # FMM-2 (finest FMM level two above the unigrid, App. A): time and error
    # at order P and at the paper's orders, and the FMM-1 vs FMM-2 potential
    # difference of a CIC point charge at the box centre on the midplane
    c = fi.cell_centres(n)
    if "fmm2" in sections and P >= 3:
        fmm2 = {}
        for q, nm in ((P, None), (3, 2)):
            plan = fmm.Plan(n, q, "fp64", nmax=nm, delta_l=2)
            phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
            g = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
            ms = _event_ms(lambda: plan.solve_into(rho64, phi, g), 5, 2)
            # the bottom kernel's own time (HIP events per stage) against its useful flops
            plan.profile(True)
            plan.profile_read()
            for _ in range(5):
                plan.solve_into(rho64, phi, g)
            torch.cuda.synchronize()
            bot_ms = plan.profile_read()["bottom"][0] / 5
            plan.profile(False)
            bot_tf = costs.solve_flops(n, q, nm, delta_l=2)["bottom"] / (bot_ms * 1e-3) / 1e12
            ps, _ = sampled(plan, rho64)
            key = f"p{q}" + ("" if nm is None else f"_nmax{nm}")
            fmm2[key] = {"ms_per_solve": ms, "cells_per_s": N / (ms * 1e-3), "phi_err_vs_direct": _rel(ps, phi_d),
                         "bottom_ms": bot_ms, "bottom_tflops": bot_tf, "bottom_frac_of_fp64_peak": bot_tf / 78.6}
            del plan, phi, g
            log(f"extras: fmm-2 {key}: {ms:.2f} ms (bottom {bot_ms:.2f} ms, {bot_tf:.1f} TF/s), "
                f"error vs direct {fmm2[key]['phi_err_vs_direct']:.3e}")
        pc = torch.as_tensor(fi.point_charge_cic(n)).cuda()
        s1 = fmm.Plan(n, 3, "fp64", nmax=2).solve(pc, want_g=False)[0][:, :, n // 2].cpu().numpy()
        s2 = fmm.Plan(n, 3, "fp64", nmax=2, delta_l=2).solve(pc, want_g=False)[0][:, :, n // 2].cpu().numpy()
        d = np.abs(s2 - s1) / np.abs(s1)
        fmm2["point_charge_fmm1_vs_fmm2"] = {"p": 3, "nmax": 2, "slice": "midplane through the charge",
                                             "max": float(d.max()), "p99": float(np.percentile(d, 99)),
                                             "p90": float(np.percentile(d, 90))}
        # against the exact potential -1/r of the point, over the whole slice
        # (the charge's own cells included)
        r = np.sqrt((c[:, None] - 0.5) ** 2 + (c[None, :] - 0.5) ** 2 + (c[n // 2] - 0.5) ** 2)
        for key, sl in (("fmm1", s1), ("fmm2", s2)):
            e = np.abs(sl + 1.0 / r) * r
            fmm2["point_charge_fmm1_vs_fmm2"][f"{key}_vs_exact_p90"] = float(np.percentile(e, 90))
            fmm2["point_charge_fmm1_vs_fmm2"][f"{key}_vs_exact_p99"] = float(np.percentile(e, 99))
        del pc
        log(f"extras: point charge FMM-1 vs FMM-2: max {d.max():.3e}, p99 {np.percentile(d, 99):.3e}")
        out["fmm2"] = fmm2
    if "particles" in sections:
        # the paper's two uniform spheres (Sec. 3), scaled to the unit box:
        # 16M particles, CIC deposit on the GPU, FMM-1 and FMM-2 at the paper's
        # orders, errors against the exact potential on the midplane
        pos, m = fi.two_spheres_particles(1 << 24)
        pos_t = torch.as_tensor(pos).cuda()
        m_t = torch.as_tensor(m).cuda()
        rho_s = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
        dep_random_ms = _event_ms(lambda: (rho_s.zero_(), fmm.deposit_cic(n, pos_t, m_t, rho=rho_s)), 5, 2)
        # the same particles in cell order, as AMR codes keep them
        order = torch.as_tensor(fi.cell_order(pos, n)).cuda()
        pos_t, m_t = pos_t[order].contiguous(), m_t[order].contiguous()
        del order
        dep_ms = _event_ms(lambda: (rho_s.zero_(), fmm.deposit_cic(n, pos_t, m_t, rho=rho_s)), 5, 2)
        pts = np.stack(np.meshgrid(c, c, [c[n // 2]], indexing="ij"), -1).reshape(-1, 3)
        exact = fi.two_spheres_potential(pts).reshape(n, n)
        spheres = {"particles": int(len(m)), "zero_and_deposit_ms_cell_order": dep_ms,
                   "zero_and_deposit_ms_random_order": dep_random_ms, "p": 3, "nmax": 2,
                   "slice": "midplane through both centres"}
        for dl in (1, 2):
            ph = fmm.Plan(n, 3, "fp64", nmax=2, delta_l=dl).solve(rho_s, want_g=False)[0]
            e = np.abs(ph[:, :, n // 2].cpu().numpy() - exact) / np.abs(exact)
            spheres[f"fmm{dl}_p90"] = float(np.percentile(e, 90))
            spheres[f"fmm{dl}_p99"] = float(np.percentile(e, 99))
            del ph
        # App. C: force magnitudes inside the spheres (cells whose centres lie
        # inside), the finite-difference force from phi and the solve's g
        X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
        pts3 = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
        inside = np.zeros(len(pts3), bool)
        for cc, rr in fi.TWO_SPHERES:
            inside |= np.linalg.norm(pts3 - np.asarray(cc), axis=1) < rr
        sel = np.nonzero(inside)[0]
        sel_t = torch.as_tensor(sel).cuda()
        fexact = np.linalg.norm(fi.two_spheres_force(pts3[sel]), axis=0)
        del X, Y, Z, pts3, inside
        ph, gg = fmm.Plan(n, 3, "fp64", nmax=2).solve(rho_s)
        fd_ms = _event_ms(lambda: fmm.fd_force(ph), 10, 2)
        for name, force in (("fd", fmm.fd_force(ph)), ("g", gg)):
            mag = torch.linalg.vector_norm(force.reshape(3, -1)[:, sel_t], dim=0).cpu().numpy()
            e = np.abs(mag - fexact) / fexact
            spheres[f"force_{name}_inside_p90"] = float(np.percentile(e, 90))
            spheres[f"force_{name}_inside_p99"] = float(np.percentile(e, 99))
        spheres["fd_force_ms"] = fd_ms
        spheres["fd_force_GBps_at_32B_per_cell"] = 32 * N / (fd_ms * 1e-3) / 1e9
        del ph, gg, sel_t
        del pos_t, m_t, rho_s
        out["two_spheres"] = spheres
        log(f"extras: two spheres force inside, P90: FD {spheres['force_fd_inside_p90']:.2e}, "
            f"g {spheres['force_g_inside_p90']:.2e}; FD force {fd_ms:.3f} ms")
        log(f"extras: two spheres: deposit {dep_ms:.2f} ms in cell order, {dep_random_ms:.2f} ms in random order; "
            f"P90/P99 FMM-1 {spheres['fmm1_p90']:.2e}/"
            f"{spheres['fmm1_p99']:.2e}, FMM-2 {spheres['fmm2_p90']:.2e}/{spheres['fmm2_p99']:.2e}")
    # mixed precision at order P
    mixed = {}
    if "mixed" in sections:
        phi_o, g_o = oracle.solve(rho64.float().double().cpu().numpy(), P, targets=cells)
    for prec in (("fp32", "bf16") if "mixed" in sections else ()):
        plan = fmm.Plan(n, P, prec)
        rho = rho64.float()
        phi = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        g = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        ms = _event_ms(lambda: plan.solve_into(rho, phi, g), 10, 3)
        ps, gs = sampled(plan, rho)
        err_d = _rel(ps, phi_d)
        # equal accuracy: the lowest FP64 order at least as accurate
        eq = next((q for q in range(1, P + 1) if fp64[q]["phi_err_vs_direct"] <= err_d), P)
        mixed[prec] = {
            "ms_per_solve": ms,
            "cells_per_s": N / (ms * 1e-3),
            "phi_rel_l2_vs_fp64_oracle": _rel(ps, phi_o),
            "g_rel_l2_vs_fp64_oracle": _rel(gs, g_o),
            "phi_err_vs_direct": err_d,
            "equal_accuracy_fp64_order": eq,
            "equal_accuracy_fp64_cells_per_s": N / (fp64[eq]["ms_per_solve"] * 1e-3),
            "speedup_vs_fp64_same_order": fp64[P]["ms_per_solve"] / ms,
            "speedup_vs_fp64_equal_accuracy": fp64[eq]["ms_per_solve"] / ms,
        }
        log(f"extras: {prec} p={P}: {ms:.2f} ms, err vs direct {err_d:.3e}, equal-accuracy FP64 p={eq}")
        del plan, phi, g
    if mixed:
        out["mixed_precision"] = mixed
    # adjoint at the workload
    adj = {}
    for prec in (("fp64", "fp32") if "adjoint" in sections else ()):
        plan = fmm.Plan(n, P, prec)
        dt = torch.float64 if prec == "fp64" else torch.float32
        dphi = torch.randn((n, n, n), dtype=dt, device="cuda")
        dg = torch.randn((3, n, n, n), dtype=dt, device="cuda")
        plan.backward(dphi, dg)  # allocates the adjoint workspace
        ms = _event_ms(lambda: plan.backward(dphi, dg), 5, 1)
        adj[prec] = {"ms_per_backward": ms, "cells_per_s": N / (ms * 1e-3)}
        log(f"extras: backward {prec}: {ms:.2f} ms")
        del plan, dphi, dg
    if adj:
        out["adjoint"] = adj
    torch.cuda.empty_cache()
    if "cpu" in sections:
        out["cpu_oracle"] = run_cpu_oracle(fi, fmm)
        torch.cuda.empty_cache()
    if "large" in sections:
        out["large_512"] = run_large(fi, fmm, costs)
    if "huge" in sections:
        out["huge_1024"] = run_large(fi, fmm, costs, n=1024)
    if "batch" not in sections:
        return out
    # the uneven batch (96 fields: 55 x 32^3, 27 x 64^3, 14 x 128^3), FP32
    sizes = fi.batch_sizes()
    cells_b = sum(m ** 3 for m in sizes)
    rhos = [fi.plummer_density(m, fi.batch_field_params(f), device="cuda").float() for f, m in enumerate(sizes)]
    batched = {"fields": len(sizes), "cells": cells_b}
    for q in (4, 6):
        B = fmm.Batch(sizes, q, "fp32")
        phis = [torch.empty((m, m, m), dtype=torch.float32, device="cuda") for m in sizes]
        gs = [torch.empty((3, m, m, m), dtype=torch.float32, device="cuda") for m in sizes]
        ms_b = _event_ms(lambda: B.solve_into(rhos, phis, gs), 5, 2)
        info = B.info()
        # per-field latency: device wall-clock time from the start of a
        # graph-replayed batch solve to the end of each field's last block
        B.timestamps(True)
        for _ in range(3):
            B.solve_into(rhos, phis, gs)
        fms = np.array(B.field_ms())
        B.timestamps(False)
        lat = {"all": {"min_ms": float(fms.min()), "median_ms": float(np.median(fms)), "max_ms": float(fms.max())}}
        for m in sorted(set(sizes)):
            sel = fms[[i for i, x in enumerate(sizes) if x == m]]
            lat[f"{m}^3"] = {"fields": int(len(sel)), "min_ms": float(sel.min()), "median_ms": float(np.median(sel)),
                             "max_ms": float(sel.max())}
        del B
        singles = [fmm.Plan(m, q, "fp32") for m in sizes]
        ms_l = _event_ms(lambda: [pl.solve_into(r, ph, gg) for pl, r, ph, gg in zip(singles, rhos, phis, gs)], 3, 1)
        del singles
        fl = sum(costs.solve_flops(m, q)["total"] for m in sizes)
        batched[f"p{q}"] = {
            "ms_per_batch": ms_b,
            "cells_per_s": cells_b / (ms_b * 1e-3),
            "useful_tflops": fl / (ms_b * 1e-3) / 1e12,
            "loop_of_single_solves_ms": ms_l,
            "speedup_vs_loop": ms_l / ms_b,
            "autotuned": {"bottom_tile": info["bottom_tile"], "m2l_grouping": info["m2l_grouping"],
                          "candidate_ms": info["tune_ms"]},
            "field_latency": lat,
        }
        log(f"extras: batch p={q}: {ms_b:.2f} ms ({cells_b / (ms_b * 1e-3):.3e} cells/s), loop {ms_l:.2f} ms")
        torch.cuda.empty_cache()
    out["batched"] = batched
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the solver "
              "runs on one GPU (its multi-GPU sharding is designed but not built)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import fmm_inputs as fi
    from paper_2606_13793_amd import costs, fmm

    if not os.path.exists(fmm.LIB_PATH):
        log("libfmm.so missing, building")
        from paper_2606_13793_amd import build
        build.build()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")

    n, p, prec, dl = args.n, args.p, args.precision, args.delta_l
    dev = "cuda"
    log(f"workload n={n} p={p} precision={prec} delta_l={dl} spheres={args.spheres} seed={args.seed}")
    params = fi.multi_plummer_params(args.spheres, args.seed)
    rho64 = fi.plummer_density(n, params, device=dev)
    torch.cuda.synchronize()
    if args.section:
        res = run_extras(args, rho64, fi, fmm, costs, sections=(args.section,))
        print(json.dumps({"section": args.section, "config": {"n": n, "p": p}, **res}), flush=True)
        return
    plan = fmm.Plan(n, p, prec, delta_l=dl)
    rho = rho64 if prec == "fp64" else rho64.float()
    phi = torch.empty((n, n, n), dtype=plan.io_dtype, device=dev)
    g = torch.empty((3, n, n, n), dtype=plan.io_dtype, device=dev)
    log(f"plan ready: {plan.workspace_bytes() / 2**30:.2f} GiB workspace")
    if args.copy_calibration:
        cnt = args.copy_calibration // 8
        src = torch.ones(cnt, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # one elementwise kernel: reads and writes cnt doubles
        torch.cuda.synchronize()
        log(f"calibration copy: {cnt * 8} bytes read, {cnt * 8} bytes written")
        del src, dst

    for _ in range(args.warmup):
        plan.solve_into(rho, phi, g)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve_into(rho, phi, g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    prof = plan.profile_read()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    cells_per_s = n ** 3 * args.steps / elapsed
    log(f"timed {args.steps} solves: {ms_per_step:.3f} ms/solve, {cells_per_s:.4e} cells/s")
    # spread of single solves (HIP events around each, after the timed
    # region): median and mean +- 1 sigma, the paper's timing protocol
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in evs:
        a.record()
        plan.solve_into(rho, phi, g)
        b.record()
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in evs])
    spread = {"samples": len(per), "median_ms": float(np.median(per)), "mean_ms": float(per.mean()),
              "std_ms": float(per.std(ddof=1)) if len(per) > 1 else 0.0, "min_ms": float(per.min()),
              "max_ms": float(per.max())}
    log(f"single solves: median {spread['median_ms']:.3f} ms, mean {spread['mean_ms']:.3f} +- {spread['std_ms']:.3f} ms")

    flops = costs.solve_flops(n, p, delta_l=dl)
    stage_flops = {"p2m": flops["p2m"], "m2m": flops["m2m"], "m2l": flops["m2l"], "bottom": flops["bottom"]}
    if dl == 1:  # level F - 1 is formed by the P2M stage, from the density
        stage_flops["p2m"] += flops["m2m_top"]
        stage_flops["m2m"] -= flops["m2m_top"]
    stages = {}
    for name, (ms, launches) in prof.items():
        if launches or ms:
            stages[name] = {"ms_per_step": ms / args.steps, "launches_per_step": launches / args.steps}
            if name in stage_flops and ms > 0:
                stages[name]["tflops"] = stage_flops[name] * args.steps / (ms * 1e-3) / 1e12
    bot_ms, bot_launches = prof["bottom"]
    bot_avg_s = bot_ms * 1e-3 / max(bot_launches, 1)
    bot_tflops = stage_flops["bottom"] / bot_avg_s / 1e12
    peak = PEAK_TFLOPS[prec]
    roofline = {
        "kernel": "k_bottom: M2P + L2P + near field",
        "bound": "mfma",
        "achieved": round(bot_tflops, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(bot_tflops / peak, 4),
        "traffic": profiled_traffic(n, p, prec, dl),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "avg_launch_ms": round(bot_avg_s * 1e3, 4),
        "flops_per_launch": stage_flops["bottom"],
        "m2p_pairs_per_launch": costs.m2p_pairs(n, dl),
    }
    m2l_ms, m2l_launches = prof["m2l"]
    solve_tflops = flops["total"] / (elapsed / args.steps) / 1e12
    extra = {
        "m2l": {"tflops": round(stage_flops["m2l"] / (m2l_ms * 1e-3 / args.steps) / 1e12, 3) if m2l_ms else None,
                "frac_of_peak": round(stage_flops["m2l"] / (m2l_ms * 1e-3 / args.steps) / 1e12 / peak, 4) if m2l_ms else None,
                "launches_per_step": m2l_launches / args.steps},
        "solve_tflops": round(solve_tflops, 3),
        "solve_frac_of_peak": round(solve_tflops / peak, 4),
        "useful_flops_per_solve": flops["total"],
    }

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        planes = args.cpu_planes
        i0 = n // 2 - planes // 2
        cells = np.arange(i0 * n * n, (i0 + planes) * n * n, dtype=np.int64)
        log(f"cpu baseline: oracle upward pass + downward on {planes} planes ({len(cells)} cells)")
        rho_host = rho64.cpu().numpy() if prec == "fp64" else rho.double().cpu().numpy()
        phi_o, g_o, t_up, t_down, threads = oracle.solve_timed(rho_host, p, cells, delta_l=dl)
        t_full = t_up + t_down * (n ** 3 / len(cells))
        cpu_model_name = cpu_model()
        cpu = {
            "value": n ** 3 / t_full,
            "unit": "cells/s",
            "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle on this host ({cpu_model_name}), {threads} OpenMP threads: full upward pass ({t_up:.2f} s) + "
                       f"downward pass for {planes} central unigrid planes ({len(cells)} cells, {t_down:.2f} s); "
                       f"full solve = upward + downward x n^3/{len(cells)} = {t_full:.1f} s"),
        }
        log(f"cpu baseline: {cpu['value']:.4e} cells/s ({threads} threads)")
        idx = torch.as_tensor(cells, device=dev)
        phi_s = phi.reshape(-1)[idx].double().cpu().numpy()
        g_s = g.reshape(3, -1)[:, idx].double().cpu().numpy()
        parity = {
            "cells": int(len(cells)),
            "phi_rel_l2": float(np.linalg.norm(phi_s - phi_o) / np.linalg.norm(phi_o)),
            "g_rel_l2": float(np.linalg.norm(g_s - g_o) / np.linalg.norm(g_o)),
        }
        log(f"parity on the slab: {parity}")

    extras = {}
    if not args.no_extras and prec == "fp64" and dl == 1:
        del plan, phi, g
        torch.cuda.empty_cache()
        extras = run_extras(args, rho64, fi, fmm, costs)

    out = {
        "metric": METRIC,
        "value": cells_per_s,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec],
        "data": "synthetic",
        "config": {
            "workload": (f"{n}^3 unigrid FMM solve, isolated BC, p={p}, {prec}, phi+g, "
                         + ("" if dl == 1 else "FMM-2 (finest FMM level two above the unigrid), ")
                         + f"{args.spheres}-sphere multi-Plummer density (seed {args.seed})"),
            "n": n, "p": p, "precision": prec, "delta_l": dl, "spheres": args.spheres, "seed": args.seed,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stages": stages,
        "kernels": extra,
        "parity_vs_oracle": parity,
        "solve_ms_spread": spread,
        "paper_flop_table": paper_flop_table(costs),
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
