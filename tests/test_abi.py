"""The C-ABI library: it loads, exports every symbol include/fmm.h declares,
and rejects invalid arguments before touching a device.  No compute calls."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


@pytest.fixture(scope="module")
def F():
    from paper_2606_13793_amd import fmm
    if not os.path.exists(fmm.LIB_PATH):
        from paper_2606_13793_amd import build
        build.build()
    return fmm


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_0-9]+)\s*\(", text)))


def test_header_lists_the_boundary():
    names = header_functions()
    for required in ("fmm_plan_create", "fmm_solve", "fmm_solve_backward", "fmm_plan_destroy", "fmm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(F):
    L = F.lib()
    names = header_functions()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(F.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fmm_\w+)", out))
    assert set(names) <= exported


def _offload_targets(path):
    """Target IDs of every device code object in a HIP shared library built
    here: the .hip_fatbin section holds one clang offload bundle per
    translation unit ("__CLANG_OFFLOAD_BUNDLE__", the entry count, then per
    entry its offset, size, ID length and ID)."""
    import struct
    out = subprocess.run(["readelf", "-S", "-W", path], capture_output=True, text=True, check=True).stdout
    sec = None
    for line in out.splitlines():
        parts = line.split()
        if ".hip_fatbin" in parts:
            i = parts.index(".hip_fatbin")
            sec = int(parts[i + 3], 16), int(parts[i + 4], 16)
    assert sec, "no .hip_fatbin section"
    with open(path, "rb") as fh:
        fh.seek(sec[0])
        data = fh.read(sec[1])
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    ids, bundles, pos = [], 0, data.find(magic)
    while pos >= 0:
        bundles += 1
        q = pos + len(magic)
        (count,) = struct.unpack_from("<Q", data, q)
        q += 8
        for _ in range(count):
            _off, size, idlen = struct.unpack_from("<QQQ", data, q)
            q += 24
            ids.append((data[q:q + idlen].decode(), size))
            q += idlen
        pos = data.find(magic, q)
    return bundles, ids


def test_library_is_built_for_gfx950(F):
    """Every device code object of libfmm.so is for gfx950 (the host entries
    of the bundles carry no code), one bundle per .hip translation unit."""
    bundles, ids = _offload_targets(F.LIB_PATH)
    from paper_2606_13793_amd import build
    assert bundles == sum(src.endswith(".hip") for src in build.SOURCES), (bundles, ids)
    device = [(t, n) for t, n in ids if not t.startswith("host-")]
    assert device and all(t.startswith("hipv4-amdgcn-amd-amdhsa--gfx950") and n > 0 for t, n in device), ids
    assert all(n == 0 for t, n in ids if t.startswith("host-")), ids
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", F.LIB_PATH], capture_output=True, text=True) \
        if os.path.exists("/opt/rocm/bin/roc-obj-ls") else None
    if out is not None and out.returncode == 0:
        assert "gfx950" in out.stdout


def _create(F, n, p, isolated=1, **opt):
    L = F.lib()
    o = F.FmmOptions()
    L.fmm_options_default(ctypes.byref(o))
    for k, v in opt.items():
        setattr(o, k, v)
    ptr = L.fmm_plan_create_ex(n, p, isolated, ctypes.byref(o))
    return ptr, L.fmm_last_status(), F.last_error()


@pytest.mark.parametrize("n,p,iso,code,text", [
    (12, 4, 1, -1, "power of two"),
    (4, 4, 1, -1, "power of two"),
    (2048, 4, 1, -1, "power of two"),
    (16, 0, 1, -1, "p must be"),
    (16, 9, 1, -1, "p must be"),
    (16, 4, 0, -2, "isolated"),
    (16, 4, 2, -1, "isolated"),
])
def test_invalid_sizes_rejected_without_device(F, n, p, iso, code, text):
    ptr, status, msg = _create(F, n, p, iso)
    assert not ptr
    assert status == code
    assert text in msg


@pytest.mark.parametrize("opt,code", [
    ({"delta_l": 3}, -2),
    ({"delta_l": 0}, -2),
    ({"nmax": 7}, -1),
    ({"nmax": -3}, -1),
    ({"precision": 5}, -1),
    ({"struct_size": 4}, -1),
    ({"coarse_fp64_levels": -1}, -1),
    ({"bottom_tile": 4}, -1),
    ({"bottom_tile": 32}, -1),
    ({"bottom_tile": 8, "delta_l": 2}, -1),
])
def test_invalid_options_rejected(F, opt, code):
    ptr, status, msg = _create(F, 16, 4, **opt)
    assert not ptr and status == code and msg


def test_delta_l_2_needs_n_16(F):
    ptr, status, msg = _create(F, 8, 4, delta_l=2)
    assert not ptr and status == -1 and "n >= 16" in msg


def test_workspace_cap_reports_out_of_memory():
    code = (
        "import ctypes, os\n"
        "from paper_2606_13793_amd import fmm\n"
        "L = fmm.lib()\n"
        "p = L.fmm_plan_create(256, 6, 1)\n"
        "print(bool(p), L.fmm_last_status(), fmm.last_error())\n"
    )
    env = dict(os.environ, FMM_TEST_MAX_WORKSPACE="1000000")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("False -3"), out.stdout
    assert "FMM_TEST_MAX_WORKSPACE" in out.stdout


def test_null_arguments(F):
    L = F.lib()
    assert L.fmm_solve(None, None, None, None, None) == -1
    assert "plan is NULL" in F.last_error()
    assert L.fmm_solve_backward(None, None, None, None, None) == -1
    assert L.fmm_plan_workspace_bytes(None) == 0
    L.fmm_plan_destroy(None)  # NULL-safe
    assert L.fmm_options_default(None) == -1
    assert L.fmm_last_error() is not None


def test_options_default(F):
    o = F.FmmOptions()
    assert F.lib().fmm_options_default(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(F.FmmOptions)
    assert (o.precision, o.nmax, o.coarse_fp64_levels, o.delta_l, o.check_finite) == (0, -1, 4, 1, 0)
    assert (o.autotune, o.bottom_tile, o.autotune_cache) == (1, 0, None)


def test_multi_index_order(F):
    """Graded order: all terms of degree n, x exponent ascending, then y."""
    for P in range(0, 10):
        mi = F.multi_index(P)
        assert len(mi) == (P + 1) * (P + 2) * (P + 3) // 6
        assert len({tuple(r) for r in mi}) == len(mi)
        deg = mi.sum(1)
        assert (mi >= 0).all() and (deg <= P).all() and (deg[1:] >= deg[:-1]).all()
        for n in range(P + 1):
            block = [tuple(r) for r in mi[deg == n]]
            assert block == sorted(block, key=lambda e: (e[0], e[1]))
    assert F.lib().fmm_multi_index(10, None, 0) == -1


def test_no_device_is_reported(F):
    """Valid arguments with no GPU visible: a device error, not a crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    ptr, status, msg = _create(F, 16, 4)
    assert not ptr and status == -4 and "device" in msg.lower()


def test_binding_refuses_cpu_tensors(F):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(F.FmmError):
        F.Plan(16, 4)


def test_batch_arguments_rejected_before_the_device(F):
    L = F.lib()
    o = F.FmmOptions()
    L.fmm_options_default(ctypes.byref(o))
    assert o.autotune == 1
    arr = (ctypes.c_int * 3)(32, 64, 128)
    assert not L.fmm_batch_plan_create(0, arr, 4, 1, ctypes.byref(o))
    assert L.fmm_last_status() == -1 and "count" in F.last_error()
    assert not L.fmm_batch_plan_create(3, None, 4, 1, ctypes.byref(o))
    assert L.fmm_last_status() == -1
    bad = (ctypes.c_int * 3)(32, 48, 128)
    assert not L.fmm_batch_plan_create(3, bad, 4, 1, ctypes.byref(o))
    assert L.fmm_last_status() == -1 and "power of two" in F.last_error()
    assert not L.fmm_batch_plan_create(3, arr, 4, 0, ctypes.byref(o))
    assert L.fmm_last_status() == -2
    assert not L.fmm_batch_plan_create(3, arr, 9, 1, ctypes.byref(o))
    assert L.fmm_last_status() == -1
    assert L.fmm_batch_solve(None, None, None, None, None) == -1
    assert L.fmm_batch_info(None, None, None, None, None, 0) == -1


def test_deposit_arguments_rejected_before_the_device(F):
    L = F.lib()
    assert L.fmm_deposit_cic(12, 1, 8, 8, 8, None) == -1            # n not a power of two
    assert L.fmm_deposit_cic(2048, 1, 8, 8, 8, None) == -1          # n too large
    assert L.fmm_deposit_cic(16, -1, 8, 8, 8, None) == -1           # negative count
    assert L.fmm_deposit_cic(16, 4, None, 8, 8, None) == -1         # NULL with particles
    assert "pos" in F.last_error()
    assert L.fmm_deposit_cic(16, 0, None, None, None, None) == 0    # nothing to do


def test_fd_force_arguments_rejected_before_the_device(F):
    L = F.lib()
    assert L.fmm_fd_force(12, 8, 4096, None) == -1           # n not a power of two
    assert L.fmm_fd_force(16, None, 8, None) == -1           # NULL phi
    assert L.fmm_fd_force(16, 8, 8 + 8 * 100, None) == -1    # f overlaps phi
    assert "overlap" in F.last_error()
