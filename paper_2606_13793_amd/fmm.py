"""Python binding of the C ABI in ``include/fmm.h`` (ctypes).

Only argument marshalling lives here: every step of a solve runs in the HIP
kernels of ``_lib/libfmm.so``.  PyTorch supplies device memory and the
current HIP stream.  There is no CPU fallback: without the built library or
without a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libfmm.so")

FMM_OK = 0
FMM_ERR_INVALID_ARG = -1
FMM_ERR_UNSUPPORTED = -2
FMM_ERR_OUT_OF_MEMORY = -3
FMM_ERR_DEVICE = -4
FMM_ERR_NONFINITE = -5

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}

# every symbol the header declares
EXPORTS = (
    "fmm_options_default", "fmm_plan_create", "fmm_plan_create_ex", "fmm_plan_destroy",
    "fmm_solve", "fmm_solve_backward", "fmm_plan_workspace_bytes", "fmm_plan_info",
    "fmm_last_error", "fmm_last_status", "fmm_debug_expansions", "fmm_multi_index",
    "fmm_profile_enable", "fmm_profile_read", "fmm_profile_stage_name",
    "fmm_batch_plan_create", "fmm_batch_solve", "fmm_batch_info", "fmm_deposit_cic",
    "fmm_fd_force", "fmm_solve_backward_noalloc", "fmm_batch_timestamps", "fmm_batch_field_ms",
)


class FmmOptions(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("nmax", ctypes.c_int),
        ("coarse_fp64_levels", ctypes.c_int),
        ("delta_l", ctypes.c_int),
        ("check_finite", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("bottom_tile", ctypes.c_int),
        ("autotune_cache", ctypes.c_char_p),
    ]


class FmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    """Load ``libfmm.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_13793_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        L.fmm_options_default.argtypes = [ctypes.POINTER(FmmOptions)]
        L.fmm_plan_create.argtypes = [i, i, i]
        L.fmm_plan_create.restype = vp
        L.fmm_plan_create_ex.argtypes = [i, i, i, ctypes.POINTER(FmmOptions)]
        L.fmm_plan_create_ex.restype = vp
        L.fmm_plan_destroy.argtypes = [vp]
        L.fmm_plan_destroy.restype = None
        L.fmm_solve.argtypes = [vp, vp, vp, vp, vp]
        L.fmm_solve_backward.argtypes = [vp, vp, vp, vp, vp]
        L.fmm_solve_backward_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.fmm_plan_workspace_bytes.argtypes = [vp]
        L.fmm_plan_workspace_bytes.restype = sz
        L.fmm_plan_info.argtypes = [vp] + [ctypes.POINTER(i)] * 5
        L.fmm_last_error.argtypes = []
        L.fmm_last_error.restype = ctypes.c_char_p
        L.fmm_last_status.argtypes = []
        L.fmm_last_status.restype = ctypes.c_int
        L.fmm_debug_expansions.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_double), sz]
        L.fmm_multi_index.argtypes = [i, ctypes.POINTER(i), sz]
        L.fmm_profile_enable.argtypes = [vp, i]
        L.fmm_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i), i]
        L.fmm_profile_stage_name.argtypes = [i]
        L.fmm_profile_stage_name.restype = ctypes.c_char_p
        L.fmm_batch_plan_create.argtypes = [i, ctypes.POINTER(i), i, i, ctypes.POINTER(FmmOptions)]
        L.fmm_batch_plan_create.restype = vp
        L.fmm_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.fmm_batch_info.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                     ctypes.POINTER(ctypes.c_double), i]
        L.fmm_batch_timestamps.argtypes = [vp, i]
        L.fmm_batch_field_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i]
        L.fmm_deposit_cic.argtypes = [i, ctypes.c_longlong, vp, vp, vp, vp]
        L.fmm_fd_force.argtypes = [i, vp, vp, vp]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().fmm_last_error().decode()


def _check(rc: int):
    if rc != FMM_OK:
        raise FmmError(rc, last_error())


def multi_index(P: int) -> np.ndarray:
    """Order of the expansion terms the kernels use, (nterms, 3) int array."""
    nt = (P + 1) * (P + 2) * (P + 3) // 6
    out = np.zeros(3 * nt, dtype=np.int32)
    rc = lib().fmm_multi_index(P, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), out.size)
    if rc < 0:
        _check(rc)
    return out.reshape(nt, 3)


def _stream_ptr(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Plan:
    """An ``fmm_plan``: tables and pyramids for one grid size and order.

    ``precision``: "fp64" (double I/O) or "fp32"/"bf16" (float I/O).
    """

    def __init__(self, n: int, p: int, precision: str = "fp64", nmax: int | None = None,
                 isolated: int = 1, check_finite: bool = False, coarse_fp64_levels: int = 4,
                 delta_l: int = 1, bottom_tile: int = 0):
        L = lib()
        opt = FmmOptions()
        L.fmm_options_default(ctypes.byref(opt))
        opt.precision = PRECISIONS[precision]
        opt.nmax = -1 if nmax is None else int(nmax)
        opt.check_finite = int(bool(check_finite))
        opt.coarse_fp64_levels = int(coarse_fp64_levels)
        opt.delta_l = int(delta_l)
        opt.bottom_tile = int(bottom_tile)
        ptr = L.fmm_plan_create_ex(int(n), int(p), int(isolated), ctypes.byref(opt))
        if not ptr:
            raise FmmError(L.fmm_last_status(), last_error())
        self._ptr = ptr
        self.n, self.p, self.precision = int(n), int(p), precision
        self.nmax = self.p if nmax is None else int(nmax)
        self.delta_l = int(delta_l)
        self.finest_level = int(np.log2(n)) - self.delta_l

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise RuntimeError("plan is closed")
        return self._ptr

    @property
    def io_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def workspace_bytes(self) -> int:
        return int(lib().fmm_plan_workspace_bytes(self.ptr))

    def close(self):
        if getattr(self, "_ptr", None):
            lib().fmm_plan_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_tensor(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.io_dtype:
            raise TypeError(f"{name} must be {self.io_dtype} for a {self.precision} plan (got {t.dtype})")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {tuple(shape)} (got {tuple(t.shape)})")

    def solve_into(self, rho, phi, g=None, stream=None):
        n = self.n
        self._check_tensor(rho, (n, n, n), "rho")
        self._check_tensor(phi, (n, n, n), "phi")
        if g is not None:
            self._check_tensor(g, (3, n, n, n), "g")
        _check(lib().fmm_solve(self.ptr, rho.data_ptr(), phi.data_ptr(),
                               None if g is None else g.data_ptr(), _stream_ptr(stream)))

    def solve(self, rho, want_g: bool = True, stream=None):
        """(phi, g) of rho on the current stream (g is None if not wanted)."""
        import torch
        n = self.n
        phi = torch.empty((n, n, n), dtype=self.io_dtype, device=rho.device)
        g = torch.empty((3, n, n, n), dtype=self.io_dtype, device=rho.device) if want_g else None
        self.solve_into(rho, phi, g, stream)
        return phi, g

    def backward(self, dphi, dg=None, stream=None):
        """drho = d(<phi, dphi> + <g, dg>)/drho."""
        import torch
        n = self.n
        self._check_tensor(dphi, (n, n, n), "dphi")
        if dg is not None:
            self._check_tensor(dg, (3, n, n, n), "dg")
        drho = torch.empty((n, n, n), dtype=self.io_dtype, device=dphi.device)
        _check(lib().fmm_solve_backward(self.ptr, dphi.data_ptr(), None if dg is None else dg.data_ptr(),
                                        drho.data_ptr(), _stream_ptr(stream)))
        return drho

    def profile(self, enable: bool = True):
        """Start (or stop) per-stage HIP-event timing of later calls."""
        _check(lib().fmm_profile_enable(self.ptr, int(bool(enable))))

    def profile_read(self) -> dict:
        """{stage: (milliseconds, kernel launches)} since the last read."""
        L = lib()
        names = []
        while True:
            nm = L.fmm_profile_stage_name(len(names))
            if nm is None:
                break
            names.append(nm.decode())
        ms = (ctypes.c_double * len(names))()
        cnt = (ctypes.c_int * len(names))()
        _check(L.fmm_profile_read(self.ptr, ms, cnt, len(names)))
        return {nm: (ms[i], cnt[i]) for i, nm in enumerate(names)}

    def expansions(self, which: str, level: int) -> np.ndarray:
        """Scaled multipoles ('M') or locals ('L') of `level` after a solve,
        (8^level, nterms) float64 in the order of ``multi_index``."""
        import torch
        torch.cuda.synchronize()
        nt = (self.nmax + 1) * (self.nmax + 2) * (self.nmax + 3) // 6 if which == "M" else \
            (self.p + 1) * (self.p + 2) * (self.p + 3) // 6
        out = np.zeros((8 ** level, nt))
        _check(lib().fmm_debug_expansions(self.ptr, 0 if which == "M" else 1, level,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
        return out


class Batch:
    """A batch plan (``fmm_batch_plan_create``): fields of the given sizes,
    one order and precision, each stage one launch over every field; solves
    replay a captured HIP graph."""

    def __init__(self, sizes, p: int, precision: str = "fp32", coarse_fp64_levels: int = 4,
                 autotune: bool = True, isolated: int = 1, delta_l: int = 1, bottom_tile: int = 0,
                 autotune_cache: str | None = None):
        L = lib()
        opt = FmmOptions()
        L.fmm_options_default(ctypes.byref(opt))
        opt.precision = PRECISIONS[precision]
        opt.coarse_fp64_levels = int(coarse_fp64_levels)
        opt.autotune = int(bool(autotune))
        opt.delta_l = int(delta_l)
        opt.bottom_tile = int(bottom_tile)
        cache = None if autotune_cache is None else os.fsencode(autotune_cache)
        opt.autotune_cache = cache  # `cache` keeps the bytes alive through the call
        self.sizes = [int(n) for n in sizes]
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        ptr = L.fmm_batch_plan_create(len(self.sizes), arr, int(p), int(isolated), ctypes.byref(opt))
        if not ptr:
            raise FmmError(L.fmm_last_status(), last_error())
        self._ptr = ptr
        self.p, self.precision = int(p), precision

    @property
    def ptr(self) -> int:
        if not self._ptr:
            raise RuntimeError("plan is closed")
        return self._ptr

    @property
    def io_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def info(self) -> dict:
        c, bz, grp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        ms = (ctypes.c_double * 4)()
        _check(lib().fmm_batch_info(self.ptr, ctypes.byref(c), ctypes.byref(bz), ctypes.byref(grp), ms, 4))
        return {"count": c.value, "bottom_tile": bz.value, "m2l_grouping": grp.value,
                "tune_ms": [ms[i] for i in range(4)]}

    def workspace_bytes(self) -> int:
        return int(lib().fmm_plan_workspace_bytes(self.ptr))

    def timestamps(self, enable: bool = True):
        """Record per-field completion times of the following solves."""
        _check(lib().fmm_batch_timestamps(self.ptr, int(bool(enable))))

    def field_ms(self) -> list:
        """Milliseconds from the start of the last timed solve to each field's completion."""
        k = len(self.sizes)
        ms = (ctypes.c_double * k)()
        _check(lib().fmm_batch_field_ms(self.ptr, ms, k))
        return [ms[i] for i in range(k)]

    def profile(self, enable: bool = True):
        _check(lib().fmm_profile_enable(self.ptr, int(bool(enable))))

    def profile_read(self) -> dict:
        return Plan.profile_read(self)

    def close(self):
        if getattr(self, "_ptr", None):
            lib().fmm_plan_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, n, comps, name):
        import torch
        shape = (n, n, n) if comps == 1 else (comps, n, n, n)
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.io_dtype:
            raise TypeError(f"{name} must be {self.io_dtype} (got {t.dtype})")
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {shape} (got {tuple(t.shape)})")

    def solve_into(self, rhos, phis, gs=None, stream=None):
        """Solve every field: rhos[i] -> phis[i] (and gs[i] unless gs is None)."""
        k = len(self.sizes)
        if len(rhos) != k or len(phis) != k or (gs is not None and len(gs) != k):
            raise ValueError(f"expected {k} fields")
        for i, n in enumerate(self.sizes):
            self._check(rhos[i], n, 1, f"rho[{i}]")
            self._check(phis[i], n, 1, f"phi[{i}]")
            if gs is not None and gs[i] is not None:
                self._check(gs[i], n, 3, f"g[{i}]")
        vp = ctypes.c_void_p
        r = (vp * k)(*[t.data_ptr() for t in rhos])
        ph = (vp * k)(*[t.data_ptr() for t in phis])
        g = None if gs is None else (vp * k)(*[0 if t is None else t.data_ptr() for t in gs])
        _check(lib().fmm_batch_solve(self.ptr, r, ph, g, _stream_ptr(stream)))

    def solve(self, rhos, want_g: bool = True, stream=None):
        import torch
        dev = rhos[0].device
        phis = [torch.empty((n, n, n), dtype=self.io_dtype, device=dev) for n in self.sizes]
        gs = [torch.empty((3, n, n, n), dtype=self.io_dtype, device=dev) for n in self.sizes] if want_g else None
        self.solve_into(rhos, phis, gs, stream)
        return phis, gs


def _autograd_fn():
    import torch

    class _FmmSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, rho, plan):
            ctx.plan = plan
            phi, g = plan.solve(rho.contiguous())
            return phi, g

        @staticmethod
        def backward(ctx, dphi, dg):
            plan = ctx.plan
            if dphi is None:
                dphi = torch.zeros((plan.n,) * 3, dtype=plan.io_dtype, device=dg.device)
            drho = plan.backward(dphi.contiguous(), None if dg is None else dg.contiguous())
            return drho, None

    return _FmmSolve


_FN = None


def solve(plan: Plan, rho):
    """Differentiable (phi, g) = FMM(rho); backward runs the adjoint kernels."""
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    return _FN.apply(rho, plan)


def deposit_cic(n: int, pos, mass, rho=None, stream=None):
    """Cloud-in-cell density of particles (``fmm_deposit_cic``): pos (k, 3)
    and mass (k,) float64 CUDA tensors in the unit box; returns rho (n, n, n)
    float64, or adds into the given ``rho``."""
    import torch
    if pos.dtype != torch.float64 or mass.dtype != torch.float64 or not pos.is_cuda or not mass.is_cuda:
        raise TypeError("pos and mass must be float64 CUDA tensors")
    pos = pos.contiguous()
    mass = mass.contiguous()
    if pos.dim() != 2 or pos.shape[1] != 3 or mass.shape != (pos.shape[0],):
        raise ValueError("pos must be (k, 3) and mass (k,)")
    if rho is None:
        rho = torch.zeros((n, n, n), dtype=torch.float64, device=pos.device)
    elif rho.dtype != torch.float64 or tuple(rho.shape) != (n, n, n) or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous float64 (n, n, n) tensor")
    _check(lib().fmm_deposit_cic(int(n), int(pos.shape[0]), pos.data_ptr(), mass.data_ptr(), rho.data_ptr(),
                                 _stream_ptr(stream)))
    return rho


def fd_force(phi, stream=None):
    """Force -grad(phi) by 5-cell fourth-order differences (``fmm_fd_force``),
    the host code's force of App. C: (3, n, n, n) float64 from a float64
    (n, n, n) CUDA tensor."""
    import torch
    if phi.dtype != torch.float64 or not phi.is_cuda or phi.dim() != 3 or len(set(phi.shape)) != 1:
        raise TypeError("phi must be a float64 (n, n, n) CUDA tensor")
    phi = phi.contiguous()
    n = phi.shape[0]
    f = torch.empty((3, n, n, n), dtype=torch.float64, device=phi.device)
    _check(lib().fmm_fd_force(int(n), phi.data_ptr(), f.data_ptr(), _stream_ptr(stream)))
    return f
