"""ctypes front of the plain FP64 CPU oracle (``fmm_oracle.c``).

TEST INFRASTRUCTURE: only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP solver
never does, and this package imports nothing from the solver.

All arrays are float64 numpy arrays; densities are (n, n, n) C order on the
unit box with G = 1; accelerations are returned as (3, ...) arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_longlong)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.or_nterms.argtypes = [ctypes.c_int]
        L.or_multi_index.argtypes = [ctypes.c_int, _ip]
        L.or_dtensor.argtypes = [_dp, ctypes.c_int, _dp]
        L.or_op_m2m.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.or_op_p2m.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.or_op_m2l.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.or_op_l2l.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.or_op_l2p.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.or_op_m2p.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.or_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                               ctypes.c_longlong, _lp, _dp, _dp]
        L.or_solve_dl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                  ctypes.c_longlong, _lp, _dp, _dp]
        L.or_expansions.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                    ctypes.c_int, ctypes.c_int, _dp]
        L.or_direct.argtypes = [ctypes.c_int, _dp, ctypes.c_longlong, _lp, _dp, _dp]
        L.or_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.or_adjoint_dl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.or_solve_timed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                     ctypes.c_longlong, _lp, _dp, _dp, _dp]
        L.or_solve_timed_dl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                        ctypes.c_longlong, _lp, _dp, _dp, _dp]
        L.or_threads.argtypes = []
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_pair_pass.argtypes = [ctypes.c_int, ctypes.c_longlong, ctypes.c_longlong]
        L.or_list_size.argtypes = [ctypes.c_int] * 4
        L.or_pair_pass_row.argtypes = [ctypes.c_int, ctypes.c_longlong, _ip]
        L.or_pair_pass_row_dl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_longlong, _ip]
        L.or_deposit_cic.argtypes = [ctypes.c_int, ctypes.c_longlong, _dp, _dp, _dp]
        L.or_fd_force.argtypes = [ctypes.c_int, _dp, _dp]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def nterms(P: int) -> int:
    return lib().or_nterms(P)


def multi_index(P: int) -> np.ndarray:
    out = np.zeros((nterms(P), 3), dtype=np.int32)
    lib().or_multi_index(P, out.ctypes.data_as(_ip))
    return out


def dtensor(R, P: int) -> np.ndarray:
    """D[g](R) = d^g(-1/|R|) for |g| <= P, oracle multi-index order."""
    R = _f64(R)
    D = np.zeros(nterms(P))
    lib().or_dtensor(_d(R), P, _d(D))
    return D


def op_p2m(nmax: int, masses, positions, centre) -> np.ndarray:
    m, x, c = _f64(masses), _f64(positions), _f64(centre)
    M = np.zeros(nterms(nmax))
    lib().or_op_p2m(nmax, len(m), _d(m), _d(x), _d(c), _d(M))
    return M


def op_m2m(nmax: int, shift, Mc) -> np.ndarray:
    d, Mc = _f64(shift), _f64(Mc)
    Mp = np.zeros(nterms(nmax))
    lib().or_op_m2m(nmax, _d(d), _d(Mc), _d(Mp))
    return Mp


def op_m2l(p: int, nmax: int, R, M) -> np.ndarray:
    R, M = _f64(R), _f64(M)
    L = np.zeros(nterms(p))
    lib().or_op_m2l(p, nmax, _d(R), _d(M), _d(L))
    return L


def op_l2l(p: int, shift, Lp) -> np.ndarray:
    a, Lp = _f64(shift), _f64(Lp)
    Lc = np.zeros(nterms(p))
    lib().or_op_l2l(p, _d(a), _d(Lp), _d(Lc))
    return Lc


def op_l2p(p: int, v, L) -> np.ndarray:
    """(phi, gx, gy, gz) of a local expansion at offset v."""
    v, L = _f64(v), _f64(L)
    out = np.zeros(4)
    lib().or_op_l2p(p, _d(v), _d(L), _d(out))
    return out


def op_m2p(nmax: int, R, M) -> np.ndarray:
    """(phi, gx, gy, gz) of a multipole at displacement R = x - c."""
    R, M = _f64(R), _f64(M)
    out = np.zeros(4)
    lib().or_op_m2p(nmax, _d(R), _d(M), _d(out))
    return out


def solve(rho, p: int, nmax: int | None = None, targets=None, delta_l: int = 1):
    """FMM potential and acceleration.  Returns (phi, g): full grid shapes
    (n,n,n) and (3,n,n,n), or (k,) and (3,k) for ``targets`` (flat indices).
    ``delta_l`` = 1 (FMM-1) or 2 (FMM-2): the finest FMM level sits that many
    levels above the unigrid (App. A)."""
    rho = _f64(rho)
    n = rho.shape[0]
    nmax = p if nmax is None else nmax
    if targets is None:
        phi = np.zeros((n, n, n))
        g = np.zeros((3, n, n, n))
        rc = lib().or_solve_dl(n, p, nmax, delta_l, _d(rho), 0, None, _d(phi), _d(g))
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        phi = np.zeros(len(t))
        g = np.zeros((3, len(t)))
        rc = lib().or_solve_dl(n, p, nmax, delta_l, _d(rho), len(t), t.ctypes.data_as(_lp), _d(phi), _d(g))
    if rc != 0:
        raise ValueError(f"oracle solve rejected n={n} p={p} nmax={nmax} delta_l={delta_l}")
    return phi, g


def expansions(rho, p: int, which: str, level: int, nmax: int | None = None) -> np.ndarray:
    """Physical multipoles ('M', level 2..F) or locals ('L', level 3..F):
    array (8^level, nterms) in the oracle's multi-index order, cells C order."""
    rho = _f64(rho)
    n = rho.shape[0]
    nmax = p if nmax is None else nmax
    nt = nterms(nmax) if which == "M" else nterms(p)
    out = np.zeros((8 ** level, nt))
    rc = lib().or_expansions(n, p, nmax, _d(rho), 0 if which == "M" else 1, level, _d(out))
    if rc != 0:
        raise ValueError("bad level")
    return out


def direct(rho, targets=None):
    """O(N^2) direct sum with the softened Green's function."""
    rho = _f64(rho)
    n = rho.shape[0]
    if targets is None:
        phi = np.zeros((n, n, n))
        g = np.zeros((3, n, n, n))
        lib().or_direct(n, _d(rho), 0, None, _d(phi), _d(g))
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        phi = np.zeros(len(t))
        g = np.zeros((3, len(t)))
        lib().or_direct(n, _d(rho), len(t), t.ctypes.data_as(_lp), _d(phi), _d(g))
    return phi, g


def adjoint(dphi, dg, p: int, nmax: int | None = None, delta_l: int = 1) -> np.ndarray:
    """d(<phi,dphi> + <g,dg>)/drho of the FMM solve (dg may be None), for the
    finest FMM level ``delta_l`` levels above the unigrid."""
    dphi = _f64(dphi)
    n = dphi.shape[0]
    nmax = p if nmax is None else nmax
    drho = np.zeros((n, n, n))
    dgv = None if dg is None else _f64(dg)
    dgp = None if dgv is None else _d(dgv)
    rc = lib().or_adjoint_dl(n, p, nmax, delta_l, _d(dphi), dgp, _d(drho))
    if rc != 0:
        raise ValueError("bad arguments")
    return drho


def pair_pass(n: int, u: int, w: int) -> int:
    """-1 near field, F M2P, s in [2, F-1] M2L from level s; -2 none, -3 several."""
    return lib().or_pair_pass(n, u, w)


def list_size(level: int, i: int, j: int, l: int) -> int:
    return lib().or_list_size(level, i, j, l)


def pair_pass_row(n: int, u: int, delta_l: int = 1) -> np.ndarray:
    out = np.zeros(n ** 3, dtype=np.int32)
    if delta_l == 1:
        lib().or_pair_pass_row(n, u, out.ctypes.data_as(_ip))
    else:
        lib().or_pair_pass_row_dl(n, delta_l, u, out.ctypes.data_as(_ip))
    return out


def solve_timed(rho, p: int, targets, nmax: int | None = None, delta_l: int = 1):
    """solve() at the listed targets, plus (upward s, downward s, threads)."""
    rho = _f64(rho)
    n = rho.shape[0]
    nmax = p if nmax is None else nmax
    t = np.ascontiguousarray(targets, dtype=np.int64)
    phi = np.zeros(len(t))
    g = np.zeros((3, len(t)))
    times = np.zeros(2)
    rc = lib().or_solve_timed_dl(n, p, nmax, delta_l, _d(rho), len(t), t.ctypes.data_as(_lp), _d(phi), _d(g),
                                 _d(times))
    if rc != 0:
        raise ValueError("bad arguments")
    return phi, g, float(times[0]), float(times[1]), int(lib().or_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    if lib().or_set_threads(int(n)) != 0:
        raise ValueError("threads must be >= 1")


def threads() -> int:
    return int(lib().or_threads())


def deposit_cic(n: int, pos, mass) -> np.ndarray:
    """Cloud-in-cell density (n, n, n) of particles pos (k, 3) in the unit box
    with masses mass (k,); shares outside the box are dropped."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float64).reshape(-1)
    if len(mass) != len(pos):
        raise ValueError("pos and mass differ in length")
    rho = np.zeros((n, n, n))
    if lib().or_deposit_cic(n, len(mass), _d(pos), _d(mass), _d(rho)) != 0:
        raise ValueError(f"oracle CIC rejected n={n}")
    return rho


def fd_force(phi) -> np.ndarray:
    """Force -grad(phi) by the 5-cell fourth-order differences (App. C),
    one-sided in the two layers next to each wall: (3, n, n, n)."""
    phi = _f64(phi)
    n = phi.shape[0]
    f = np.zeros((3, n, n, n))
    if lib().or_fd_force(n, _d(phi), _d(f)) != 0:
        raise ValueError(f"oracle FD force rejected n={n}")
    return f
