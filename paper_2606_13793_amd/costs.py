"""Exact algorithmic operation counts of one solve (boundary-clipped).

Used to turn measured kernel times into achieved FLOP/s.  A count is the
number of useful floating-point operations of the method (one fused
multiply-add = 2), independent of how the kernels issue them (padding of
matrix-core tiles is not counted).

Interaction counts follow the fixed geometry of Sec. 2.2: for a cell T of a
grid with m cells per axis, the clipped list has
    prod_i a(T_i) - prod_i b(T_i)
members, with a(t) = |[2(t//2 - 1), 2(t//2 + 1) + 1] & [0, m)| (children of the
parent's neighbours) and b(t) = |[t - 1, t + 1] & [0, m)| (the cell's own
neighbours), so summed over the grid it is (sum_t a)^3 - (sum_t b)^3.
"""
from __future__ import annotations

from math import comb


def nterms(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def _a(t: int, m: int) -> int:
    lo, hi = 2 * (t // 2 - 1), 2 * (t // 2 + 1) + 1
    return max(0, min(hi, m - 1) - max(lo, 0) + 1)


def _b(t: int, m: int) -> int:
    return max(0, min(t + 1, m - 1) - max(t - 1, 0) + 1)


def list_pairs(m: int) -> int:
    """Sum over the m^3 cells of a grid of their clipped list sizes."""
    sa = sum(_a(t, m) for t in range(m))
    sb = sum(_b(t, m) for t in range(m))
    return sa ** 3 - sb ** 3


def near_pairs(n: int, delta_l: int = 1) -> int:
    """Sum over unigrid cells of their near-field source count (incl. self):
    every unigrid cell of the finest FMM cells adjacent to the target's own,
    8^delta_l of them per FMM cell."""
    m = n >> delta_l
    sb = sum(_b(t, m) for t in range(m))
    return 8 ** (2 * delta_l) * sb ** 3


def pair_count_m2l(p: int, nmax: int | None = None) -> int:
    """(a, b) terms of one M2L pair: |b| <= p, |a| <= min(nmax, p - |b|)."""
    nmax = p if nmax is None else nmax
    return sum(comb(mb + 2, 2) * nterms(min(nmax, p - mb)) for mb in range(p + 1))


def solve_flops(n: int, p: int, nmax: int | None = None, delta_l: int = 1) -> dict:
    """Useful flops of each stage of one solve (phi and g)."""
    nmax = p if nmax is None else nmax
    L = n.bit_length() - 1
    F = L - delta_l
    NM, NL = nterms(nmax), nterms(p)
    out = {}
    out["p2m"] = 2 * NM * n ** 3
    # M2M: each child term a of the parent takes every b <= a
    m2m_terms = sum((a + 1) * (b + 1) * (c + 1)
                    for a in range(nmax + 1) for b in range(nmax + 1 - a) for c in range(nmax + 1 - a - b))
    out["m2m"] = sum(2 * m2m_terms * 8 ** k for k in range(3, F + 1))
    out["m2l"] = sum(2 * pair_count_m2l(p, nmax) * 8 * list_pairs(2 ** (k - 1)) for k in range(3, F + 1))
    out["l2l"] = sum(2 * pair_count_m2l(p, p) * 8 ** k for k in range(4, F + 1))
    out["near_l2p"] = 8 * near_pairs(n, delta_l) + (8 * NL * n ** 3 if F >= 3 else 0)
    out["m2p"] = 2 * 4 * NM * 8 ** delta_l * list_pairs(2 ** F)
    out["total"] = sum(out.values())
    # per fused kernel stage of the HIP solve
    out["m2l_l2l"] = out["m2l"] + out["l2l"]
    out["bottom"] = out["m2p"] + out["near_l2p"]
    # the M2M into level F - 1, which FMM-1 solves form in the P2M stage
    # straight from the density (the same multipoles)
    out["m2m_top"] = 2 * m2m_terms * 8 ** F if F >= 3 else 0
    return out


def m2p_pairs(n: int, delta_l: int = 1) -> int:
    """(unigrid target, list source) pairs of the M2P stage."""
    return 8 ** delta_l * list_pairs(n >> delta_l)


# The paper's per-operator counts at its own orders (Sec. 4: locals p = 3,
# multipoles nmax = 2, only the potential at the finest level), per cell and
# interaction, as printed there.
PAPER_SEC4 = {"m2m": 10, "l2l": 357, "l2p": 74, "m2l": 228, "m2p": 36, "p2p": 2}


def operator_counts(p: int = 3, nmax: int | None = None) -> dict:
    """Flops of one application of each operator in this library's counting
    (one multiply-add of a coefficient and an expansion term = 2; the
    coefficients are precomputed tables, so nothing else is counted):
      m2m  one child's multipoles shifted into the parent: every b <= a
      l2l  one parent local shifted to a child: every (b, g), |b| + |g| <= p
      m2l  one (target, source) pair: every (a, b), |b| <= p, |a| <= min(nmax, p - |b|)
      l2p  one unigrid target from its local: each term for phi, the terms
           with b_d >= 1 for g_d
      m2p  one (unigrid target, source cell) pair: every a <= nmax for phi,
           and once more per component of g
      p2p  one (target, source) cell pair: phi, and phi and g
    Returned per operator as (phi only, phi and g) where the distinction
    exists (the finest level), else the single count."""
    nmax = p if nmax is None else nmax
    NM, NL = nterms(nmax), nterms(p)
    m2m = 2 * sum((a + 1) * (b + 1) * (c + 1)
                  for a in range(nmax + 1) for b in range(nmax + 1 - a) for c in range(nmax + 1 - a - b))
    l2p_g = sum(1 for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)
                for d in (a, b, c) if d >= 1)
    return {
        "m2m": m2m,
        "l2l": 2 * pair_count_m2l(p, p),
        "m2l": 2 * pair_count_m2l(p, nmax),
        "l2p": (2 * NL, 2 * (NL + l2p_g)),
        "m2p": (2 * NM, 2 * 4 * NM),
        "p2p": (2, 8),
    }
