"""The operation-count model used to turn kernel times into achieved FLOP/s
(paper_2606_13793_amd/costs.py) against the oracle's interaction lists and
the paper's interior counts (Sec. 2.2, Sec. 4)."""
import json
import os

import pytest

from paper_2606_13793_amd import costs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


@pytest.mark.parametrize("level", [2, 3, 4])
def test_list_pairs_equal_summed_oracle_lists(orc, level):
    m = 1 << level
    total = sum(orc.list_size(level, i, j, l) for i in range(m) for j in range(m) for l in range(m))
    assert costs.list_pairs(m) == total


def test_interior_counts_match_the_paper():
    counts = json.load(open(GOLDEN))
    # an interior cell (index 10 of 64 per axis) has the full list and near field
    m = 64
    assert costs._a(10, m) ** 3 - costs._b(10, m) ** 3 == counts["list_octs"]["value"]
    assert 8 * costs._b(10, m) ** 3 == counts["near_cells_delta1"]["value"]
    assert costs.nterms(2) == counts["multipole_terms_order2"]["value"]
    assert costs.nterms(3) == counts["local_terms_order3"]["value"]


def test_pair_count_m2l_is_the_truncated_term_count():
    # (a, b) pairs with |a| + |b| <= p counted by brute force
    for p in range(1, 9):
        terms = [(a, b, c) for n in range(p + 1) for a in range(n + 1) for b in range(n + 1 - a)
                 for c in [n - a - b]]
        brute = sum(1 for x in terms for y in terms if sum(x) + sum(y) <= p)
        assert costs.pair_count_m2l(p) == brute


def test_near_pairs_brute_force():
    n = 16
    m = n // 2
    brute = 0
    for t in range(m ** 3):
        ti, tj, tl = t // (m * m), (t // m) % m, t % m
        cnt = 0
        for i in range(max(0, ti - 1), min(m, ti + 2)):
            for j in range(max(0, tj - 1), min(m, tj + 2)):
                for l in range(max(0, tl - 1), min(m, tl + 2)):
                    cnt += 8
        brute += 8 * cnt
    assert costs.near_pairs(n) == brute


@pytest.mark.parametrize("n,dl", [(16, 1), (16, 2), (32, 2)])
def test_near_and_m2p_pairs_equal_the_oracle_partition(orc, n, dl):
    """Summed over every target, the oracle's near-field and M2P sources
    (FMM-1 and FMM-2) are the pair counts the model gives."""
    import numpy as np
    F = int(np.log2(n)) - dl
    near = m2p = 0
    for u in range(n ** 3):
        row = orc.pair_pass_row(n, u, delta_l=dl)
        near += int((row == -1).sum())
        m2p += int((row == F).sum())
    assert costs.near_pairs(n, dl) == near
    # the oracle reports unigrid sources; an M2P source is a finest FMM cell of 8^dl of them
    assert costs.m2p_pairs(n, dl) * 8 ** dl == m2p


def test_operator_counts_at_the_papers_orders():
    """Per-operator counts at p = 3, nmax = 2 (the paper's Sec. 4 setting),
    each re-derived by enumerating the terms the operator sums."""
    c = costs.operator_counts(3, 2)
    deg = lambda t: sum(t)
    terms = lambda P: [(a, b, k) for a in range(P + 1) for b in range(P + 1 - a) for k in range(P + 1 - a - b)]
    # M2M: pairs b <= a (componentwise), |a| <= 2
    assert c["m2m"] == 2 * sum(1 for a in terms(2) for b in terms(2) if all(x <= y for x, y in zip(b, a)))
    # L2L: pairs (b, g) with |b| + |g| <= 3
    assert c["l2l"] == 2 * sum(1 for b in terms(3) for g in terms(3) if deg(b) + deg(g) <= 3)
    # M2L: pairs (a, b) with |b| <= 3, |a| <= min(2, 3 - |b|)
    assert c["m2l"] == 2 * sum(1 for b in terms(3) for a in terms(2) if deg(a) <= 3 - deg(b))
    assert c["l2p"] == (2 * 20, 2 * (20 + 3 * 10))
    assert c["m2p"] == (2 * 10, 8 * 10)
    assert c["p2p"] == (2, 8)
    # the paper's direct-sum count is this counting's potential-only one
    assert costs.PAPER_SEC4["p2p"] == c["p2p"][0]
