"""Pins of the oracle's traversal counts against what Sec. 4 of the paper fixes
for uniformly distributed molecules (Table hitrate and the text around it).

The hit rate of a traversal is the number of visited molecule triplets that
satisfy the cutoff over the number visited (Sec. 4, Table hitrate).  Setup of
the paper's table: uniform molecules, cells of side rc.  Here: density 0.7016
(the paper's benchmark fluid, Sec. 5.3) in a periodic box of 5^3 cells of
side 2.5 = rc, several seeds.

Pinned here:
* 3c01, pairwise cutoff: the hit rate has a closed form.  The partners of a
  molecule are drawn from its 27-cell neighbourhood, a cube of 27 rc^3; both
  lie inside its cutoff sphere with probability (4 pi / 81)^2, and two
  uniform points of a ball of radius rc are closer than rc with probability
  15/32 (distance law of two uniform points in a ball), so the hit rate is
  (4 pi / 81)^2 * 15/32 = 1.128 %.
* 3c01, product cutoff: an independent Monte Carlo over the geometry of one
  molecule in its cell and two partners in its 27-cell neighbourhood.
* Both 3c01 figures against the printed ones (1.19 % and 7.50 %) within
  10 % relative: the paper's simulation size is unstated, and the closed
  form already lies 5 % below its pairwise figure.
* The orderings the paper states: the hit rate rises from 3c01 to 3c18 to
  3c08 for both cutoffs, the product cutoff has the higher hit rate for every
  traversal, and under the product cutoff 3c01 finds the most distinct
  triplets, then 3c18, then 3c08 (Sec. 4, end of the 3c08 paragraph).

The printed 3c18 and 3c08 hit rates (2.71 / 4.00 % pairwise) are not
reproduced by the readings of those cell sets used here (1.5 / 2.4 %); they
stay unpinned apart from the orderings.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

RC = 2.5
L = 12.5
RHO = 0.7016
SEEDS = (10, 11, 12, 13)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_hitrate.json")


def _systems():
    n = int(round(RHO * L ** 3))
    return [workloads.uniform(n, [L, L, L], seed=s) for s in SEEDS]


@pytest.fixture(scope="module")
def counts(orc):
    """Summed counts over the seeds for every traversal and cutoff."""
    out = {}
    for trunc in ("pair", "product"):
        for var in ("3c01", "3c18", "3c08"):
            c = t = d = 0
            for pos, box in _systems():
                r = orc.brute(pos, box, rc=RC, truncation=trunc, variant=var, terms=2)
                c += r.n_candidates
                t += r.n_triplets
                d += r.n_distinct
            out[trunc, var] = {"candidates": c, "triplets": t, "distinct": d, "hit": t / c}
    return out


def test_hitrate_3c01_pair_closed_form(counts):
    closed = (4.0 * math.pi / 81.0) ** 2 * 15.0 / 32.0
    got = counts["pair", "3c01"]["hit"]
    # seed-to-seed spread of one 1370-molecule box is 1.3 % relative
    assert abs(got / closed - 1.0) < 0.025, (got, closed)


def _product_hitrate_mc(samples=4_000_000, seed=7):
    """P(x y z < rc^6) for a molecule uniform in its cell and two partners
    uniform in the 27 cells around it (cell side = rc = 1), by plain
    sampling of the geometry."""
    rng = np.random.default_rng(seed)
    hits = 0
    for _ in range(samples // 500_000):
        m = 500_000
        i = rng.uniform(0.0, 1.0, (m, 3))
        j = rng.uniform(-1.0, 2.0, (m, 3))
        k = rng.uniform(-1.0, 2.0, (m, 3))
        x = ((i - j) ** 2).sum(1)
        y = ((i - k) ** 2).sum(1)
        z = ((j - k) ** 2).sum(1)
        hits += int(np.count_nonzero(x * y * z < 1.0))
    return hits / samples


def test_hitrate_3c01_product_against_geometry(counts):
    mc = _product_hitrate_mc()
    got = counts["product", "3c01"]["hit"]
    assert abs(got / mc - 1.0) < 0.02, (got, mc)


def test_hitrate_3c01_against_printed_table(counts):
    with open(GOLDEN) as f:
        paper = json.load(f)
    for trunc in ("pair", "product"):
        printed = paper["3c01"][trunc] / 100.0
        got = counts[trunc, "3c01"]["hit"]
        assert abs(got / printed - 1.0) < 0.10, (trunc, got, printed)


def test_hitrate_orderings(counts):
    for trunc in ("pair", "product"):
        h = [counts[trunc, v]["hit"] for v in ("3c01", "3c18", "3c08")]
        assert h[0] < h[1] < h[2], (trunc, h)
    for var in ("3c01", "3c18", "3c08"):
        assert counts["product", var]["hit"] > counts["pair", var]["hit"], var


def test_product_rule_found_triplets_order(counts):
    d = [counts["product", v]["distinct"] for v in ("3c01", "3c18", "3c08")]
    assert d[0] > d[1] > d[2], d
    # under the pairwise cutoff every traversal finds the same triplets
    p = {counts["pair", v]["distinct"] for v in ("3c01", "3c18", "3c08")}
    assert len(p) == 1, p
