"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
textbook angle form of the ATM potential, closed forms, finite differences,
symmetry invariants, independent numpy brute force (graph triangles), lattice
sums, and the paper's counting equations (Sec. 3).
"""
import itertools
import math

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

NU = 0.073
RC = 2.5


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


# --------------------------------------------------------------------------
# eq. (atm): the law-of-cosines form equals the angle form
# nu (1 + 3 cos(th_i) cos(th_j) cos(th_k)) / (r_ij r_ik r_jk)^3
# --------------------------------------------------------------------------
def test_atm_energy_equals_angle_form(orc):
    rng = np.random.default_rng(11)
    checked = 0
    while checked < 300:
        ri, rj, rk = rng.uniform(-1.6, 1.6, (3, 3))
        a, b, c = _norm(ri - rj), _norm(ri - rk), _norm(rj - rk)
        if min(a, b, c) < 0.4:
            continue
        cos_i = np.dot(rj - ri, rk - ri) / (a * b)
        cos_j = np.dot(ri - rj, rk - rj) / (a * c)
        cos_k = np.dot(ri - rk, rj - rk) / (b * c)
        ref = NU * (1.0 + 3.0 * cos_i * cos_j * cos_k) / (a * b * c) ** 3
        assert orc.atm_energy(a, b, c, NU) == pytest.approx(ref, rel=1e-11, abs=1e-15)
        checked += 1


@pytest.mark.parametrize("r", [0.9, 1.0, 1.2345, 2.4])
def test_atm_closed_forms(orc, r):
    # equilateral: u = 11 nu / (8 r^9)
    assert orc.atm_energy(r, r, r, NU) == pytest.approx(11 * NU / (8 * r ** 9), rel=1e-13)
    # collinear (r, 2r, r): u = -nu / (4 r^9)
    assert orc.atm_energy(r, 2 * r, r, NU) == pytest.approx(-NU / (4 * r ** 9), rel=1e-12)
    # right angle at i (legs r and 1.3 r): cos(th_i) = 0 so u = nu / (r_ij r_ik r_jk)^3
    a, b = r, 1.3 * r
    c = math.hypot(a, b)
    assert orc.atm_energy(a, b, c, NU) == pytest.approx(NU / (a * b * c) ** 3, rel=1e-12)
    # eq. (ATMGradient) at the equilateral point: du/dr_ij = -33 nu / (8 r^10)
    assert orc.atm_dudr(r, r, r, NU) == pytest.approx(-33 * NU / (8 * r ** 10), rel=1e-12)


def test_atm_gradient_equals_finite_difference(orc):
    """eq. (ATMGradient) with each side in turn (roles cycled) against central
    differences of eq. (atm)."""
    rng = np.random.default_rng(12)
    n = 0
    while n < 200:
        ri, rj, rk = rng.uniform(-1.6, 1.6, (3, 3))
        s = [_norm(ri - rj), _norm(ri - rk), _norm(rj - rk)]
        if min(s) < 0.5:
            continue
        for k in range(3):
            h = 1e-5 * s[k]
            sp, sm = list(s), list(s)
            sp[k] += h
            sm[k] -= h
            fd = (orc.atm_energy(*sp, NU) - orc.atm_energy(*sm, NU)) / (2 * h)
            others = [s[m] for m in range(3) if m != k]
            g = orc.atm_dudr(s[k], others[0], others[1], NU)
            scale = abs(orc.atm_energy(*s, NU)) / s[k] + abs(g)
            assert abs(g - fd) <= 2e-7 * scale
        n += 1


def test_triplet_newton3_torque_virial(orc):
    rng = np.random.default_rng(13)
    for _ in range(100):
        ri, rj, rk = rng.uniform(-1.5, 1.5, (3, 3))
        if min(_norm(ri - rj), _norm(ri - rk), _norm(rj - rk)) < 0.5:
            continue
        fi, fj, fk, u, w = orc.triplet(ri - rj, ri - rk, rj - rk, NU)
        scale = max(np.abs(fi).max(), np.abs(fj).max(), np.abs(fk).max())
        # eq. (newton3rdlaw): F_i + F_j = -F_k
        assert np.abs(fi + fj + fk).max() <= 1e-12 * scale
        # no net torque (central force pairs)
        tq = np.cross(ri, fi) + np.cross(rj, fj) + np.cross(rk, fk)
        assert np.abs(tq).max() <= 1e-11 * scale * 3
        # eq. (P_3) virial term: degree -9 homogeneity gives W = 9 u
        assert w == pytest.approx(9 * u, rel=1e-11, abs=1e-14)


def test_equilateral_force_closed_form(orc):
    r = 1.1
    ri = np.array([0.0, 0.0, 0.0])
    rj = np.array([r, 0.0, 0.0])
    rk = np.array([r / 2, r * math.sqrt(3) / 2, 0.0])
    fi, fj, fk, u, w = orc.triplet(ri - rj, ri - rk, rj - rk, NU)
    cen = (ri + rj + rk) / 3
    mag = 33 * math.sqrt(3) * NU / (8 * r ** 10)
    for p, f in ((ri, fi), (rj, fj), (rk, fk)):
        assert _norm(f) == pytest.approx(mag, rel=1e-12)
        out = (p - cen) / _norm(p - cen)
        assert np.dot(f, out) == pytest.approx(mag, rel=1e-12)  # repulsive, away from centroid


# --------------------------------------------------------------------------
# Lennard-Jones closed forms (Sec. 5, reduced units, unshifted)
# --------------------------------------------------------------------------
def test_lj_closed_forms(orc):
    box = np.array([20.0, 20.0, 20.0])
    for r, u_ref, f_ref in ((2 ** (1 / 6), -1.0, 0.0), (1.0, 0.0, 24.0), (1.5, 4 * (1.5 ** -12 - 1.5 ** -6),
                                                                          24 * (2 * 1.5 ** -12 - 1.5 ** -6) / 1.5)):
        pos = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        res = orc.brute(pos, box, terms=1)
        assert res.e_lj == pytest.approx(u_ref, abs=1e-14)
        assert res.forces[0, 0] == pytest.approx(-f_ref, abs=1e-12)
        assert res.forces[1, 0] == pytest.approx(f_ref, abs=1e-12)
        assert res.w_lj == pytest.approx(f_ref * r, abs=1e-12)
        assert res.n_pairs == 1


# --------------------------------------------------------------------------
# Whole-system checks
# --------------------------------------------------------------------------
def _fluid(n, rho, jitter, seed):
    return workloads.fcc(n, rho, jitter=jitter, seed=seed)


@pytest.mark.parametrize("terms", [1, 2])
@pytest.mark.parametrize("truncation,variant,rho,n", [
    ("pair", "3c08", 0.6, 200), ("pair", "3c18", 0.6, 200), ("pair", "3c01", 0.6, 200),
    ("product", "3c08", 0.13, 256)])
def test_forces_are_minus_energy_gradient(orc, terms, truncation, variant, rho, n):
    """F = -grad E (reading of the sign at the end of Sec. 2) by central
    differences of the total energy, for LJ and ATM separately."""
    pos, box = _fluid(n, rho, 0.3, 21)
    kw = dict(truncation=truncation, variant=variant, terms=terms)
    base = orc.brute(pos, box, **kw)
    rng = np.random.default_rng(5)
    fscale = np.sqrt((base.forces ** 2).sum(axis=1).mean())
    for _ in range(6):
        i, d = int(rng.integers(n)), int(rng.integers(3))
        h = 1e-6
        pp, pm = pos.copy(), pos.copy()
        pp[i, d] += h
        pm[i, d] -= h
        ep, em = orc.brute(pp, box, **kw), orc.brute(pm, box, **kw)
        e = (lambda r: r.e_lj + r.e_atm)
        fd = -(e(ep) - e(em)) / (2 * h)
        assert abs(fd - base.forces[i, d]) <= 1e-5 * fscale


@pytest.mark.parametrize("terms", [1, 2])
def test_virial_equals_scaling_derivative(orc, terms):
    """W = sum r.F equals -dE/d(ln lambda) when positions and box are scaled
    by lambda (eq. P_3 for the three-body part)."""
    pos, box = _fluid(300, 0.6, 0.2, 22)
    base = orc.brute(pos, box, terms=terms)
    h = 1e-8
    ep = orc.brute(pos * (1 + h), box * (1 + h), terms=terms)
    em = orc.brute(pos * (1 - h), box * (1 - h), terms=terms)
    # the truncation is discontinuous: no pair or triplet may cross rc
    for r in (ep, em):
        assert (r.n_pairs, r.n_triplets) == (base.n_pairs, base.n_triplets)
    e = (lambda r: r.e_lj + r.e_atm)
    w = base.w_lj + base.w_atm
    fd = -(e(ep) - e(em)) / (2 * h)
    assert fd == pytest.approx(w, rel=1e-6)


@pytest.mark.parametrize("truncation,variant", [
    ("pair", "3c08"), ("pair", "3c18"), ("pair", "3c01"), ("product", "3c08"),
    ("product", "3c18"), ("product", "3c01")])
def test_w3_is_nine_e3_and_momentum(orc, truncation, variant):
    if truncation == "product":
        pos, box = workloads.uniform(500, [17.6, 17.6, 17.6], seed=31)
    else:
        pos, box = workloads.uniform(400, [9.0, 9.0, 9.0], seed=31)
    r = orc.brute(pos, box, truncation=truncation, variant=variant, terms=2)
    assert r.n_triplets > 0
    assert r.w_atm == pytest.approx(9 * r.e_atm, rel=1e-11)
    fsum = np.abs(r.forces.sum(axis=0)).max()
    fscale = np.abs(r.forces).max()
    if variant != "3c01" or truncation == "pair":
        assert fsum <= 1e-11 * fscale * len(pos)


def test_translation_invariance(orc):
    pos, box = _fluid(400, 0.6, 0.1, 23)
    a = orc.brute(pos, box)
    shifted = pos + np.array([3.3, -7.1, 0.77])
    b = orc.brute(shifted, box)
    assert (a.n_pairs, a.n_triplets) == (b.n_pairs, b.n_triplets)
    assert b.e_atm == pytest.approx(a.e_atm, rel=1e-11)
    assert b.e_lj == pytest.approx(a.e_lj, rel=1e-11)
    assert np.abs(a.forces - b.forces).max() <= 1e-10 * np.abs(a.forces).max()


@pytest.mark.parametrize("truncation", ["pair", "product"])
def test_axis_permutation_and_reflection(orc, truncation):
    L = 12.6 if truncation == "product" else 9.0
    pos, box = workloads.uniform(350 if truncation == "pair" else 450, [L, L, L], seed=24)
    a = orc.brute(pos, box, truncation=truncation, terms=2)
    perm = pos[:, [1, 2, 0]]
    b = orc.brute(perm, box, truncation=truncation, terms=2)
    assert a.n_triplets == b.n_triplets
    assert np.abs(a.forces[:, [1, 2, 0]] - b.forces).max() <= 1e-10 * np.abs(a.forces).max()
    refl = pos.copy()
    refl[:, 0] = L - refl[:, 0] - 1e-9
    c = orc.brute(refl, box, truncation=truncation, terms=2)
    assert a.n_triplets == c.n_triplets
    fr = a.forces.copy()
    fr[:, 0] *= -1
    assert np.abs(fr - c.forces).max() <= 1e-7 * np.abs(a.forces).max()


def test_rotation_invariance_isolated_cluster(orc):
    rng = np.random.default_rng(25)
    cl, _ = workloads.fcc(32, 0.7, jitter=0.1, seed=26)
    cl = cl - cl.mean(axis=0)
    box = np.array([40.0, 40.0, 40.0])
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    a = orc.brute(cl + 20.0, box)
    b = orc.brute(cl @ q.T + 20.0, box)
    assert a.n_triplets == b.n_triplets and a.n_triplets > 0
    assert b.e_atm == pytest.approx(a.e_atm, rel=1e-11)
    assert np.abs(a.forces @ q.T - b.forces).max() <= 1e-10 * np.abs(a.forces).max()


@pytest.mark.parametrize("truncation,variant,L,n", [
    ("pair", "3c08", 9.0, 300), ("pair", "3c18", 9.0, 300), ("pair", "3c01", 9.0, 300),
    ("product", "3c08", 12.6, 500), ("product", "3c18", 17.6, 900), ("product", "3c01", 17.6, 900)])
def test_brute_equals_per_molecule(orc, truncation, variant, L, n):
    pos, box = workloads.uniform(n, [L, L, L], seed=27)
    a = orc.brute(pos, box, truncation=truncation, variant=variant)
    b = orc.molecules(pos, box, truncation=truncation, variant=variant)
    assert (a.n_pairs, a.n_triplets) == (b.n_pairs, b.n_triplets)
    scale = np.sqrt((a.forces ** 2).sum(axis=1)).max()
    assert np.abs(a.forces - b.forces).max() <= 1e-12 * scale
    assert b.e_atm == pytest.approx(a.e_atm, rel=1e-12)
    sample = np.array([0, 7, n // 2, n - 1])
    c = orc.molecules(pos, box, truncation=truncation, variant=variant, sample=sample)
    assert np.abs(c.forces - a.forces[sample]).max() <= 1e-12 * scale


@pytest.mark.parametrize("kind,n,L", [("uniform", 300, 9.0), ("uniform", 700, 12.6), ("fcc", 1000, None)])
def test_linked_cells_equal_brute_force(orc, kind, n, L):
    """The Newton-3 linked-cell evaluation over the 3c08 sets (the timed CPU
    reference) finds the same pairs and triplets as brute force, and the same
    forces, energies and virials up to the order of the FP64 sums; its
    candidate count is that of the 3c08 sets."""
    if kind == "fcc":
        pos, box = workloads.make("fcc1k")
    else:
        pos, box = workloads.uniform(n, [L, L, L], seed=29)
    for terms in (1, 2, 3):
        a = orc.brute(pos, box, terms=terms)
        b = orc.cells(pos, box, terms=terms)
        assert (a.n_pairs, a.n_triplets) == (b.n_pairs, b.n_triplets)
        scale = np.sqrt((a.forces ** 2).sum(axis=1)).max()
        assert np.abs(a.forces - b.forces).max() <= 1e-12 * scale
        for f in ("e_lj", "e_atm", "w_lj", "w_atm"):
            assert getattr(b, f) == pytest.approx(getattr(a, f), rel=1e-12, abs=1e-300)
        if terms & 2:
            assert b.n_candidates == a.n_candidates
    # a range of base cells covers its share: the two halves add up
    full = orc.cells(pos, box)
    nc = orc.grid(box, RC)
    half = int(np.prod(nc)) // 2
    lo = orc.cells(pos, box, base_cells=(0, half))
    hi = orc.cells(pos, box, base_cells=(half, int(np.prod(nc))))
    assert lo.n_triplets + hi.n_triplets == full.n_triplets
    assert np.abs(lo.forces + hi.forces - full.forces).max() <= 1e-12 * np.abs(full.forces).max()


# --------------------------------------------------------------------------
# Counting pins
# --------------------------------------------------------------------------
def _fcc_lattice_counts(rho):
    """Pairs and triplets per molecule of the infinite FCC lattice (rc=2.5)
    by direct enumeration of the neighbour shell of one site."""
    a = (4.0 / rho) ** (1.0 / 3.0)
    basis = np.array([[0, 0, 0], [.5, .5, 0], [.5, 0, .5], [0, .5, .5]])
    rr = range(-4, 5)
    pts = np.array([(np.array(c) + b) * a for c in itertools.product(rr, rr, rr) for b in basis])
    d = np.linalg.norm(pts, axis=1)
    S = pts[(d > 0) & (d < RC)]
    D = np.linalg.norm(S[:, None, :] - S[None, :, :], axis=2)
    adj = (D < RC) & ~np.eye(len(S), dtype=bool)
    return len(S) / 2, adj.sum() / 2 / 3


@pytest.mark.parametrize("rho,ncell,pairs,trips", [(0.6, 5, 21, 124), (0.75, 6, 27, 210)])
def test_perfect_fcc_lattice_counts(orc, rho, ncell, pairs, trips):
    p_ref, t_ref = _fcc_lattice_counts(rho)
    assert (p_ref, t_ref) == (pairs, trips)
    n = 4 * ncell ** 3
    pos, box = workloads.fcc(n, rho, jitter=0.0, seed=1)
    r = orc.brute(pos, box)
    assert r.n_pairs == pairs * n
    assert r.n_triplets == trips * n
    # every site is a centre of symmetry: all forces vanish
    assert np.abs(r.forces).max() < 1e-9


@pytest.mark.parametrize("variant", ["3c08", "3c18", "3c01"])
def test_pair_rule_is_complete(orc, variant):
    """Under the pairwise cutoff every traversal finds every triplet whose
    three sides are inside rc (Sec. 4): the count equals the number of
    triangles of the 'within rc' graph, trace(A^3)/6, computed in numpy."""
    pos, box = workloads.uniform(350, [9.3, 9.3, 9.3], seed=28)
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.rint(d / box)
    A = ((d ** 2).sum(axis=2) < RC * RC).astype(np.int64)
    np.fill_diagonal(A, 0)
    tri = int(np.trace(A @ A @ A)) // 6
    r = orc.brute(pos, box, variant=variant)
    mult = 3 if variant == "3c01" else 1
    assert r.n_triplets == mult * tri
    assert r.n_pairs == A.sum() // 2


def test_pair_set_inside_product_set(orc):
    """Every triplet valid under the pairwise cutoff is valid under the
    product cutoff (Sec. 2, Fig. 3body_surface), so the counts nest."""
    pos, box = workloads.uniform(500, [12.6, 12.6, 12.6], seed=29)
    for v in ("3c08",):
        a = orc.brute(pos, box, truncation="pair", variant=v, terms=2)
        b = orc.brute(pos, box, truncation="product", variant=v, terms=2)
        assert b.n_triplets > a.n_triplets
        assert b.n_candidates == a.n_candidates


@pytest.mark.parametrize("c,inside", [(3.9, True), (3.91, False)])
def test_product_rule_boundary(orc, c, inside):
    """Product cutoff (Sec. 2): an isosceles triplet with sides 2, 2, c is
    kept iff 2*2*c < rc^3 = 15.625, although its long side exceeds rc, while
    the pairwise cutoff always drops it."""
    box = np.array([20.0, 20.0, 20.0])  # 8 cells of side 2.5
    h = math.sqrt(4.0 - (c / 2) ** 2)
    pos = np.array([[2.6, 3.0, 3.0], [2.6 + c, 3.0, 3.0], [2.6 + c / 2, 3.0 + h, 3.0]])
    pr = orc.brute(pos, box, truncation="product", terms=2)
    pa = orc.brute(pos, box, truncation="pair", terms=2)
    assert pr.n_triplets == (1 if inside else 0)
    assert pa.n_triplets == 0
    if inside:
        d = [np.linalg.norm(pos[a] - pos[b]) for a, b in ((0, 1), (0, 2), (1, 2))]
        assert pr.e_atm == pytest.approx(orc.atm_energy(d[0], d[1], d[2], NU), rel=1e-12)


def _comb(n, k):
    return math.comb(int(n), k)


def _block_sets(variant):
    """Cell sets visited per base cell, as offset tuples (Sec. 3/4)."""
    if variant == "3c08":
        cube = list(itertools.product((0, 1), repeat=3))
        ones = [s for s in cube]
        pairs = [p for p in itertools.combinations(ones, 2)
                 if all(min(a[d], b[d]) == 0 for d in range(3) for a, b in [p])]
        trips = [t for t in itertools.combinations(ones, 3)
                 if all(min(c[d] for c in t) == 0 for d in range(3))]
        return pairs, trips
    fwd = [o for o in itertools.product((-1, 0, 1), repeat=3) if (o[2], o[1], o[0]) > (0, 0, 0)]
    pairs = [((0, 0, 0), o) for o in fwd]
    trips = [((0, 0, 0), a, b) for a, b in itertools.combinations(fwd, 2)]
    return pairs, trips


@pytest.mark.parametrize("variant", ["3c08", "3c18", "3c01"])
def test_candidates_follow_counting_equations(orc, variant):
    """The number of molecule triplets a traversal visits equals the sum over
    base cells of eq. (celltriplet), eq. (twoonetriplets) and
    eq. (carttriplets) over its cell sets (3c08: 13 pairs and 44 triples of
    the 2x2x2 block with the base as minimum corner; 3c18: the 13 forward
    neighbours and their 78 pairs); 3c01 visits C(M-1, 2) pairs per molecule,
    M the population of its 27-cell neighbourhood."""
    L = 12.6
    pos, box = workloads.uniform(400, [L, L, L], seed=30)
    cxyz, clin, nc = orc.bin_cells(pos, box, RC)
    occ = np.zeros(tuple(nc[::-1]), dtype=np.int64)  # [z][y][x]
    for c in cxyz:
        occ[c[2], c[1], c[0]] += 1

    def N(b, o):
        return occ[(b[2] + o[2]) % nc[2], (b[1] + o[1]) % nc[1], (b[0] + o[0]) % nc[0]]

    total = 0
    if variant == "3c01":
        for c in cxyz:
            M = sum(N(c, o) for o in itertools.product((-1, 0, 1), repeat=3))
            total += _comb(M - 1, 2)
    else:
        pairs, trips = _block_sets(variant)
        assert len(pairs) == 13 and len(trips) == (44 if variant == "3c08" else 78)
        for b in itertools.product(range(nc[0]), range(nc[1]), range(nc[2])):
            total += _comb(N(b, (0, 0, 0)), 3)
            for p, q in pairs:
                total += N(b, q) * _comb(N(b, p), 2) + N(b, p) * _comb(N(b, q), 2)
            for p, q, r in trips:
                total += N(b, p) * N(b, q) * N(b, r)
    res = orc.brute(pos, box, truncation="product", variant=variant, terms=2)
    assert res.n_candidates == total


def test_total_interactions_identity():
    """eq. (totalInteractions): C(N,3) splits into the one-, two- and
    three-cell counts for any split N = N_b + N_n1 + N_n2."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        nb, n1, n2 = (int(v) for v in rng.integers(0, 30, 3))
        N = nb + n1 + n2

        def two(a, b):
            return b * _comb(a, 2) + a * _comb(b, 2)
        s = _comb(nb, 3) + _comb(n1, 3) + _comb(n2, 3) + two(nb, n1) + two(nb, n2) + two(n1, n2) + nb * n1 * n2
        assert s == _comb(N, 3)


# --------------------------------------------------------------------------
# Binning (Sec. 4: cell side >= rc, lexicographic order)
# --------------------------------------------------------------------------
def test_binning_edge_cases(orc):
    box = np.array([10.0, 10.0, 10.0])  # n = 4, side 2.5
    xs = [0.0, 2.5, np.nextafter(2.5, 0), 10.0, -0.1, -1e-300, np.nextafter(10.0, 0), 25.0, 7.5, -10.0]
    want = [0, 1, 0, 0, 3, 3, 3, 2, 3, 0]
    pos = np.array([[x, 0.0, 0.0] for x in xs])
    cxyz, clin, nc = orc.bin_cells(pos, box, RC)
    assert list(nc) == [4, 4, 4]
    assert list(cxyz[:, 0]) == want
    # lexicographic linear index, x fastest
    pos2 = np.array([[2.6, 5.1, 7.6]])
    c2, l2, _ = orc.bin_cells(pos2, box, RC)
    assert list(c2[0]) == [1, 2, 3] and l2[0] == (3 * 4 + 2) * 4 + 1
    # L / rc just above an integer
    n = orc.grid(np.array([10.000001, 12.5, 7.4999]), RC)
    assert list(n) == [4, 5, 2]


# --------------------------------------------------------------------------
# planar long-range correction of the LJ force (slab runs, Sec. 5.2)
# --------------------------------------------------------------------------
def _sheet_force_by_quadrature(xi, areal, rc, eps=1.0, sigma=1.0):
    """The definition integrated numerically: every molecule of a uniform
    sheet farther than rc pulls with the LJ pair force f(r) along the
    separation; only the z-components survive the lateral integral."""
    from scipy.integrate import quad

    def f(r):  # LJ pair force magnitude, positive when repulsive
        return 24.0 * eps * (2.0 * sigma ** 12 / r ** 13 - sigma ** 6 / r ** 7)

    s0 = np.sqrt(max(0.0, rc * rc - xi * xi))
    val, _ = quad(lambda s: f(np.hypot(s, xi)) * xi / np.hypot(s, xi) * 2.0 * np.pi * s, s0, np.inf,
                  epsabs=1e-14, epsrel=1e-12, limit=400)
    return areal * val


@pytest.mark.parametrize("xi", [0.3, 1.7, -2.2, 2.5, 2.9, -4.1, 7.0])
def test_sheet_force_matches_quadrature(xi):
    from oracle import slab
    got = float(slab.sheet_force(xi, 0.37, 2.5))
    ref = _sheet_force_by_quadrature(xi, 0.37, 2.5)
    assert got == pytest.approx(ref, rel=1e-9, abs=1e-13)


def test_lrc_vanishes_for_uniform_density_and_flips_under_mirror():
    from oracle import slab
    box = np.array([6.0, 5.0, 30.0])
    nb = 61
    # one molecule at the centre of every bin: uniform profile, the force on
    # each (at a bin centre) cancels pairwise (an odd bin count leaves no bin
    # at exactly half the box, whose minimum image is a tie)
    z = (np.arange(nb) + 0.5) * box[2] / nb
    pos = np.stack([np.full(nb, 1.0), np.full(nb, 2.0), z], axis=1)
    fz, hist = slab.lrc_forces(pos, box, nb, 2.5)
    assert (hist == 1).all()
    assert np.abs(fz).max() < 1e-12
    # a slab: mirroring z -> L_z - z mirrors the profile and flips the force
    rng = np.random.default_rng(5)
    p = np.concatenate([rng.uniform([0, 0, 10], [6, 5, 20], (300, 3)), rng.uniform([0, 0, 0], [6, 5, 30], (20, 3))])
    fz1, _ = slab.lrc_forces(p, box, 600, 2.5)
    q = p.copy()
    q[:, 2] = box[2] - p[:, 2]
    fz2, _ = slab.lrc_forces(q, box, 600, 2.5)
    # (no molecule sits on a bin edge here, so the bins mirror exactly)
    assert np.allclose(fz2, -fz1, rtol=0, atol=1e-12 * np.abs(fz1).max())
    # molecules inside the slab near its lower face are pulled up (+z)
    near = (p[:, 2] > 10.5) & (p[:, 2] < 12.0)
    assert (fz1[near] > 0).mean() > 0.9
    # no net force: bins act on each other with opposite forces
    assert abs(fz1.sum()) < 1e-12 * np.abs(fz1).sum()


# --------------------------------------------------------------------------
# diagonal of the virial tensor (pressure tensor, the interface motivation)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("trunc,var", [("pair", "3c08"), ("product", "3c08"), ("product", "3c18"),
                                       ("product", "3c01")])
def test_virial_diagonal_trace_and_axis_permutation(orc, trunc, var):
    """The trace equals the scalar virial (accumulated separately), and
    permuting the axes of positions and box permutes the diagonal."""
    box = np.array([11.0, 13.0, 14.0])
    pos, _ = workloads.rsa(400, box, 0.85, seed=77)
    wl, wa, r = orc.virial_diag(pos, box, truncation=trunc, variant=var)
    assert wl.sum() == pytest.approx(r.w_lj, rel=1e-12)
    assert wa.sum() == pytest.approx(r.w_atm, rel=1e-12)
    assert wa.sum() == pytest.approx(9.0 * r.e_atm, rel=1e-9)
    perm = [2, 0, 1]
    wl2, wa2, _ = orc.virial_diag(pos[:, perm], box[perm], truncation=trunc, variant=var)
    if var == "3c08" or trunc == "pair":  # cell sets are not symmetric under axis permutation otherwise
        assert np.allclose(wl2, wl[perm], rtol=1e-12)
        assert np.allclose(wa2, wa[perm], rtol=1e-10)


def test_virial_diagonal_is_isotropic_on_a_perfect_crystal(orc):
    """A perfect FCC lattice in a cubic box has cubic symmetry: equal
    diagonal components (pair rule, where the triplet set does not depend on
    the cell sets)."""
    from paper_2510_21230_amd import workloads as w
    pos = w.fcc_sites(4, 4, 4, (1.65, 1.65, 1.65)) + 0.3
    box = np.array([6.6, 6.6, 6.6])
    wl, wa, r = orc.virial_diag(pos, box, rc=2.2)
    assert r.n_triplets > 0
    assert np.allclose(wl, wl.mean(), rtol=1e-11)
    assert np.allclose(wa, wa.mean(), rtol=1e-11)
