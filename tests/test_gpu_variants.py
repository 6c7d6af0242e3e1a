"""The product cutoff and the 3c18 / 3c01 cell sets on the GPU against the
O(N^3) oracle: forces (1e-5 in the norm of the exact path), energies and
virials (1e-6 relative), pair / triplet / candidate counts exact."""
import sys

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

pytestmark = pytest.mark.gpu

RC, NU = 2.5, 0.073

# (truncation, variant, box side, molecules): at least 3 cells per dimension
# (5 for 3c18); the product cases span the minimum-image regimes of the
# one-sided kernel (both wraps, candidate-pair wrap only, none)
CASES = [
    ("pair", "3c18", 13.0, 1000),
    ("pair", "3c01", 8.0, 330),
    ("pair", "3c01", 13.0, 1000),
    ("product", "3c08", 13.0, 700),
    ("product", "3c18", 18.0, 900),
    ("product", "3c01", 18.0, 900),
    ("product", "3c08", 8.0, 330),
    ("product", "3c01", 8.0, 330),
    ("product", "3c01", 10.5, 600),
    ("product", "3c18", 13.0, 1000),
    ("product", "3c08", 20.5, 1400),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def force_err(fg, fr):
    nref = np.linalg.norm(fr, axis=1)
    frms = float(np.sqrt(np.mean(nref ** 2)))
    return float(np.max(np.linalg.norm(fg - fr, axis=1) / np.maximum(nref, frms)))


@pytest.mark.parametrize("case", range(len(CASES)))
def test_variant_against_brute_force(torch_cuda, orc, case):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    trunc, var, L, n = CASES[case]
    box = np.array([L, L, L])
    pos, _ = workloads.rsa(n, box, dmin=0.85, seed=workloads.SEED_BASE + 700 + case)
    _say(f"[{trunc} {var}] n={len(pos)} box={L}")
    ref = orc.brute(pos, box, rc=RC, nu=NU, truncation=trunc, variant=var)
    f, r = atm3.compute_forces(torch.from_numpy(pos).cuda(), box, nu=NU, truncation=trunc, variant=var)
    torch.cuda.synchronize()
    fg = f.cpu().numpy().astype(np.float64)
    err = force_err(fg, ref.forces)
    _say(f"  force err {err:.2e}; triplets {r['n_triplets']} (ref {ref.n_triplets}); candidates "
         f"{r['n_candidates']} (ref {ref.n_candidates})")
    assert r["n_pairs"] == ref.n_pairs
    assert r["n_triplets"] == ref.n_triplets
    assert r["n_candidates"] == ref.n_candidates
    assert err <= 1e-5
    assert r["e_lj"] == pytest.approx(ref.e_lj, rel=1e-6)
    assert r["w_lj"] == pytest.approx(ref.w_lj, rel=1e-6)
    assert r["e_atm"] == pytest.approx(ref.e_atm, rel=1e-6)
    assert r["w_atm"] == pytest.approx(ref.w_atm, rel=1e-6)


def test_small_boxes_are_rejected(torch_cuda):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.uniform(300, [11.0, 11.0, 11.0], seed=5)
    p = torch.from_numpy(pos).cuda()
    _say("[variant boxes]")
    with pytest.raises(ValueError, match="box too small"):
        atm3.compute_forces(p, box, variant="3c18")  # 4 cells < 5
    with pytest.raises(ValueError, match="box too small"):
        atm3.compute_forces(p, box, variant="3c18", truncation="product")


@pytest.mark.parametrize("k", range(9))
def test_fuzz_product_rule(torch_cuda, orc, k):
    """Seeded orthorhombic boxes of 3-7 cells per dimension (5-7 for 3c18),
    molecules at least 0.8 sigma apart, every cell set under the product
    rule: counts exact, forces and energies as above."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    var = ["3c08", "3c18", "3c01"][k % 3]
    rng = np.random.default_rng(4200 + k)
    lo = 12.6 if var == "3c18" else 7.6
    box = rng.uniform(lo, 18.0, 3)
    n = int(rng.integers(100, int(min(1200, 0.5 * np.prod(box)))))
    pos, _ = workloads.rsa(n, box, 0.8, seed=4300 + k)
    _say(f"[fuzz product {var}] k={k} n={len(pos)} box={np.round(box, 2)}")
    ref = orc.brute(pos, box, rc=RC, nu=NU, truncation="product", variant=var)
    f, r = atm3.compute_forces(torch.from_numpy(pos).cuda(), box, nu=NU, truncation="product", variant=var)
    torch.cuda.synchronize()
    assert r["n_pairs"] == ref.n_pairs
    assert r["n_triplets"] == ref.n_triplets
    assert r["n_candidates"] == ref.n_candidates
    assert force_err(f.cpu().numpy().astype(np.float64), ref.forces) <= 1e-5
    assert r["e_atm"] == pytest.approx(ref.e_atm, rel=1e-6)
    assert r["w_atm"] == pytest.approx(ref.w_atm, rel=1e-6)
    assert r["e_lj"] == pytest.approx(ref.e_lj, rel=1e-6)


@pytest.mark.parametrize("var", ["3c08", "3c18", "3c01"])
def test_product_rule_fcc32k_sampled(torch_cuda, orc, var):
    """The product rule on fcc32k (14^3 cells: one one-sided block per cell
    for the LJ part, one block-kernel block per base cell): forces of 200
    sampled molecules against the per-molecule oracle, and the LJ pairs,
    energy and virial equal to the pairwise-cutoff path's."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.make("fcc32k")
    p = torch.from_numpy(pos).cuda()
    _say(f"[product fcc32k {var}]")
    f, r = atm3.compute_forces(p, box, nu=NU, truncation="product", variant=var)
    _, r2 = atm3.compute_forces(p, box, nu=NU)
    torch.cuda.synchronize()
    assert r["n_pairs"] == r2["n_pairs"]
    assert r["e_lj"] == pytest.approx(r2["e_lj"], rel=1e-9)
    assert r["w_lj"] == pytest.approx(r2["w_lj"], rel=1e-9)
    sample = np.random.default_rng(11).choice(len(pos), 200, replace=False)
    ref = orc.molecules(pos, box, rc=RC, nu=NU, truncation="product", variant=var, sample=sample)
    fg = f.cpu().numpy().astype(np.float64)[sample]
    assert force_err(fg, ref.forces) <= 1e-5


@pytest.mark.parametrize("trunc,var,terms", [("pair", "3c08", 3), ("pair", "3c18", 2), ("product", "3c08", 3),
                                             ("product", "3c18", 3), ("product", "3c08", 1)])
def test_virial_diagonal_against_oracle(torch_cuda, orc, trunc, var, terms):
    """atm3_virial_diag: the diagonal of the LJ and ATM virial tensors
    against the O(N^3) oracle (1e-5 of the largest component), and the
    trace equal to the scalar virial of atm3_compute_forces."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    box = np.array([13.0, 14.0, 15.5])
    pos, _ = workloads.rsa(900, box, dmin=0.85, seed=workloads.SEED_BASE + 720)
    _say(f"[virial tensor {trunc} {var} terms={terms}] n={len(pos)}")
    wl_ref, wa_ref, ref = orc.virial_diag(pos, box, rc=RC, nu=NU, truncation=trunc, variant=var, terms=terms)
    ctx = atm3.context(0)
    p = torch.from_numpy(pos).cuda()
    wl, wa = ctx.virial_diag(p, box, rc=RC, nu=NU, truncation=trunc, variant=var, terms=terms)
    _, r = atm3.compute_forces(p, box, rc=RC, nu=NU, truncation=trunc, variant=var, terms=terms)
    _say(f"  lj {wl} (ref {wl_ref})  atm {wa} (ref {wa_ref})")
    for got, want in ((wl, wl_ref), (wa, wa_ref)):
        scale = max(np.abs(want).max(), 1e-12)
        assert np.abs(got - want).max() <= 1e-5 * scale
    if terms & 1:
        assert wl.sum() == pytest.approx(r["w_lj"], rel=1e-6)
    if terms & 2:
        assert wa.sum() == pytest.approx(r["w_atm"], rel=1e-5)
    else:
        assert np.all(wa == 0.0)


@pytest.mark.parametrize("var,L,n", [("3c08", 13.0, 2000), ("3c18", 15.2, 2900)])
def test_product_rule_dense_mixes_both_tiers(torch_cuda, orc, var, L, n):
    """Dense packings (density 0.91 and 0.83, molecules 0.8 sigma apart at
    least) under the product rule: about 40 % of the 3c08 blocks hold more
    than the 128 molecules of the shell-pruned tier and about 25 % of the
    3c18 cell sets more than its 192, so one evaluation mixes that tier with
    the blocks it hands on to k_prod_block.  Whole-system parity against the
    O(N^3) oracle."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    box = np.array([L, L, L])
    pos, _ = workloads.rsa(n, box, dmin=0.8, seed=workloads.SEED_BASE + 730)
    _say(f"[dense product {var}] n={len(pos)} box={L}")
    ref = orc.brute(pos, box, rc=RC, nu=NU, truncation="product", variant=var)
    f, r = atm3.compute_forces(torch.from_numpy(pos).cuda(), box, nu=NU, truncation="product", variant=var)
    torch.cuda.synchronize()
    assert r["status"] == 0
    assert (r["n_pairs"], r["n_triplets"], r["n_candidates"]) == (ref.n_pairs, ref.n_triplets, ref.n_candidates)
    err = force_err(f.cpu().numpy().astype(np.float64), ref.forces)
    _say(f"  force err {err:.2e}; triplets {r['n_triplets']}")
    assert err <= 1e-5
    for key in ("e_lj", "e_atm", "w_lj", "w_atm"):
        assert r[key] == pytest.approx(getattr(ref, key), rel=1e-6), key


@pytest.mark.parametrize("var", ["3c08", "3c18"])
def test_product_rule_fcc1m_sampled(torch_cuda, orc, var):
    """The product rule at the benchmark size (fcc1m: N = 10^6, 44^3 cells,
    the shell-pruned tier with the LJ pairs folded in, as timed): forces of
    2,000 seeded-random molecules against the per-molecule FP64 oracle, the
    evaluation reproducible bit for bit, and the LJ pairs, energy and virial
    equal to the pairwise-cutoff path's."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.make("fcc1m")
    p = torch.from_numpy(pos).cuda()
    _say(f"[product fcc1m {var}]")
    f, r = atm3.compute_forces(p, box, nu=NU, truncation="product", variant=var)
    f2, r2 = atm3.compute_forces(p, box, nu=NU, truncation="product", variant=var)
    _, rp = atm3.compute_forces(p, box, nu=NU)
    torch.cuda.synchronize()
    assert r["status"] == 0
    assert torch.equal(f, f2) and r == r2
    assert r["n_pairs"] == rp["n_pairs"]
    assert r["e_lj"] == pytest.approx(rp["e_lj"], rel=1e-9)
    assert r["w_lj"] == pytest.approx(rp["w_lj"], rel=1e-9)
    sample = np.sort(np.random.default_rng(12).choice(len(pos), 2000, replace=False))
    ref = orc.molecules(pos, box, rc=RC, nu=NU, truncation="product", variant=var, sample=sample)
    err = force_err(f.cpu().numpy().astype(np.float64)[sample], ref.forces)
    _say(f"  force err {err:.2e} over 2000 molecules; triplets {r['n_triplets']}")
    assert err <= 1e-5


@pytest.mark.parametrize("case", ["fuzz", "fcc32k"])
def test_product_rule_cutoff_3_takes_the_three_word_tier(torch_cuda, orc, case):
    """The product rule (3c08) at rc = 3.0 and density 0.65-0.75: a 2x2x2
    block holds about 170 molecules, beyond the 128 of the two-word
    shell-pruned tier, so its three-word version (192 molecules) runs over
    every base cell and hands on the larger blocks.  The fuzz case against
    the O(N^3) oracle (whole system), fcc32k on 1,000 sampled molecules
    against the per-molecule oracle."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    rc = 3.0
    if case == "fuzz":
        pos, box = workloads.rsa(1400, [13.0, 13.0, 13.0], dmin=0.85, seed=workloads.SEED_BASE + 45)
    else:
        pos, box = workloads.make("fcc32k")
    _say(f"[product rc 3] {case} n={len(pos)}")
    f, r = atm3.compute_forces(torch.from_numpy(pos).cuda(), box, rc=rc, nu=NU, truncation="product")
    torch.cuda.synchronize()
    assert r["status"] == 0
    fg = f.cpu().numpy().astype(np.float64)
    if case == "fuzz":
        ref = orc.brute(pos, box, rc=rc, nu=NU, truncation="product")
        assert (r["n_pairs"], r["n_triplets"], r["n_candidates"]) == (ref.n_pairs, ref.n_triplets, ref.n_candidates)
        err = force_err(fg, ref.forces)
        for key in ("e_lj", "e_atm", "w_lj", "w_atm"):
            assert r[key] == pytest.approx(getattr(ref, key), rel=1e-6), key
    else:
        sample = np.sort(np.random.default_rng(13).choice(len(pos), 1000, replace=False))
        ref = orc.molecules(pos, box, rc=rc, nu=NU, truncation="product", sample=sample)
        err = force_err(fg[sample], ref.forces)
    _say(f"  force err {err:.2e}; triplets {r['n_triplets']}")
    assert err <= 1e-5
