"""GPU path (through the C ABI) against the FP64 oracle.

Bars: cell indices, cell starts, permutation and pair/triplet counts
bit-exact; forces within 1e-5 in the norm
    max_i |F_gpu,i - F_ref,i| / max(|F_ref,i|, F_rms)
(total forces, and ATM-only forces separately); energies and virials within
1e-6 relative.
"""
import sys

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

pytestmark = pytest.mark.gpu

RC, NU = 2.5, 0.073
FTOL, ETOL = 1e-5, 1e-6


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
    if frms == 0.0:
        return float(np.max(np.linalg.norm(fg - fr, axis=1)))
    return float(np.max(np.linalg.norm(fg - fr, axis=1) / np.maximum(nref, frms)))


def gpu_eval(torch, pos, box, **kw):
    import paper_2510_21230_amd as atm3
    f, r = atm3.compute_forces(torch.from_numpy(np.ascontiguousarray(pos)).to("cuda:0"), box, **kw)
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64), r


def check_against(ref, f, r, terms=3, exact_counts=True):
    if terms & 1:
        assert r["n_pairs"] == ref.n_pairs
        assert r["e_lj"] == pytest.approx(ref.e_lj, rel=ETOL, abs=1e-9)
        assert r["w_lj"] == pytest.approx(ref.w_lj, rel=ETOL, abs=1e-9)
    if terms & 2:
        assert r["n_triplets"] == ref.n_triplets
        assert r["e_atm"] == pytest.approx(ref.e_atm, rel=ETOL, abs=1e-12)
        assert r["w_atm"] == pytest.approx(ref.w_atm, rel=ETOL, abs=1e-12)
    err = force_err(f, ref.forces)
    assert err <= FTOL, err
    return err


# --------------------------------------------------------------------------
# binning: bit-exact against the oracle's FP64 cells and a stable sort
# --------------------------------------------------------------------------
def _binning_cases():
    p1, b1 = workloads.fcc(1000, 0.6, seed=workloads.SEED_BASE + 1)
    p2, b2 = workloads.uniform(3000, [13.0, 9.1, 17.7], seed=41)
    L = 10.0
    xs = np.array([0.0, 2.5, np.nextafter(2.5, 0), 10.0, -0.1, -1e-300, np.nextafter(10.0, 0), 25.0, 7.5, -10.0])
    p3 = np.stack([xs, xs[::-1], np.roll(xs, 3)], axis=1)
    p3 = np.concatenate([p3, workloads.uniform(50, [L, L, L], seed=42)[0]])
    # runs of equal cells in consecutive molecules, of random lengths (1-90),
    # across wave boundaries, N not a multiple of 64
    rng = np.random.default_rng(43)
    b4 = np.array([20.0, 15.0, 12.5])
    lens = rng.integers(1, 91, 120)
    anchors = rng.uniform(0.0, 1.0, (len(lens), 3)) * b4
    p4 = np.concatenate([a + rng.uniform(-0.3, 0.3, (m, 3)) for a, m in zip(anchors, lens)])
    # cell-count scans of exactly 4,096 tiles of 1,024 cells (256 x 128 x 128
    # cells) and of more (162^3 cells: the separate scan of the tile totals)
    b5 = np.array([640.0, 320.0, 320.0])
    p5 = workloads.uniform(20000, b5, seed=44)[0]
    b6 = np.array([405.0, 405.0, 405.0])
    p6 = workloads.uniform(20000, b6, seed=45)[0]
    return [("fcc1k", p1, b1), ("ortho", p2, b2), ("edges", p3, np.array([L, L, L])), ("runs", p4, b4),
            ("tiles4096", p5, b5), ("tiles4152", p6, b6)]


@pytest.mark.parametrize("case", range(6))
def test_binning_bit_exact(torch_cuda, orc, case):
    import paper_2510_21230_amd as atm3
    name, pos, box = _binning_cases()[case]
    _say(f"[binning] {name} n={len(pos)}")
    cxyz, clin, nc = orc.bin_cells(pos, box, RC)
    cell_of, start, perm, ncell = atm3.bin_cells(torch_cuda.from_numpy(pos).to("cuda:0"), box, RC)
    torch_cuda.cuda.synchronize()
    assert tuple(ncell) == tuple(int(v) for v in nc)
    assert np.array_equal(cell_of.cpu().numpy(), clin)
    ncells = int(np.prod(nc))
    ref_start = np.concatenate([[0], np.cumsum(np.bincount(clin, minlength=ncells))])
    assert np.array_equal(start.cpu().numpy(), ref_start)
    assert np.array_equal(perm.cpu().numpy(), np.argsort(clin, kind="stable"))


# --------------------------------------------------------------------------
# FCC rho 0.6, N = 1000: one evaluation against O(N^3) brute force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("terms", [3, 2, 1])
def test_fcc1k_against_brute_force(torch_cuda, orc, terms):
    pos, box = workloads.make("fcc1k")
    _say(f"[fcc1k] terms={terms}")
    ref = orc.brute(pos, box, rc=RC, nu=NU, terms=terms)
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=terms)
    err = check_against(ref, f, r, terms)
    assert r["ncell"] == (4, 4, 4)
    _say(f"  force err {err:.2e}  triplets {r['n_triplets']}  pairs {r['n_pairs']}")


# --------------------------------------------------------------------------
# seeded small systems: uniform, orthorhombic, clustered, empty cells,
# pairs placed at rc (1 +- 1e-7), several tiles and ragged blocks
# --------------------------------------------------------------------------
def _fuzz_case(k):
    """Seeded physical small systems: molecules never closer than 0.8 sigma
    (an LJ fluid never gets closer), ragged blocks and several tiles."""
    rng = np.random.default_rng(1000 + k)
    if k % 5 == 0:  # uniform, orthorhombic, 3-5 cells per dimension
        box = rng.uniform(7.6, 13.0, 3)
        n = int(rng.integers(50, int(0.45 * np.prod(box))))
        pos, _ = workloads.rsa(n, box, 0.8, seed=2000 + k)
    elif k % 5 == 1:  # dense clusters with empty cells in between
        box = np.array([12.5, 10.0, 15.0])
        parts = []
        for c in range(3):
            lo = rng.uniform(0, 1, 3) * box
            parts.append(workloads.rsa(80, box, 0.85, lo=lo, hi=lo + 4.5, seed=2100 + 10 * k + c)[0])
        pos = np.concatenate(parts)
        d = pos[:, None, :] - pos[None, :, :]
        d -= box * np.rint(d / box)
        r2 = (d ** 2).sum(axis=2) + np.eye(len(pos)) * 1e9
        keep = np.ones(len(pos), bool)
        for i in range(len(pos)):
            if keep[i] and (r2[i, keep] < 0.64).any():
                keep[i] = False
        pos = pos[keep]
    elif k % 5 == 2:  # pairs placed at rc (1 +- 1e-7), (1 +- 3e-6) and exactly rc
        box = np.array([10.0, 10.0, 10.0])
        base, _ = workloads.rsa(80, box, 1.8, seed=3000 + k)
        d = rng.normal(size=(80, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        scale = RC * (1.0 + rng.choice([-1e-7, 1e-7, -3e-6, 3e-6, 0.0], size=(80, 1)))
        part = (base + d * scale) % box
        pos = base
        for q in part:  # keep partners that stay 0.8 sigma from everything else
            e = pos - q
            e -= box * np.rint(e / box)
            if (e ** 2).sum(axis=1).min() >= 0.64:
                pos = np.concatenate([pos, q[None]])
    elif k % 5 == 3:  # dense jittered lattice
        pos, box = workloads.fcc(864, 0.75, jitter=0.15, seed=4000 + k)
    else:  # one compressed crystallite (rho 1.19: blocks of > 128 molecules
        # take the big-block kernel), the rest of the box empty
        box = np.array([20.0, 20.0, 20.0])
        pos = workloads.fcc_sites(4, 4, 4, (1.5, 1.5, 1.5)) + 7.0
        pos = pos + rng.uniform(-0.05, 0.05, pos.shape)
    return pos, np.asarray(box, dtype=np.float64)


@pytest.mark.parametrize("k", range(10))
def test_fuzz_small_systems(torch_cuda, orc, k):
    pos, box = _fuzz_case(k)
    _say(f"[fuzz] k={k} n={len(pos)} box={box}")
    ref = orc.brute(pos, box, rc=RC, nu=NU)
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU)
    check_against(ref, f, r)
    ref2 = orc.brute(pos, box, rc=RC, nu=NU, terms=2)
    f2, r2 = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=2)
    check_against(ref2, f2, r2, terms=2)
    assert r["n_candidates"] == ref.n_candidates


# --------------------------------------------------------------------------
# larger workloads against the per-molecule oracle (every molecule)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["fcc32k", "slab20k"])
def test_larger_workloads_full(torch_cuda, orc, name):
    pos, box = workloads.make(name)
    _say(f"[{name}] n={len(pos)}")
    ref = orc.molecules(pos, box, rc=RC, nu=NU)
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU)
    err = check_against(ref, f, r)
    ref2 = orc.molecules(pos, box, rc=RC, nu=NU, terms=2)
    f2, r2 = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=2)
    err2 = check_against(ref2, f2, r2, terms=2)
    _say(f"  force err {err:.2e} (ATM only {err2:.2e})")


def _candidates_3c08(cell_count, ncell):
    """Molecule triplets of the 3c08 cell sets from the cell populations:
    per base cell, the 2x2x2 block's corners a, b, c (3-bit offsets) with
    a & b & c == 0, counted per eqs. (celltriplet), (twoonetriplets) and
    (carttriplets)."""
    nx, ny, nz = ncell
    cnt = cell_count.reshape(nz, ny, nx).astype(np.int64)
    pop = [np.roll(cnt, shift=(-(o >> 2), -((o >> 1) & 1), -(o & 1)), axis=(0, 1, 2)) for o in range(8)]
    total = pop[0] * (pop[0] - 1) * (pop[0] - 2) // 6
    for a in range(8):
        for b in range(8):
            if a != b and (a & b) == 0:
                total = total + pop[a] * (pop[a] - 1) // 2 * pop[b]
    for a in range(8):
        for b in range(a + 1, 8):
            for c in range(b + 1, 8):
                if (a & b & c) == 0:
                    total = total + pop[a] * pop[b] * pop[c]
    return int(total.sum())


def test_fcc1m_full_size(torch_cuda, orc):
    """The full-size workload in the benchmark's launch configuration: every
    molecule's force against the per-molecule oracle, exact counts, and the
    candidate count against the counting equations."""
    pos, box = workloads.make("fcc1m")
    _say(f"[fcc1m] n={len(pos)}")
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU)
    ref = orc.molecules(pos, box, rc=RC, nu=NU)
    err = check_against(ref, f, r)
    _, clin, ncell = orc.bin_cells(pos, box, RC)
    counts = np.bincount(clin, minlength=int(np.prod(ncell)))
    assert r["n_candidates"] == _candidates_3c08(counts, ncell)
    f2, r2 = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=2)
    ref2 = orc.molecules(pos, box, rc=RC, nu=NU, terms=2)
    err2 = check_against(ref2, f2, r2, terms=2)
    _say(f"  force err {err:.2e} (ATM only {err2:.2e}); triplets {r['n_triplets']}")


def test_async_equals_sync_and_repeats(torch_cuda):
    import paper_2510_21230_amd as atm3
    from paper_2510_21230_amd import _lib
    torch = torch_cuda
    pos, box = workloads.make("fcc32k")
    _say("[async] fcc32k")
    p = torch.from_numpy(pos).to("cuda:0")
    f1, r1 = atm3.compute_forces(p, box)
    ctx = atm3.context(0)
    f2 = torch.empty_like(f1)
    res = torch.zeros(128, dtype=torch.uint8, device="cuda:0")
    for _ in range(3):
        ctx.compute_forces_async(p, box, f2, res, atm3.make_params())
    torch.cuda.synchronize()
    r2 = _lib.result_from_bytes(res.cpu().numpy().tobytes())
    # fixed-point force accumulation, a fixed pair order and fixed reduction
    # trees: every output is reproducible bit for bit
    assert r2 == r1
    assert torch.equal(f1, f2)


def test_invalid_arguments(torch_cuda):
    import paper_2510_21230_amd as atm3
    torch = torch_cuda
    pos, box = workloads.uniform(100, [7.0, 7.0, 7.0], seed=5)
    _say("[errors]")
    p = torch.from_numpy(pos).to("cuda:0")
    with pytest.raises(ValueError, match="box too small"):
        atm3.compute_forces(p, box)  # floor(7/2.5) = 2 < 3 cells
    with pytest.raises(ValueError):
        atm3.compute_forces(p, [10.0, 10.0, 10.0], rc=-1.0)
    with pytest.raises(ValueError):
        atm3.compute_forces(p.float(), [10.0, 10.0, 10.0])
    bad = pos.copy()
    bad[7, 1] = np.nan
    with pytest.raises(atm3.Atm3Error, match="not finite"):
        atm3.compute_forces(torch.from_numpy(bad).to("cuda:0"), [10.0, 10.0, 10.0], check_finite=True)
    ok, _ = workloads.rsa(100, [10.0, 10.0, 10.0], dmin=0.9, seed=6)
    f, r = atm3.compute_forces(torch.from_numpy(ok).to("cuda:0"), [10.0, 10.0, 10.0], check_finite=True)
    assert r["status"] == 0 and r["n_pairs"] > 0


def test_block_overflow_is_reported(torch_cuda):
    """More than 512 molecules in one 2x2x2 block: the kernels' own size
    check turns it into ATM3_EOVERFLOW (no out-of-range LDS access)."""
    import paper_2510_21230_amd as atm3
    torch = torch_cuda
    rng = np.random.default_rng(9)
    box = np.array([10.0, 10.0, 10.0])
    pos = np.concatenate([rng.uniform(0.1, 2.4, (600, 3)), rng.uniform(0, 10, (200, 3))])
    _say("[overflow]")
    with pytest.raises(atm3.Atm3Error, match="512"):
        atm3.compute_forces(torch.from_numpy(pos).to("cuda:0"), box)
    # a large but admissible block (between 128 and 512) takes the big-block path
    pos2 = workloads.fcc_sites(4, 4, 4, (1.5, 1.5, 1.5)) + 1.2
    pos2 = pos2 + rng.uniform(-0.05, 0.05, pos2.shape)
    import oracle
    ref = oracle.brute(pos2, box, terms=2)
    f, r = gpu_eval(torch, pos2, box, terms=2)
    check_against(ref, f, r, terms=2)


def test_dense_liquid_blocks_take_the_wide_tier(torch_cuda, orc):
    """A dense disordered packing (rho 0.85, molecules 0.72 sigma apart at
    least): many 2x2x2 blocks hold more than 1536 pairs within rc, more than
    the regular blocks' lists take, and go through the wide tier."""
    box = np.array([12.5, 12.5, 12.5])
    pos, _ = workloads.rsa(1660, box, dmin=0.72, seed=workloads.SEED_BASE + 41)
    _say(f"[dense liquid] n={len(pos)}")
    ref = orc.brute(pos, box, rc=RC, nu=NU)
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU)
    assert r["status"] == 0
    err = check_against(ref, f, r)
    assert r["n_candidates"] == ref.n_candidates
    # the ATM-only error at this density (the FP32 triplet arithmetic is the
    # part of the error that grows with density)
    ref2 = orc.brute(pos, box, rc=RC, nu=NU, terms=2)
    f2, r2 = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=2)
    err2 = check_against(ref2, f2, r2, terms=2)
    _say(f"  force err {err:.2e}, ATM only {err2:.2e}")


@pytest.mark.parametrize("case", ["fuzz", "fcc32k"])
def test_cutoff_3_takes_the_four_word_tier(torch_cuda, orc, case):
    """rc = 3.0 at density 0.7-0.75: a 2x2x2 block holds about 170-190
    molecules, beyond the two-word tier, so the four-word tier (up to 256
    molecules) is launched over every base cell directly (the dense liquid
    above takes it through the queue).  Whole-system parity against the
    oracle."""
    rc = 3.0
    if case == "fuzz":
        pos, box = workloads.rsa(1400, [13.0, 13.0, 13.0], dmin=0.85, seed=workloads.SEED_BASE + 44)
        ref = orc.brute(pos, box, rc=rc, nu=NU)
    else:
        pos, box = workloads.make("fcc32k")
        ref = orc.cells(pos, box, rc=rc, nu=NU)
    _say(f"[rc 3] {case} n={len(pos)}")
    f, r = gpu_eval(torch_cuda, pos, box, rc=rc, nu=NU)
    assert r["status"] == 0
    err = check_against(ref, f, r)
    _say(f"  force err {err:.2e}; triplets {r['n_triplets']}")


@pytest.mark.parametrize("terms", [3, 1])
def test_close_pair_takes_general_path(torch_cuda, orc, terms):
    """A pair at 0.5 sigma has an LJ force near 4e5, beyond the 2^18 range of
    the regular blocks' rounding conversion: those blocks are redone by the
    general path, and the result still matches the oracle."""
    pos, _ = workloads.rsa(300, [10.0, 10.0, 10.0], dmin=0.9, seed=17)
    box = np.array([10.0, 10.0, 10.0])
    e = pos[1:] - pos[0]
    e -= box * np.rint(e / box)
    far = np.sqrt((e ** 2).sum(axis=1)) > 1.45  # room for a partner at 0.5
    pos = np.concatenate([pos[:1], pos[1:][far]])
    pos = np.concatenate([pos, (pos[:1] + np.array([[0.5, 0.0, 0.0]])) % box])
    _say(f"[close pair] terms={terms} n={len(pos)}")
    ref = orc.brute(pos, box, rc=RC, nu=NU, terms=terms)
    assert np.abs(ref.forces).max() > 2.0 ** 18
    f, r = gpu_eval(torch_cuda, pos, box, rc=RC, nu=NU, terms=terms)
    assert r["status"] == 0
    check_against(ref, f, r, terms)
