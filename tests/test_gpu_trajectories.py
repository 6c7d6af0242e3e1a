"""Molecular-dynamics trajectories on the GPU checked against the FP64 oracle
on the trajectory's own positions (the validation protocol of Sec. 5: MD with
both cutoff rules and every traversal).

* 32k fluid: N = 32,000 (jittered FCC 20^3 at density 0.7), Maxwell
  velocities at T = 1.0, 100 velocity-Verlet steps at dt = 0.002, for the
  pairwise and the product cutoff and the 3c08, 3c18 and 3c01 cell sets.
  Every 10 steps (pairwise cutoff) the forces of every molecule, the
  energies and the pair and triplet counts are compared with the oracle's
  linked-cell evaluation of the whole system; every 20 steps (product
  cutoff) the forces of 2,000 seeded-random molecules with the oracle's
  per-molecule evaluation.  The energy drift is reported: the potentials are
  truncated without a shift, so the drift is also given with the LJ energy
  shifted by u(rc) per pair inside rc, which removes the pair-crossing jumps.
* 20k slab: box 30 x 30 x 90, liquid slab of density 0.7 and vapour of
  density 0.02 (uneven cell occupancy), Maxwell velocities at T = 0.8, 200
  steps at dt = 0.002, forces, energies and counts against the oracle every
  20 steps, and the 600-bin density profile along z bit-exact against a
  numpy histogram of the same positions.

Bars: counts exact; forces max_i |dF_i| / max(|F_i|, F_rms) <= 1e-5;
energies and virials relative 1e-6.
"""
import sys

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

pytestmark = pytest.mark.gpu

RC, NU = 2.5, 0.073
U_RC = 4.0 * (RC ** -12 - RC ** -6)  # LJ energy of a pair at the cutoff


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _force_err(f_gpu, f_ref, f_rms=None):
    nref = np.linalg.norm(f_ref, axis=1)
    if f_rms is None:
        f_rms = float(np.sqrt(np.mean(nref ** 2)))
    return float(np.max(np.linalg.norm(f_gpu - f_ref, axis=1) / np.maximum(nref, f_rms)))


def _run(torch, pos, box, vel, steps, every, **kw):
    import paper_2510_21230_amd as atm3
    p = torch.from_numpy(pos.copy()).cuda()
    v = torch.from_numpy(vel.copy()).cuda()
    frames = []
    rec = atm3.md_run(p, v, box, steps, dt=0.002, record_every=every, frames=frames, nu=NU, **kw)
    torch.cuda.synchronize()
    return rec, frames


@pytest.mark.parametrize("trunc,var", [("pair", "3c08"), ("pair", "3c18"), ("pair", "3c01"),
                                       ("product", "3c08"), ("product", "3c18"), ("product", "3c01")])
def test_fluid32k_trajectory_against_oracle(torch_cuda, orc, trunc, var):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.make("fcc32k")
    n = len(pos)
    vel = workloads.maxwell(n, 1.0, seed=workloads.SEED_BASE + 70)
    every = 10 if trunc == "pair" else 20
    _say(f"[fluid32k] {trunc} {var}: n={n} 100 steps, check every {every}")
    rec, frames = _run(torch, pos, box, vel, 100, every, truncation=trunc, variant=var)
    e_shift = []
    worst = 0.0
    for (fpos, f), r0 in zip(frames, rec):
        step = r0["step"]
        x = fpos.cpu().numpy()
        fg = f.cpu().numpy().astype(np.float64)
        f2, r = atm3.compute_forces(fpos, box, nu=NU, truncation=trunc, variant=var)
        # the same positions give the same forces, bit for bit
        assert np.array_equal(f2.cpu().numpy(), f.cpu().numpy())
        if trunc == "pair":
            ref = orc.cells(x, box, rc=RC, nu=NU)
            assert r["n_pairs"] == ref.n_pairs, (step, r, ref.n_pairs)
            assert r["n_triplets"] == (3 if var == "3c01" else 1) * ref.n_triplets, (step, r, ref.n_triplets)
            for key in ("e_lj", "e_atm", "w_lj", "w_atm"):
                assert r[key] == pytest.approx(getattr(ref, key), rel=1e-6), (step, key)
            err = _force_err(fg, ref.forces)
        else:
            rng = np.random.default_rng(1000 + step)
            sample = np.sort(rng.choice(n, size=2000, replace=False))
            ref = orc.molecules(x, box, rc=RC, nu=NU, truncation=trunc, variant=var, sample=sample)
            err = _force_err(fg[sample], ref.forces)
        worst = max(worst, err)
        assert err <= 1e-5, (step, err)
        e_shift.append(r0["total"] - r["n_pairs"] * U_RC)
    e = np.array([r0["total"] for r0 in rec]) / n
    es = np.array(e_shift) / n
    _say(f"  max force error {worst:.2e}; E/N {e[0]:.6f} -> {e[-1]:.6f} (drift {e[-1] - e[0]:+.2e}); "
         f"with the LJ shift {es[0]:.6f} -> {es[-1]:.6f} (drift {es[-1] - es[0]:+.2e})")
    assert abs(es[-1] - es[0]) < 2e-3


def test_fluid32k_pair_rule_trajectories_agree_across_cell_sets(torch_cuda):
    """Under the pairwise cutoff every cell set includes the same triplets
    (and the same kernel evaluates them), so the three trajectories are
    bit-identical."""
    torch = torch_cuda
    pos, box = workloads.make("fcc32k")
    vel = workloads.maxwell(len(pos), 1.0, seed=workloads.SEED_BASE + 70)
    out = []
    for var in ("3c08", "3c18", "3c01"):
        _, frames = _run(torch, pos, box, vel, 30, 30, variant=var)
        out.append(frames[-1][0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_slab20k_trajectory_and_profile(torch_cuda, orc):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.make("slab20k")
    n = len(pos)
    vel = workloads.maxwell(n, 0.8, seed=workloads.SEED_BASE + 71)
    _say(f"[slab20k] n={n} box {box.tolist()} 200 steps at T 0.8, check every 20")
    rec, frames = _run(torch, pos, box, vel, 200, 20)
    worst = 0.0
    for (fpos, f), r0 in zip(frames, rec):
        step = r0["step"]
        x = fpos.cpu().numpy()
        _, r = atm3.compute_forces(fpos, box, nu=NU)
        ref = orc.cells(x, box, rc=RC, nu=NU)
        assert (r["n_pairs"], r["n_triplets"]) == (ref.n_pairs, ref.n_triplets), step
        for key in ("e_lj", "e_atm", "w_lj", "w_atm"):
            assert r[key] == pytest.approx(getattr(ref, key), rel=1e-6), (step, key)
        err = _force_err(f.cpu().numpy().astype(np.float64), ref.forces)
        worst = max(worst, err)
        assert err <= 1e-5, (step, err)
    e = np.array([r0["total"] for r0 in rec]) / n
    _say(f"  max force error {worst:.2e}; E/N {e[0]:.6f} -> {e[-1]:.6f}")
    # the 600-bin density profile of the final positions
    nbins = 600
    fpos = frames[-1][0]
    hist = torch.zeros(nbins, dtype=torch.int64, device=fpos.device)
    scratch = torch.zeros((n, 3), dtype=torch.float32, device=fpos.device)
    atm3.context(fpos.device).slab_lrc(fpos, box, scratch, nbins=nbins, rc=RC, hist_sum=hist)
    z = fpos.cpu().numpy()[:, 2]
    lz = float(box[2])
    zw = z - lz * np.floor(z / lz)
    k = np.clip(np.floor(zw * (nbins / lz)), 0, nbins - 1).astype(np.int64)
    ref_hist = np.bincount(k, minlength=nbins)
    assert np.array_equal(hist.cpu().numpy(), ref_hist)
    rho = ref_hist / (box[0] * box[1] * lz / nbins)
    zc = (np.arange(nbins) + 0.5) * lz / nbins
    liquid = rho[(zc > 35) & (zc < 55)].mean()
    vapour = rho[(zc < 20) | (zc > 70)].mean()
    _say(f"  profile: liquid {liquid:.3f}, vapour {vapour:.4f}")
    assert 0.6 < liquid < 0.8 and vapour < 0.06
