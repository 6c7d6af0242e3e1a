"""Liquid-vapour slab with three-body forces (Sec. 5.2, Table 'rhoPars'): the
paper's protocol on the GPU, compared with the printed liquid and vapour
densities and interface widths (tests/golden/paper_slab.json).

Protocol as printed: N = 3800 at T = 0.9, dt = 0.004, rc = 2.5;
10,000 steps in a homogeneous 12.5 x 12.5 x 25 box, then the box extended to
12.5 x 12.5 x 75 with fresh zero-momentum velocities and 100,000 steps with
the long-range correction of the LJ forces (none for ATM); the z density
profile (600 bins) is sampled every step and each half fitted to a tanh
profile.  Choices the paper leaves open: an FCC lattice start (3800 of 4096
sites of 8 x 8 x 16 cells),
the isokinetic thermostat of the single-phase runs, the planar correction
of atm3_md_slab_lrc (the LJ force of the molecules beyond rc of laterally
uniform sheets, from the instantaneous profile), the liquid placed in the
middle third of the extended box, and the tanh profile with the sign that
puts the liquid inside (the printed formula carries the sum of the densities
in both terms).

With ATM the released block (rho 0.97, at high pressure) does not stay in
one piece: it cavitates in the middle within a few thousand steps, the two
halves move apart and merge across the periodic boundary within 10,000 to
30,000 steps (LJ alone keeps it whole).  The liquid therefore does not keep
its place: the profile is summed over chunks of 1,000 steps,
each rolled so that the liquid's circular centre of mass is in the middle,
and only the last 60,000 steps are used, without the chunks that do not
hold one slab (a liquid fragment in the vapour, or a vapour gap inside).
After each of those chunks the surface tension is sampled from the diagonal
of the pressure tensor (atm3_virial_diag plus the kinetic part, no
long-range part): gamma = L_z / 2 (P_zz - (P_xx + P_yy) / 2).  It is
printed, not tested: 60 samples give a standard error of about 0.2, more
than the three-body effect (sampled every 10 steps, tension_every=10, it is
resolved: 0.44 +- 0.05 for LJ alone, 0.31 +- 0.03 with ATM).

Reading of the width: the printed tanh formula is garbled (the sum of the
densities in both terms); with the tanh(2 (z - z0) / d) form used here the
LJ-only width is 2.33 against the printed 1.19, with tanh((z - z0) / d) it
is 1.16, so the printed d is read in the second convention (d / 2 here).

Tolerances cover sampling and the unstated choices: the paper's own
pairwise-cutoff traversal rows (identical triplets) spread by 0.0024 in
rho_l, 0.0012 in rho_g and 0.019 in d.  rho_l within 0.01, rho_g within
0.004, d / 2 within 20 % of the printed values, and the three-body shift of
rho_l (nu = 0.072 minus nu = 0) within 20 % of the printed one.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_slab.json")))
SKIP = 40000  # slab steps discarded before sampling (the spallation transient)


def fit_halves(profile, box, steps):
    """rho(z) from the summed histogram; tanh fit of each half (liquid in the
    middle): returns [(rho_l, rho_g, z0, d) left, (...) right]."""
    from scipy.optimize import curve_fit
    nb = len(profile)
    lz = box[2]
    dz = lz / nb
    z = (np.arange(nb) + 0.5) * dz
    rho = profile / (steps * box[0] * box[1] * dz)
    out = []
    for side in (-1.0, 1.0):  # left interface: liquid at larger z
        sel = z < lz / 2 if side < 0 else z >= lz / 2

        def f(zz, rl, rg, z0, d):
            return 0.5 * (rl + rg) - side * 0.5 * (rl - rg) * np.tanh(2.0 * (zz - z0) / d)

        z0 = lz / 3 if side < 0 else 2 * lz / 3
        p, _ = curve_fit(f, z[sel], rho[sel], p0=[0.7, 0.02, z0, 1.5])
        out.append(tuple(float(v) for v in p))
    return out


def recentre(profile):
    """Roll a z profile (per-bin counts) so that the liquid's circular centre
    of mass sits in the middle bin (integer bin shifts: counts unchanged)."""
    nb = len(profile)
    th = 2.0 * math.pi * (np.arange(nb) + 0.5) / nb
    w = np.asarray(profile, dtype=np.float64)
    c = math.atan2(float((w * np.sin(th)).sum()), float((w * np.cos(th)).sum()))
    centre = (c / (2.0 * math.pi)) % 1.0 * nb - 0.5
    return np.roll(profile, int(round(nb / 2 - 0.5 - centre)))


def slab_run(nu, truncation="pair", variant="3c08", steps_h=None, steps_s=None, skip=None, chunk=1000,
             tension_every=1000, seed=workloads.SEED_BASE + 70):
    """The Sec. 5.2 protocol; the profile is accumulated in chunks of `chunk`
    steps, each recentred on the liquid, and averaged after the first `skip`
    steps; the surface tension is sampled every `tension_every` steps (a
    divisor of `chunk`) after them.  Returns (left fit, right fit, summed
    profile, chunks used, chunk profiles, tension samples)."""
    import torch
    import paper_2510_21230_amd as atm3
    T, dt, rc, nb = G["T"], G["dt"], G["rc"], G["bins"]
    steps_h = steps_h or G["steps_homogeneous"]
    steps_s = steps_s or G["steps_slab"]
    skip = SKIP if skip is None else skip
    kw = dict(rc=rc, nu=nu, truncation=truncation, variant=variant)
    if nu == 0.0:
        kw["terms"] = atm3.TERM_LJ
    pos, box_h = workloads.fcc_box(G["n"], G["box_homogeneous"])
    p = torch.from_numpy(pos).cuda()
    v = torch.from_numpy(workloads.maxwell(G["n"], T, seed=seed)).cuda()
    atm3.md_nvt(p, v, box_h, steps_h, dt, T, sample_every=steps_h, **kw)
    # extend the box: the liquid fills the middle third
    lzh = G["box_homogeneous"][2]
    p[:, 2] = p[:, 2] - lzh * torch.floor(p[:, 2] / lzh) + lzh
    box = np.array(G["box_slab"])
    v = torch.from_numpy(workloads.maxwell(G["n"], T, seed=seed + 1)).cuda()
    chunks = torch.zeros((steps_s // chunk, nb), dtype=torch.int64, device="cuda")
    ctx = atm3.context(0)
    tension = []
    sample = not (truncation == "product" and variant == "3c01")
    for c in range(steps_s // chunk):
        sub = tension_every if (sample and c * chunk >= skip) else chunk
        for _ in range(chunk // sub):
            atm3.md_nvt(p, v, box, sub, dt, T, sample_every=sub, lrc_bins=nb, profile=chunks[c], **kw)
            if sub == tension_every and c * chunk >= skip and sample:
                # pressure tensor diagonal, P_aa V = sum v_a^2 + W_aa (no
                # long-range part), and the tension of the two interfaces
                wl, wa = ctx.virial_diag(p, box, **kw)
                pv = (v * v).sum(dim=0).cpu().numpy() + wl + wa
                pzz, pt = pv[2], 0.5 * (pv[0] + pv[1])
                tension.append(0.5 * box[2] * (pzz - pt) / float(np.prod(box)))
    chunks = chunks.cpu().numpy()
    assert (chunks.sum(axis=1) == G["n"] * chunk).all()
    prof, used = profile_of(chunks, skip // chunk, chunk, box)
    return fit_halves(prof.astype(np.float64), box, used * chunk) + [prof, used, chunks, np.array(tension)]


def profile_of(chunks, first, chunk, box):
    """Sum of the recentred chunk profiles from chunk `first` on that hold
    one slab; returns (profile, chunks used)."""
    used = [r for r in (recentre(h) for h in chunks[first:]) if single_slab(r, chunk, box)]
    assert 2 * len(used) >= len(chunks) - first, "the liquid did not gather into one slab"
    return sum(used), len(used)


def single_slab(profile, steps, box):
    """True if a recentred chunk profile holds one slab: every 20-bin block
    of the outer third below density 0.2 (no fragment in the vapour) and
    every block of the middle third above 0.45 (no vapour gap in the
    liquid)."""
    nb = len(profile)
    rho = profile / (steps * box[0] * box[1] * box[2] / nb)
    blocks = rho[: nb // 20 * 20].reshape(-1, 20).mean(axis=1)
    k = len(blocks)
    outer = np.concatenate([blocks[: k // 6], blocks[k - k // 6:]])
    middle = blocks[k // 3: k - k // 3]
    return bool(outer.max() < 0.2 and middle.min() > 0.45)


def test_tanh_fit_recovers_a_profile():
    """The fit on a synthetic profile with known parameters (CPU)."""
    box = np.array(G["box_slab"])
    nb = 600
    z = (np.arange(nb) + 0.5) * box[2] / nb
    rl, rg, d = 0.7, 0.017, 1.4
    rho = np.where(z < 37.5, 0.5 * (rl + rg) + 0.5 * (rl - rg) * np.tanh(2 * (z - 20.5) / d),
                      0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh(2 * (z - 54.2) / d))
    steps = 10
    prof = rho * steps * box[0] * box[1] * box[2] / nb
    (l, r) = fit_halves(prof, box, steps)
    assert l == pytest.approx((rl, rg, 20.5, d), rel=1e-6)
    assert r == pytest.approx((rl, rg, 54.2, d), rel=1e-6)


@pytest.mark.gpu
def test_slab_table():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    res = {}
    for key, nu in [("lj", 0.0), ("3c08_pair", G["nu"])]:
        print(f"[slab] {key}", flush=True)
        sys.stdout.flush()
        l, r, _, _, _, tension = slab_run(nu)
        mean = [(a + b) / 2 for a, b in zip(l, r)]
        res[key] = mean
        ref = G["rows"][key]
        res[key + "_gamma"] = float(tension.mean())
        print(f"  rho_l {mean[0]:.4f} (paper {ref['rho_l']})  rho_g {mean[1]:.4f} (paper {ref['rho_g']})  "
              f"d/2 {mean[3] / 2:.3f} (paper {ref['d']})  z0 {l[2]:.2f} / {r[2]:.2f}  "
              f"gamma {tension.mean():.3f} +- {tension.std(ddof=1) / math.sqrt(len(tension)):.3f}", flush=True)
        assert abs(mean[0] - ref["rho_l"]) < 0.01
        assert abs(mean[1] - ref["rho_g"]) < 0.004
        assert abs(mean[3] / 2 - ref["d"]) < 0.2 * ref["d"]
    shift = res["3c08_pair"][0] - res["lj"][0]
    ref_shift = G["rows"]["3c08_pair"]["rho_l"] - G["rows"]["lj"]["rho_l"]
    assert abs(shift - ref_shift) < 0.2 * abs(ref_shift), (shift, ref_shift)


def test_recentre_moves_the_liquid_to_the_middle():
    """A slab across the periodic boundary ends up centred (CPU)."""
    p = np.zeros(600, dtype=np.int64)
    p[550:] = 7
    p[:50] = 7
    r = recentre(p)
    assert r.sum() == p.sum()
    nz = np.nonzero(r)[0]
    assert nz.min() == 250 and nz.max() == 349


def test_single_slab_filter():
    """A chunk with a liquid fragment in the vapour is rejected (CPU)."""
    box = np.array(G["box_slab"])
    steps = 10
    per_bin = steps * box[0] * box[1] * box[2] / 600
    rho = np.full(600, 0.02)
    rho[200:400] = 0.7
    assert single_slab(rho * per_bin, steps, box)
    rho[20:60] = 0.6
    assert not single_slab(rho * per_bin, steps, box)
    rho[20:60] = 0.02
    rho[280:320] = 0.05  # two slabs with a gap, centred on the gap
    assert not single_slab(rho * per_bin, steps, box)
