"""Velocity-Verlet driver on the GPU: one step against the same step done in
FP64 with the oracle's forces, the kinetic-energy reduction, time
reversibility and momentum conservation (NVE, dt = 0.002, T = 1.0 start)."""
import sys

import numpy as np
import pytest

from paper_2510_21230_amd import workloads

pytestmark = pytest.mark.gpu

RC, NU = 2.5, 0.073


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_one_step_matches_fp64_verlet(torch_cuda, orc):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.fcc(864, 0.7, jitter=0.05, seed=workloads.SEED_BASE + 60)
    vel = workloads.maxwell(len(pos), 1.0, seed=workloads.SEED_BASE + 61)
    dt = 0.002
    _say(f"[md step] n={len(pos)}")
    p = torch.from_numpy(pos.copy()).cuda()
    v = torch.from_numpy(vel.copy()).cuda()
    rec = atm3.md_run(p, v, box, 1, dt=dt, nu=NU)
    torch.cuda.synchronize()
    # the same step in FP64 with the oracle's forces
    f0 = orc.molecules(pos, box, rc=RC, nu=NU).forces
    v1 = vel + 0.5 * dt * f0
    x1 = pos + dt * v1
    f1 = orc.molecules(x1, box, rc=RC, nu=NU).forces
    v2 = v1 + 0.5 * dt * f1
    np.testing.assert_allclose(p.cpu().numpy(), x1, rtol=0, atol=1e-9)
    np.testing.assert_allclose(v.cpu().numpy(), v2, rtol=0, atol=1e-6)
    assert rec[0]["kinetic"] == pytest.approx(0.5 * np.sum(vel * vel), rel=1e-12)
    assert rec[1]["kinetic"] == pytest.approx(0.5 * np.sum(v2 * v2), rel=1e-9)


def test_reversibility_and_momentum(torch_cuda):
    """Velocity Verlet is time reversible: 20 steps forward, velocities
    reversed, 20 steps back return the start.  Newton's third law keeps the
    total momentum at zero.  (The total energy is not a conserved check here:
    the potentials are truncated without a shift, so pairs and triplets
    crossing rc change it in jumps; it is reported, not bounded.)"""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = workloads.fcc(4000, 0.7, jitter=0.0, seed=workloads.SEED_BASE + 62)
    vel = workloads.maxwell(len(pos), 1.0, seed=workloads.SEED_BASE + 63)
    p = torch.from_numpy(pos.copy()).cuda()
    v = torch.from_numpy(vel.copy()).cuda()
    _say(f"[md nve] n={len(pos)}")
    rec = atm3.md_run(p, v, box, 20, dt=0.002, record_every=10, nu=NU)
    mom = float(torch.linalg.norm(v.sum(dim=0)))
    v.neg_()
    atm3.md_run(p, v, box, 20, dt=0.002, record_every=20, nu=NU)
    torch.cuda.synchronize()
    back = float(np.max(np.abs(p.cpu().numpy() - pos)))
    e = [r["total"] / len(pos) for r in rec]
    _say(f"  E/N {e}; |sum v| after 20 steps {mom:.2e}; max |x_back - x0| {back:.2e}")
    assert back < 1e-6
    assert mom < 1e-6 * len(pos)
    np.testing.assert_allclose(-v.cpu().numpy(), vel, atol=1e-5)


def test_rescale_sets_kinetic_energy(torch_cuda):
    """atm3_md_rescale: sum v^2/2 = dof T / 2 afterwards (FP64 host check),
    directions unchanged; invalid temperature or dof are ATM3_EINVAL."""
    torch = torch_cuda
    import ctypes
    import paper_2510_21230_amd as atm3
    from paper_2510_21230_amd import _lib
    n = 1000
    vel = workloads.maxwell(n, 0.7, seed=workloads.SEED_BASE + 62)
    v = torch.from_numpy(vel.copy()).cuda()
    ctx = atm3.context(v.device)
    _say(f"[md rescale] n={n}")
    ctx._stream()
    ctx._check(ctx.lib.atm3_md_rescale(ctx.h, _lib._ptr(v), n, 1.25, 3 * n - 3))
    torch.cuda.synchronize()
    got = v.cpu().numpy()
    assert 0.5 * float((got * got).sum()) == pytest.approx(0.5 * (3 * n - 3) * 1.25, rel=1e-12)
    lam = got / vel
    assert np.allclose(lam, lam.flat[0], rtol=1e-12)
    for T, dof in [(0.0, 3 * n - 3), (-1.0, 3), (float("nan"), 3), (1.0, 0), (1.0, 3 * n + 1)]:
        assert ctx.lib.atm3_md_rescale(ctx.h, _lib._ptr(v), n, T, dof) == -1


def test_slab_correction_matches_oracle(torch_cuda):
    """atm3_md_slab_lrc: the z histogram bit for bit and the z-force of the
    planar LJ long-range correction within 3e-6 of the FP64 oracle, on a
    liquid slab with vapour (600 bins over L_z = 75, the paper's slab box);
    x and y untouched; the histogram accumulates over calls; invalid
    arguments are ATM3_EINVAL."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    from oracle import slab
    box = np.array([12.5, 12.5, 75.0])
    liq, _ = workloads.rsa(2600, box, dmin=0.85, lo=np.array([0.0, 0.0, 25.0]), hi=np.array([12.5, 12.5, 50.0]),
                           seed=workloads.SEED_BASE + 63)
    gas, _ = workloads.rsa(60, box, dmin=0.85, lo=np.array([0.0, 0.0, 55.0]), hi=np.array([12.5, 12.5, 95.0]),
                           seed=workloads.SEED_BASE + 64)
    pos = np.concatenate([liq, gas])  # the vapour band crosses the periodic boundary in z
    n = len(pos)
    _say(f"[slab lrc] n={n}")
    fz_ref, hist_ref = slab.lrc_forces(pos, box, 600, 2.5)
    ctx = atm3.context(0)
    p = torch.from_numpy(pos).cuda()
    f0 = np.random.default_rng(3).normal(size=(n, 3)).astype(np.float32)
    f = torch.from_numpy(f0.copy()).cuda()
    h = torch.zeros(600, dtype=torch.int64, device="cuda")
    ctx.slab_lrc(p, box, f, 600, rc=2.5, hist_sum=h)
    ctx.slab_lrc(p, box, torch.zeros_like(f), 600, rc=2.5, hist_sum=h)
    torch.cuda.synchronize()
    got = f.cpu().numpy()
    assert (h.cpu().numpy() == 2 * hist_ref).all()
    assert (got[:, :2] == f0[:, :2]).all()
    dz = got[:, 2].astype(np.float64) - f0[:, 2].astype(np.float64)
    scale = np.abs(fz_ref).max()
    assert scale > 0.1
    err = np.abs(dz - fz_ref).max() / scale
    _say(f"  max |F_z| {scale:.3f}, max error {err:.2e}")
    # FP64 sums; the one FP32 rounding of the updated force (|f| up to about
    # 4 here) is 2.4e-7 absolute, under 1e-6 of the largest correction
    assert err < 3e-6
    # molecules just inside the liquid's faces are pulled into the liquid
    assert (fz_ref[(pos[:, 2] > 25.2) & (pos[:, 2] < 26.5)] > 0).mean() > 0.9
    assert (fz_ref[(pos[:, 2] > 48.5) & (pos[:, 2] < 49.8)] < 0).mean() > 0.9
    for args in [dict(nbins=0), dict(nbins=5000), dict(rc=40.0), dict(rc=-1.0), dict(eps=0.0)]:
        kw = dict(nbins=600, rc=2.5, eps=1.0, sigma=1.0)
        kw.update(args)
        with pytest.raises(ValueError):
            ctx.slab_lrc(p, box, f, **kw)


@pytest.mark.parametrize("case", ["pair", "product", "slab"])
def test_graph_run_equals_eager(torch_cuda, case):
    """md_nvt with graph=True (one step captured as a HIP graph, launched per
    step) against the same steps launched one by one: every sampled result
    row, the final positions and velocities (and the slab profile) equal bit
    for bit, over two graph runs separated by eager work and a host
    synchronisation."""
    torch = torch_cuda
    import time
    import paper_2510_21230_amd as atm3
    if case == "slab":
        box = np.array([12.5, 12.5, 40.0])
        pos, _ = workloads.rsa(1500, box, dmin=0.9, lo=np.array([0.0, 0.0, 12.0]), hi=np.array([12.5, 12.5, 28.0]),
                               seed=workloads.SEED_BASE + 65)
        kw = dict(rc=2.5, nu=0.072, lrc_bins=320)
    else:
        pos, box = workloads.sc(1270, 12.5)
        kw = dict(rc=2.5, nu=0.072, truncation=case)
    vel = workloads.maxwell(len(pos), 1.0, seed=workloads.SEED_BASE + 66)
    _say(f"[md graph] {case} n={len(pos)}")
    out = {}
    for graph in (False, True):
        p = torch.from_numpy(pos.copy()).cuda()
        v = torch.from_numpy(vel.copy()).cuda()
        prof = torch.zeros(320, dtype=torch.int64, device="cuda") if case == "slab" else None
        extra = dict(profile=prof) if prof is not None else {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r1 = atm3.md_nvt(p, v, box, 150, 0.004, 1.0, sample_every=10, graph=graph, **extra, **kw)
        t1 = time.perf_counter()
        f, _ = atm3.compute_forces(p, box, rc=2.5, nu=0.072)  # eager work and a sync in between
        r2 = atm3.md_nvt(p, v, box, 150, 0.004, 1.0, sample_every=10, graph=graph, **extra, **kw)
        torch.cuda.synchronize()
        out[graph] = (r1, r2, p.cpu().numpy(), v.cpu().numpy(), None if prof is None else prof.cpu().numpy())
        _say(f"  graph={graph}: {1e3 * (t1 - t0) / 150:.3f} ms per step (first run)")
    a, b = out[False], out[True]
    assert a[0].shape == (15, 4)
    for x, y in zip(a, b):
        if x is not None:
            assert np.array_equal(x, y)
