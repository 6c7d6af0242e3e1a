"""The no-allocation entry point (atm3_compute_forces_noalloc) against the
allocating one (atm3_compute_forces_async): same kernels, so the forces and
the result struct must agree bit for bit.  Two calls in a row, the second
on a smaller input (the fixed array keeps the first call's contents), one
at the size limit, and the host-side limit checks."""
import numpy as np
import pytest

from paper_2510_21230_amd import _lib, workloads

pytestmark = pytest.mark.gpu


def _run(ctx, fn, pos_np, box, **kw):
    import torch
    dev = ctx.device
    pos = torch.from_numpy(pos_np).to(dev)
    forces = torch.full((len(pos_np), 3), float("nan"), dtype=torch.float32, device=dev)
    res = torch.zeros(128, dtype=torch.uint8, device=dev)
    fn(pos, box, forces, res, _lib.make_params(**kw))
    torch.cuda.synchronize(dev)
    raw = res.cpu().numpy().tobytes()
    return forces.cpu().numpy(), raw[:72], _lib.result_from_bytes(raw)


def _same(ctx, pos, box, **kw):
    fa, ra, da = _run(ctx, ctx.compute_forces_async, pos, box, **kw)
    fb, rb, db = _run(ctx, ctx.compute_forces_noalloc, pos, box, **kw)
    print(f"n={len(pos)} {kw} triplets={db['n_triplets']} status={db['status']}", flush=True)
    assert da["status"] == 0 and db["status"] == 0, (da, db)
    assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32))
    assert ra == rb, (da, db)
    return db


def test_noalloc_equals_allocating_path_twice():
    import torch
    ctx = _lib.context(0)
    torch.cuda.set_device(0)
    pos, box = workloads.fcc(4000, 0.7, jitter=0.05, seed=workloads.SEED_BASE + 41)
    r1 = _same(ctx, pos, box, rc=2.5, nu=0.073)
    pos2, box2 = workloads.make("fcc1k")
    r2 = _same(ctx, pos2, box2, rc=2.5, nu=0.073, variant="3c01")
    assert r2["n_triplets"] < r1["n_triplets"]
    _same(ctx, pos2, box2, rc=2.5, nu=0.073, terms=_lib.TERM_ATM)


def test_noalloc_at_the_size_limit():
    ctx = _lib.context(0)
    pos, box = workloads.fcc(_lib.NOALLOC_MAX_N, 0.75, jitter=0.05, seed=workloads.SEED_BASE + 42)
    _same(ctx, pos, box, rc=2.5, nu=0.073, variant="3c18")


def test_noalloc_rejects_what_it_cannot_hold():
    import torch
    ctx = _lib.context(0)
    dev = ctx.device
    pos_np, box = workloads.fcc(_lib.NOALLOC_MAX_N + 1, 0.75, jitter=0.05, seed=workloads.SEED_BASE + 43)
    pos = torch.from_numpy(pos_np).to(dev)
    forces = torch.empty((len(pos_np), 3), dtype=torch.float32, device=dev)
    res = torch.zeros(128, dtype=torch.uint8, device=dev)
    with pytest.raises(ValueError, match="no-allocation limits"):
        ctx.compute_forces_noalloc(pos, box, forces, res, _lib.make_params())
    small, sbox = workloads.make("fcc1k")
    sp = torch.from_numpy(small).to(dev)
    with pytest.raises(ValueError, match="pairwise cutoff only"):
        ctx.compute_forces_noalloc(sp, sbox, forces, res, _lib.make_params(truncation="product"))
    # cells beyond the limit: a sparse box of 41^3 = 68,921 cells
    with pytest.raises(ValueError, match="no-allocation limits"):
        ctx.compute_forces_noalloc(sp, [41 * 2.5] * 3, forces, res, _lib.make_params())
