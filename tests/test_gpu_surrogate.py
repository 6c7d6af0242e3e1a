"""GPU surrogate (through the C ABI) against the FP64 surrogate reference.

* neighbour pairs: the exact pair set of the reference (bit-exact decision);
* descriptors: FP32 kernels against FP64, |dD| <= 2e-4 (1 + |D|);
* forward s, t and the per-molecule force and error estimate: against the
  reference with the same bfloat16 operand rounding; what remains is FP32
  against FP64 accumulation order, which can move a BF16 rounding by one
  unit (2^-8 relative) in an activation;
* gradients (BF16 MFMA backward): per-tensor relative L2 error;
* Adam: FP32 update against the FP64 formula;
* exact fallback: threshold below every estimate reproduces the exact
  LJ + ATM forces of the per-molecule oracle (1e-5 bar of the exact path);
* a zero output layer leaves the exact LJ term alone (1e-5 / 1e-6 bars);
* training on the GPU lowers the force error below that of LJ alone.
"""
import sys

import numpy as np
import pytest

from oracle import surrogate as S
from paper_2510_21230_amd import workloads

pytestmark = pytest.mark.gpu

RC, NU = 2.5, 0.073
SHAPES = {"W1": (80, 128), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128, 128), "b3": (128,),
          "W4": (128, 2), "b4": (2,)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dict(flat):
    out, o = {}, 0
    for k in S.PARAM_ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(SHAPES[k])
        o += n
    assert o == len(flat)
    return out


def to_flat(d):
    return np.concatenate([np.asarray(d[k], dtype=np.float32).ravel() for k in S.PARAM_ORDER])


def _params(seed):
    p = S.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape)
    p["W4"] = rng.normal(0, 0.2, p["W4"].shape)
    p["b4"] = np.array([0.05, -1.0])
    return to_dict(to_flat(p))  # the FP32 values both sides use


def _system(n=600, rho=0.7, seed=3, jitter=0.12):
    return workloads.fcc(n, rho, jitter=jitter, seed=workloads.SEED_BASE + 40 + seed)


def _setup(torch, pos, box, params, seed=0):
    import paper_2510_21230_amd as atm3
    pairs, disp = S.neighbour_pairs(pos, box, RC)
    draw = S.raw_descriptors(len(pos), pairs, disp, RC)
    m64, s64 = S.descriptor_stats(draw)
    m32, s32 = m64.astype(np.float32), s64.astype(np.float32)
    mlp = atm3.Mlp(seed=seed)
    mlp.set_params(to_flat(params))
    mlp.set_stats(m32, s32)
    stats = (m32.astype(np.float64), s32.astype(np.float64))
    return mlp, stats, pairs, disp


def _canon(ij, vals):
    ij = np.sort(ij, axis=1)
    order = np.lexsort((ij[:, 1], ij[:, 0]))
    return ij[order], vals[order]


def test_pairs_descriptors_and_forward(torch_cuda):
    torch = torch_cuda
    pos, box = _system()
    params = _params(1)
    mlp, stats, pairs, disp = _setup(torch, pos, box, params)
    _say(f"[surrogate forward] n={len(pos)} pairs={len(pairs)}")
    out = mlp.pairs(torch.from_numpy(pos).cuda(), box)
    torch.cuda.synchronize()
    assert out["n_pairs"] == len(pairs)
    ij, st = _canon(out["pair_ij"].cpu().numpy(), out["st"].cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(ij, pairs)
    draw = S.raw_descriptors(len(pos), pairs, disp, RC)
    D = (draw - stats[0]) * stats[1]
    Dg = out["desc"].cpu().numpy().astype(np.float64)
    derr = np.max(np.abs(Dg - D) / (1.0 + np.abs(D)))
    _say(f"  descriptor err {derr:.2e}")
    assert derr <= 2e-4
    ref = S.forward(params, D, pairs, disp, RC, bf16_ops=True)
    rs = np.sqrt(np.mean(ref["s"] ** 2))
    rt = np.sqrt(np.mean(ref["t"] ** 2))
    es = np.abs(st[:, 0] - ref["s"]) / rs
    et = np.abs(st[:, 1] - ref["t"]) / rt
    _say(f"  s err max {es.max():.2e} mean {es.mean():.2e}; t err max {et.max():.2e} mean {et.mean():.2e}")
    assert es.max() <= 2e-2 and es.mean() <= 2e-3
    assert et.max() <= 2e-2 and et.mean() <= 2e-3
    F = out["f3"].cpu().numpy().astype(np.float64)
    frms = np.sqrt(np.mean(np.sum(ref["F"] ** 2, axis=1)))
    ferr = np.max(np.linalg.norm(F - ref["F"], axis=1)) / frms
    e = out["err"].cpu().numpy().astype(np.float64)
    eerr = np.max(np.abs(e - ref["e"]) / np.maximum(np.abs(ref["e"]), 1e-3))
    _say(f"  force err {ferr:.2e}, error-estimate err {eerr:.2e}")
    assert ferr <= 2e-2
    assert eerr <= 1e-2
    # Newton 3 holds exactly up to FP32 summation
    assert np.linalg.norm(F.sum(axis=0)) <= 1e-4 * frms * np.sqrt(len(pos))
    # against the FP64 model itself (no operand rounding): rounding to
    # bfloat16 perturbs each operand by at most 2^-9 relative, and eight
    # rounded operand sets lie on the path to s and t (inputs, W1, H1, W2, H2,
    # W3, H3, W4), so to first order the outputs move by at most 8 * 2^-9 of
    # their dot products' absolute sums: the mean deviation is bounded by
    # that, relative to the RMS output, and the largest by 4 times that
    # (cancellation inside a dot product)
    bound = 8 * 2.0 ** -9
    f64 = S.forward(params, D, pairs, disp, RC, bf16_ops=False)
    for key, got in (("s", st[:, 0]), ("t", st[:, 1])):
        rr = np.sqrt(np.mean(f64[key] ** 2))
        d = np.abs(got - f64[key]) / rr
        _say(f"  {key} against FP64: max {d.max():.2e} mean {d.mean():.2e} (bounds {4 * bound:.2e} / {bound:.2e})")
        assert d.mean() <= bound and d.max() <= 4 * bound
    frms64 = np.sqrt(np.mean(np.sum(f64["F"] ** 2, axis=1)))
    dF = np.linalg.norm(F - f64["F"], axis=1) / frms64
    _say(f"  F against FP64: max {dF.max():.2e} rms {np.sqrt(np.mean(dF ** 2)):.2e}")
    assert np.sqrt(np.mean(dF ** 2)) <= bound and dF.max() <= 4 * bound


def test_fit_stats(torch_cuda):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    pos, box = _system(seed=5)
    mlp = atm3.Mlp(seed=0)
    mlp.fit_stats(torch.from_numpy(pos).cuda(), box)
    m, s = mlp.get_stats()
    pairs, disp = S.neighbour_pairs(pos, box, RC)
    m64, s64 = S.descriptor_stats(S.raw_descriptors(len(pos), pairs, disp, RC))
    _say("[fit stats]")
    np.testing.assert_allclose(m, m64, rtol=2e-4, atol=1e-30)
    # 1/sd of near-constant features is capped at 1e6 on both sides
    np.testing.assert_allclose(s, s64, rtol=2e-3)


def test_gradient_matches_reference(torch_cuda):
    torch = torch_cuda
    pos, box = _system(n=500, seed=7)
    params = _params(2)
    mlp, stats, pairs, disp = _setup(torch, pos, box, params)
    T = np.random.default_rng(11).normal(0, 0.3, (len(pos), 3)).astype(np.float32)
    _say(f"[surrogate grad] n={len(pos)} pairs={len(pairs)}")
    g, loss = mlp.grad(torch.from_numpy(pos).cuda(), box, torch.from_numpy(T).cuda(), lam=1.0)
    torch.cuda.synchronize()
    g = to_dict(g.cpu().numpy())
    draw = S.raw_descriptors(len(pos), pairs, disp, RC)
    D = (draw - stats[0]) * stats[1]
    c = S.forward(params, D, pairs, disp, RC, bf16_ops=True)
    ref_loss = S.loss(c["F"], c["e"], T.astype(np.float64))
    ref = S.backward(params, c, pairs, T.astype(np.float64), bf16_ops=True)
    _say(f"  loss {loss:.6e} ref {ref_loss:.6e}")
    assert loss == pytest.approx(ref_loss, rel=2e-3)
    for k in S.PARAM_ORDER:
        rel = np.linalg.norm(g[k] - ref[k]) / max(np.linalg.norm(ref[k]), 1e-30)
        _say(f"  {k}: rel L2 err {rel:.2e}")
        assert rel <= 3e-2, k
    # and the FP64 gradient is within the BF16 operand-rounding effect
    ref64 = S.backward(params, S.forward(params, D, pairs, disp, RC), pairs, T.astype(np.float64))
    for k in S.PARAM_ORDER:
        rel = np.linalg.norm(g[k] - ref64[k]) / max(np.linalg.norm(ref64[k]), 1e-30)
        assert rel <= 1e-1, k


def test_adam_step(torch_cuda):
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    params = _params(3)
    mlp = atm3.Mlp(seed=0)
    mlp.set_params(to_flat(params))
    rng = np.random.default_rng(4)
    state = {}
    ref = {k: v.copy() for k, v in params.items()}
    _say("[adam]")
    for step in range(3):
        gflat = rng.normal(0, 0.1, atm3.MLP_NPARAM).astype(np.float32)
        mlp.adam(torch.from_numpy(gflat).cuda(), lr=1e-3)
        S.adam_step(ref, to_dict(gflat), state, lr=1e-3)
    got = to_dict(mlp.get_params())
    for k in S.PARAM_ORDER:
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-5, atol=2e-7)


def test_fallback_below_every_estimate_is_exact(torch_cuda, orc):
    torch = torch_cuda
    pos, box = _system(n=900, seed=9, jitter=0.05)
    params = _params(5)
    mlp, stats, pairs, disp = _setup(torch, pos, box, params)
    _say(f"[fallback] n={len(pos)}")
    f, r, nf, err = mlp.forces(torch.from_numpy(pos).cuda(), box, threshold=-1.0, nu=NU, want_err=True)
    torch.cuda.synchronize()
    ref = orc.molecules(pos, box, rc=RC, nu=NU)
    assert nf == len(pos)
    assert r["n_pairs"] == ref.n_pairs
    assert r["n_triplets"] == 3 * ref.n_triplets
    fg = f.cpu().numpy().astype(np.float64)
    nref = np.linalg.norm(ref.forces, axis=1)
    frms = np.sqrt(np.mean(nref ** 2))
    ferr = np.max(np.linalg.norm(fg - ref.forces, axis=1) / np.maximum(nref, frms))
    _say(f"  force err {ferr:.2e}")
    assert ferr <= 1e-5
    assert r["e_lj"] == pytest.approx(ref.e_lj, rel=1e-6)
    assert r["w_lj"] == pytest.approx(ref.w_lj, rel=1e-6)


def test_zero_output_layer_leaves_exact_lj(torch_cuda, orc):
    torch = torch_cuda
    pos, box = _system(n=700, seed=12)
    params = _params(6)
    params["W4"][:] = 0.0
    params["b4"][:] = 0.0
    mlp, stats, _, _ = _setup(torch, pos, box, params)
    _say("[lj only]")
    f, r, nf, _ = mlp.forces(torch.from_numpy(pos).cuda(), box, threshold=float("inf"))
    torch.cuda.synchronize()
    ref = orc.molecules(pos, box, rc=RC, nu=NU, terms=1)
    assert nf == 0 and r["n_triplets"] == 0
    fg = f.cpu().numpy().astype(np.float64)
    nref = np.linalg.norm(ref.forces, axis=1)
    frms = np.sqrt(np.mean(nref ** 2))
    assert np.max(np.linalg.norm(fg - ref.forces, axis=1) / np.maximum(nref, frms)) <= 1e-5
    assert r["e_lj"] == pytest.approx(ref.e_lj, rel=1e-6)
    assert r["w_lj"] == pytest.approx(ref.w_lj, rel=1e-6)
    assert np.isnan(r["e_atm"])


def test_rotation_equivariance(torch_cuda):
    """An isolated cluster in a large box: rotating it rotates the surrogate
    force (invariant s_ij times a rotating unit vector)."""
    torch = torch_cuda
    rng = np.random.default_rng(21)
    pts = [np.zeros(3)]
    while len(pts) < 60:
        c = rng.uniform(-2.6, 2.6, 3)
        if min(np.linalg.norm(c - p) for p in pts) > 0.9:
            pts.append(c)
    box = np.array([24.0, 24.0, 24.0])
    pos = np.array(pts) + 12.0
    q, r_ = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r_))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    pos2 = (pos - 12.0) @ q.T + 12.0
    params = _params(7)
    mlp, _, _, _ = _setup(torch, pos, box, params)
    a = mlp.pairs(torch.from_numpy(pos).cuda(), box)["f3"].cpu().numpy().astype(np.float64)
    b = mlp.pairs(torch.from_numpy(pos2).cuda(), box)["f3"].cpu().numpy().astype(np.float64)
    scale = np.max(np.linalg.norm(a, axis=1))
    _say(f"[equivariance] max |F(Rx) - R F(x)| / max|F| = {np.max(np.abs(b - a @ q.T)) / scale:.2e}")
    assert np.max(np.abs(b - a @ q.T)) <= 3e-2 * scale
    assert np.linalg.norm(a.sum(axis=0)) <= 1e-4 * scale * len(pos)


def test_training_on_gpu_beats_lj_alone(torch_cuda):
    """Trained on exact ATM forces that the exact kernel generates (densities
    0.6 and 0.7), the surrogate's LJ + three-body force is closer to exact
    LJ + ATM than LJ alone is, on a configuration it was not trained on."""
    torch = torch_cuda
    import paper_2510_21230_amd as atm3
    frames = []
    for k in range(6):
        rho = 0.6 if k % 2 == 0 else 0.7
        pos, box = workloads.fcc(4000, rho, jitter=0.15, seed=workloads.SEED_BASE + 300 + k)
        p = torch.from_numpy(pos).cuda()
        f3, _ = atm3.compute_forces(p, box, nu=NU, terms=atm3.TERM_ATM)
        frames.append((p, box, f3))
    mlp = atm3.Mlp(seed=2)
    mlp.fit_stats(frames[0][0], frames[0][1])
    losses = []
    for it in range(240):
        p, box, f3 = frames[it % len(frames)]
        losses.append(mlp.train_step(p, box, f3, lam=1.0, lr=2e-3))
    pos, box = workloads.fcc(4000, 0.65, jitter=0.12, seed=workloads.SEED_BASE + 399)
    p = torch.from_numpy(pos).cuda()
    f_ex, _ = atm3.compute_forces(p, box, nu=NU)
    f_lj, _ = atm3.compute_forces(p, box, nu=NU, terms=atm3.TERM_LJ)
    f_sur, _, nf, _ = mlp.forces(p, box, threshold=float("inf"), nu=NU)
    torch.cuda.synchronize()
    rms = lambda a: float(torch.sqrt(torch.mean(torch.sum((a - f_ex) ** 2, dim=1))))
    e_lj, e_sur = rms(f_lj), rms(f_sur)
    _say(f"[training] loss {losses[0]:.3e} -> {np.mean(losses[-12:]):.3e}; force RMS error vs exact: "
         f"LJ only {e_lj:.4f}, LJ + surrogate {e_sur:.4f} (gain {e_lj / e_sur:.2f}x)")
    assert np.mean(losses[-12:]) < 0.5 * losses[0]
    assert e_sur < 0.7 * e_lj
