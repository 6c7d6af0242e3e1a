"""Seeded input generators: shapes, densities and determinism (CPU)."""
import numpy as np

from paper_2510_21230_amd import workloads


def test_sc_start_of_the_single_phase_runs():
    for n, rho in [(1270, 0.65), (1596, 0.817)]:
        pos, box = workloads.sc(n, 12.5)
        assert pos.shape == (n, 3) and np.all(box == 12.5)
        assert abs(n / 12.5 ** 3 - rho) < 5e-4
        assert np.all((pos > 0) & (pos < 12.5))
        k = int(np.ceil(n ** (1 / 3)))
        a = 12.5 / k
        # every coordinate sits on the lattice, every site at most once
        idx = np.rint(pos / a - 0.5).astype(int)
        assert np.allclose(pos, (idx + 0.5) * a)
        assert len({tuple(r) for r in idx}) == n
        d = pos[:, None, :] - pos[None, :, :]
        d -= 12.5 * np.rint(d / 12.5)
        r2 = (d ** 2).sum(-1) + np.eye(n) * 1e9
        assert abs(np.sqrt(r2.min()) - a) < 1e-12
        assert np.array_equal(pos, workloads.sc(n, 12.5)[0])


def test_maxwell_has_zero_momentum_and_exact_temperature():
    v = workloads.maxwell(1000, 0.746)
    assert np.abs(v.sum(axis=0)).max() < 1e-12
    assert abs((v * v).sum() / (3 * 1000 - 3) - 0.746) < 1e-12


def test_lattice_start_of_the_slab_runs():
    box = np.array([12.5, 12.5, 25.0])
    pos, b = workloads.lattice(3800, box)
    assert pos.shape == (3800, 3) and np.all(b == box)
    assert np.all((pos > 0) & (pos < box))
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.rint(d / box)
    r2 = (d ** 2).sum(-1) + np.eye(len(pos)) * 1e9
    assert np.sqrt(r2.min()) > 0.95  # spacings 12.5/13 and 25/26
    assert len({tuple(np.round(r, 9)) for r in pos}) == 3800
    assert np.array_equal(pos, workloads.lattice(3800, box)[0])


def test_fcc_box_start_of_the_slab_runs():
    box = np.array([12.5, 12.5, 25.0])
    pos, b = workloads.fcc_box(3800, box)
    assert pos.shape == (3800, 3) and np.all(b == box)
    assert np.all((pos > 0) & (pos < box))
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.rint(d / box)
    r2 = (d ** 2).sum(-1) + np.eye(len(pos)) * 1e9
    # 8 x 8 x 16 cells of edge 1.5625: nearest neighbours at a / sqrt(2)
    assert abs(np.sqrt(r2.min()) - 1.5625 / np.sqrt(2)) < 1e-12
    assert np.array_equal(pos, workloads.fcc_box(3800, box)[0])
