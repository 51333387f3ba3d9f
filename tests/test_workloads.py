"""Seeded synthetic inputs: determinism, charges, geometry, density."""
import math

import numpy as np
import pytest

import workloads


def test_seeded_and_deterministic():
    a = workloads.config("C1")
    b = workloads.config("C1")
    assert a.pos.tobytes() == b.pos.tobytes() and a.q.tobytes() == b.q.tobytes()
    c = workloads.water_box(216, 18.6, [[9.3] * 3], [1.0], seed=2)[0]
    assert not np.array_equal(a.pos, c)


@pytest.mark.parametrize("name,n,z", [("C1", 649, 1.0), ("C2", 30001, 2.0), ("PA", 3241, 2.0)])
def test_sizes_and_net_charge(name, n, z):
    w = workloads.config(name)
    assert w.n == n
    assert w.q.sum() == pytest.approx(z, abs=1e-9)
    assert w.mask.sum() == 1 and w.mask[-1] == 1 and w.q[-1] == z
    assert (w.pos >= 0).all() and (w.pos < w.box).all()


def test_water_geometry():
    w = workloads.config("C1")
    pos = w.pos[:-1].reshape(-1, 3, 3)
    box = w.box
    d1 = pos[:, 1] - pos[:, 0]
    d2 = pos[:, 2] - pos[:, 0]
    d1 -= box * np.round(d1 / box)
    d2 -= box * np.round(d2 / box)
    r1, r2 = np.linalg.norm(d1, axis=1), np.linalg.norm(d2, axis=1)
    np.testing.assert_allclose(r1, 1.0, atol=1e-12)
    np.testing.assert_allclose(r2, 1.0, atol=1e-12)
    ang = np.degrees(np.arccos((d1 * d2).sum(1) / (r1 * r2)))
    np.testing.assert_allclose(ang, 109.47, atol=1e-9)
    np.testing.assert_allclose(w.q[:-1].reshape(-1, 3), np.tile([-0.8476, 0.4238, 0.4238], (216, 1)))


def test_density_and_batch():
    assert workloads.box_for(333333) == pytest.approx(215.30, abs=0.01)
    ws = workloads.batch_windows(n_boxes=4, lo=600, hi=900)
    assert len(ws) == 4
    for k, w in enumerate(ws):
        assert w.n == 3 * w.meta["n_waters"] + 1
        assert w.box ** 3 * workloads.WATER_DENSITY == pytest.approx(w.meta["n_waters"], rel=1e-12)
        assert w.q[-1] == pytest.approx(w.meta["lam"] * w.meta["z"])


def test_sample_indices():
    s = workloads.sample_indices(1000, 50, 3)
    assert len(np.unique(s)) == 50 and s.max() < 1000
    np.testing.assert_array_equal(s, workloads.sample_indices(1000, 50, 3))
